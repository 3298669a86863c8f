// The PW advection stencil at one grid point, shared by every kernel variant.
//
// Paper Sec. II-A, Listing 1 gives su; sv is its x<->y mirror and sw applies
// the same staggered-grid flux rule to w (u on x faces, v on y faces, w on z
// faces; each flux = neighbour value x sum of the two advecting velocities
// straddling the face).  Per field: 21 floating-point operations, 17 for su
// and sv at the column top where the upper vertical flux is dropped (Sec. III).
//
// `A` reads an input at a compile-time offset (dk, dj, di) from the point:
//   A.template u<dk, dj, di>(), A.template v<...>(), A.template w<...>().
// Offsets with dk = +1 are only requested when k < nz, dk = -1 only when
// k >= 2, so no level outside 1..nz is ever read.
#pragma once

#include "pw_types.hpp"

namespace pw {

// lower-minus-upper vertical flux added to the running sum s:
// FP64 keeps Listing 1's textual order (s + c1*a*b) - c2*c*d;
// FP32 evaluates the flux difference in compensated form.
__device__ __forceinline__ double add_vertical(double s, double c1, double a, double b,
                                               double c2, double c, double d) {
    return (s + c1 * a * b) - c2 * c * d;
}
__device__ __forceinline__ float add_vertical(float s, float c1, float a, float b,
                                              float c2, float c, float d) {
    return s + pdiff(c1 * a, b, c2 * c, d);
}

template <typename CT>
struct LevelCoefs {
    CT c1, c2, d1, d2;   // tzc1(k), tzc2(k), tzd1(k), tzd2(k)
};

template <typename CT, typename Acc>
__device__ __forceinline__ void pw_point(const Acc& A, int k, int nz, CT tcx, CT tcy,
                                         const LevelCoefs<CT>& z, CT& su, CT& sv, CT& sw) {
    if (k < 2) {
        su = CT(0);
        sv = CT(0);
        sw = CT(0);
        return;
    }
    const CT u0 = A.template u<0, 0, 0>();
    const CT v0 = A.template v<0, 0, 0>();
    const CT w0 = A.template w<0, 0, 0>();
    const CT u_xm = A.template u<0, 0, -1>();
    const CT u_xp = A.template u<0, 0, 1>();
    const CT u_ym = A.template u<0, -1, 0>();
    const CT u_yp = A.template u<0, 1, 0>();
    const CT v_xm = A.template v<0, 0, -1>();
    const CT v_xp = A.template v<0, 0, 1>();
    const CT v_ym = A.template v<0, -1, 0>();
    const CT v_yp = A.template v<0, 1, 0>();
    const CT w_zm = A.template w<-1, 0, 0>();
    const CT u_zm = A.template u<-1, 0, 0>();
    const CT v_zm = A.template v<-1, 0, 0>();

    // su: Listing 1
    CT s = tcx * pdiff(u_xm, u0 + u_xm, u_xp, u0 + u_xp);
    s = s + tcy * pdiff(u_ym, v_ym + A.template v<0, -1, 1>(), u_yp, v0 + v_xp);
    // sv: mirror, own-direction (y) term first
    CT t = tcy * pdiff(v_ym, v0 + v_ym, v_yp, v0 + v_yp);
    t = t + tcx * pdiff(v_xm, u_xm + A.template u<0, 1, -1>(), v_xp, u0 + u_yp);

    const CT wz_u_lo = w_zm + A.template w<-1, 0, 1>();    // w at the lower z face of u
    const CT wz_v_lo = w_zm + A.template w<-1, 1, 0>();    // ... of v
    if (k < nz) {
        const CT w_xp = A.template w<0, 0, 1>();
        const CT w_yp = A.template w<0, 1, 0>();
        s = add_vertical(s, z.c1, u_zm, wz_u_lo, z.c2, A.template u<1, 0, 0>(), w0 + w_xp);
        t = add_vertical(t, z.c1, v_zm, wz_v_lo, z.c2, A.template v<1, 0, 0>(), w0 + w_yp);
        // sw
        const CT u_zp = A.template u<1, 0, 0>();
        const CT v_zp = A.template v<1, 0, 0>();
        const CT w_zp = A.template w<1, 0, 0>();
        CT r = tcx * pdiff(A.template w<0, 0, -1>(), u_xm + A.template u<1, 0, -1>(), w_xp, u0 + u_zp);
        r = r + tcy * pdiff(A.template w<0, -1, 0>(), v_ym + A.template v<1, -1, 0>(), w_yp, v0 + v_zp);
        r = add_vertical(r, z.d1, w_zm, w0 + w_zm, z.d2, w_zp, w0 + w_zp);
        sw = r;
    } else {
        // column top: the upper vertical flux of su and sv is dropped; sw = 0
        s = s + z.c1 * u_zm * wz_u_lo;
        t = t + z.c1 * v_zm * wz_v_lo;
        sw = CT(0);
    }
    su = s;
    sv = t;
}

}  // namespace pw
