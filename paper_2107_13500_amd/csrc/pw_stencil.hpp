// The PW advection stencil at one grid point, shared by every kernel variant.
//
// Paper Sec. II-A, Listing 1 gives su; sv is its x<->y mirror and sw applies
// the same staggered-grid flux rule to w (u on x faces, v on y faces, w on z
// faces; each flux = neighbour value x sum of the two advecting velocities
// straddling the face).  Per field: 21 floating-point operations in Listing 1's
// form, 17 for su and sv at the column top where the upper vertical flux is
// dropped (Sec. III).
//
// Each directional term is a flux difference "lower - upper".  Four shapes
// occur:
//   self   A (U + A) - C (U + C)             own velocity along its own axis
//   cross  E (v1 + v2) - G (v3 + v4)         advected by another velocity
//   vert   c1 a (w1 + w2) - c2 c (w3 + w4)   vertical, per-level coefficients
//   vself  d1 m (w + m) - d2 p (w + p)       w along z
// FP64 evaluates them exactly as written (Listing 1's order).  FP32 (the
// reduced-storage forms) evaluates the algebraically identical difference-
// first forms below: neighbouring values are subtracted first, which is exact
// when they are within a factor of two of each other (Sterbenz), so the
// rounding error is relative to the result instead of to the two cancelling
// products; the coefficient-weighted vertical difference c1 a - c2 c uses
// Kahan's fused multiply-add algorithm.
//
// `A` reads an input at a compile-time offset (dk, dj, di) from the point:
//   A.template u<dk, dj, di>(), A.template v<...>(), A.template w<...>().
// Offsets with dk = +1 are only requested when k < nz, dk = -1 only when
// k >= 2, so no level outside 1..nz is ever read.
#pragma once

#include "pw_types.hpp"

namespace pw {

// ---------------------------------------------------------------- FP64: as written
__device__ __forceinline__ double self_flux(double A, double U, double C) {
    return A * (U + A) - C * (U + C);
}
__device__ __forceinline__ double cross_flux(double E, double v1, double v2, double G, double v3, double v4) {
    return E * (v1 + v2) - G * (v3 + v4);
}
__device__ __forceinline__ double add_vert(double s, double c1, double a, double w1, double w2, double c2, double c,
                                           double w3, double w4) {
    return (s + c1 * a * (w1 + w2)) - c2 * c * (w3 + w4);
}
__device__ __forceinline__ double add_vself(double s, double d1, double m, double w, double d2, double p) {
    return (s + d1 * m * (w + m)) - d2 * p * (w + p);
}

// ---------------------------------------------------------------- FP32: difference first
// A (U + A) - C (U + C) = (A - C) (U + A + C)
__device__ __forceinline__ float self_flux(float A, float U, float C) {
    return (A - C) * ((U + A) + C);
}
// E F - G H = ((E - G)(F + H) + (E + G)(F - H)) / 2, with F - H = (v1 - v3) + (v2 - v4)
__device__ __forceinline__ float cross_flux(float E, float v1, float v2, float G, float v3, float v4) {
    const float fph = (v1 + v2) + (v3 + v4);
    const float fmh = (v1 - v3) + (v2 - v4);
    return 0.5f * __builtin_fmaf(E - G, fph, (E + G) * fmh);
}
// c1 a (w1 + w2) - c2 c (w3 + w4) with e - g = c1 a - c2 c by Kahan's algorithm
__device__ __forceinline__ float add_vert(float s, float c1, float a, float w1, float w2, float c2, float c,
                                          float w3, float w4) {
    const float g = c2 * c;
    const float eg = __builtin_fmaf(c2, c, -g);            // c2 c - g, exact
    const float emg = __builtin_fmaf(c1, a, -g) - eg;      // c1 a - c2 c
    const float epg = __builtin_fmaf(c1, a, g);            // c1 a + c2 c
    const float fph = (w1 + w2) + (w3 + w4);
    const float fmh = (w1 - w3) + (w2 - w4);
    return s + 0.5f * __builtin_fmaf(emg, fph, epg * fmh);
}
// d1 m (w + m) - d2 p (w + p): F - H = m - p, F + H = (w + m) + (w + p)
__device__ __forceinline__ float add_vself(float s, float d1, float m, float w, float d2, float p) {
    const float g = d2 * p;
    const float eg = __builtin_fmaf(d2, p, -g);
    const float emg = __builtin_fmaf(d1, m, -g) - eg;
    const float epg = __builtin_fmaf(d1, m, g);
    return s + 0.5f * __builtin_fmaf(emg, (w + m) + (w + p), epg * (m - p));
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

    // su: Listing 1 -- x term, y term, then the vertical term
    CT s = tcx * self_flux(u_xm, u0, u_xp);
    s = s + tcy * cross_flux(u_ym, v_ym, A.template v<0, -1, 1>(), u_yp, v0, v_xp);
    // sv: mirror of su, own-direction (y) term first
    CT t = tcy * self_flux(v_ym, v0, v_yp);
    t = t + tcx * cross_flux(v_xm, u_xm, A.template u<0, 1, -1>(), v_xp, u0, u_yp);

    const CT w_u_lo = A.template w<-1, 0, 1>();   // w(k-1, j, i+1): lower z face of u
    const CT w_v_lo = A.template w<-1, 1, 0>();   // w(k-1, j+1, i): lower z face of v
    if (k < nz) {
        const CT w_xp = A.template w<0, 0, 1>();
        const CT w_yp = A.template w<0, 1, 0>();
        const CT u_zp = A.template u<1, 0, 0>();
        const CT v_zp = A.template v<1, 0, 0>();
        const CT w_zp = A.template w<1, 0, 0>();
        s = add_vert(s, z.c1, u_zm, w_zm, w_u_lo, z.c2, u_zp, w0, w_xp);
        t = add_vert(t, z.c1, v_zm, w_zm, w_v_lo, z.c2, v_zp, w0, w_yp);
        // sw: x and y terms with u, v summed over levels k, k+1; then w along z
        CT r = tcx * cross_flux(A.template w<0, 0, -1>(), u_xm, A.template u<1, 0, -1>(), w_xp, u0, u_zp);
        r = r + tcy * cross_flux(A.template w<0, -1, 0>(), v_ym, A.template v<1, -1, 0>(), w_yp, v0, v_zp);
        sw = add_vself(r, z.d1, w_zm, w0, z.d2, w_zp);
    } else {
        // column top: the upper vertical flux of su and sv is dropped; sw = 0
        s = s + z.c1 * u_zm * (w_zm + w_u_lo);
        t = t + z.c1 * v_zm * (w_zm + w_v_lo);
        sw = CT(0);
    }
    su = s;
    sv = t;
}

}  // namespace pw
