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
// Three arithmetic policies evaluate them:
//   ArithF64    FP64, exactly as written (Listing 1's order); also for 32-bit
//               fixed-point storage.
//   ArithSplit  FP32 storage, FP32 compute: algebraically identical
//               difference-first forms -- neighbouring values are subtracted
//               first, which is exact when they are within a factor of two of
//               each other (Sterbenz), so the rounding error is relative to the
//               result instead of to the two cancelling products; the
//               coefficient-weighted vertical difference c1 a - c2 c uses
//               Kahan's fused multiply-add algorithm.
//   ArithKahan  16-bit storage, FP32 compute: the sum of two stored values
//               is exact in FP32 for int16 (at most 17 bits), and for BF16
//               (8-bit significand) or FP16 (11-bit) when the two exponents
//               differ by at most 15 or 12; each product difference E F - G H is
//               evaluated by Kahan's FMA algorithm (error <= 2 ulp of the
//               result; Jeannerod, Louvet, Muller, Math. Comp. 82 (2013)); the
//               self term uses the exact factorisation (A - C)(U + A + C).
//
// `A` reads an input at a compile-time offset (dk, dj, di) from the point:
//   A.template u<dk, dj, di>(), A.template v<...>(), A.template w<...>().
// Offsets with dk = +1 are only requested when k < nz, dk = -1 only when
// k >= 2, so no level outside 1..nz is ever read.
#pragma once

#include "pw_types.hpp"

namespace pw {

// ---------------------------------------------------------------- FP64: as written
struct ArithF64 {
    using T = double;
    static constexpr bool kCarrySums = true;   // has cross_sums (x-face sums carried along the march)
    static constexpr double kCrossScale = 1.0;   // cross_flux returns the flux difference itself
    static constexpr bool kExactZeroFlux = true;   // c2 * 0 * (w3 + w4) leaves the sum unchanged
    static __device__ __forceinline__ double self_flux(double A, double U, double C) {
        return A * (U + A) - C * (U + C);
    }
    // E F - G H on the two face sums; cross_flux forms the sums first, so a
    // caller that already holds them (carried from the previous x plane)
    // gets bit-identical results
    static __device__ __forceinline__ double cross_sums(double E, double F, double G, double H) {
        return E * F - G * H;
    }
    static __device__ __forceinline__ double cross_flux(double E, double v1, double v2, double G, double v3,
                                                        double v4) {
        return cross_sums(E, v1 + v2, G, v3 + v4);
    }
    static __device__ __forceinline__ double add_vert(double s, double c1, double a, double w1, double w2, double c2,
                                                      double c, double w3, double w4) {
        return (s + c1 * a * (w1 + w2)) - c2 * c * (w3 + w4);
    }
    static __device__ __forceinline__ double add_vself(double s, double d1, double m, double w, double d2, double p) {
        return (s + d1 * m * (w + m)) - d2 * p * (w + p);
    }
};

// ---------------------------------------------------------------- FP32: difference first
struct ArithSplit {
    using T = float;
    static constexpr bool kCarrySums = false;   // its cross form needs the four values, not two sums
    // the difference-first vertical form still rounds w3 + w4 when c = 0
    static constexpr bool kExactZeroFlux = false;
    // A (U + A) - C (U + C) = (A - C) (U + A + C)
    static __device__ __forceinline__ float self_flux(float A, float U, float C) { return (A - C) * ((U + A) + C); }
    // 2 (E F - G H) = (E - G)(F + H) + (E + G)(F - H), with F - H = (v1 - v3) + (v2 - v4);
    // the factor 1/2 goes into the term's coefficient (kCrossScale), exactly
    static constexpr float kCrossScale = 0.5f;
    static __device__ __forceinline__ float cross_flux(float E, float v1, float v2, float G, float v3, float v4) {
        const float fph = (v1 + v2) + (v3 + v4);
        const float fmh = (v1 - v3) + (v2 - v4);
        return __builtin_fmaf(E - G, fph, (E + G) * fmh);
    }
    // c1 a (w1 + w2) - c2 c (w3 + w4) with e - g = c1 a - c2 c by Kahan's algorithm
    static __device__ __forceinline__ float add_vert(float s, float c1, float a, float w1, float w2, float c2, float c,
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
    static __device__ __forceinline__ float add_vself(float s, float d1, float m, float w, float d2, float p) {
        const float g = d2 * p;
        const float eg = __builtin_fmaf(d2, p, -g);
        const float emg = __builtin_fmaf(d1, m, -g) - eg;
        const float epg = __builtin_fmaf(d1, m, g);
        return s + 0.5f * __builtin_fmaf(emg, (w + m) + (w + p), epg * (m - p));
    }
};

// ---------------------------------------------------------------- FP32: Kahan product differences
struct ArithKahan {
    using T = float;
    static constexpr bool kCarrySums = true;
    static constexpr float kCrossScale = 1.0f;
    static constexpr bool kExactZeroFlux = true;   // a b - 0 d = RN(a b) exactly
    // a b - c d: w = RN(c d); e = c d - w exactly; RN(RN(a b - w) - e)
    static __device__ __forceinline__ float pdiff(float a, float b, float c, float d) {
        const float w = c * d;
        const float e = __builtin_fmaf(c, d, -w);
        return __builtin_fmaf(a, b, -w) - e;
    }
    static __device__ __forceinline__ float self_flux(float A, float U, float C) { return (A - C) * ((U + A) + C); }
    static __device__ __forceinline__ float cross_sums(float E, float F, float G, float H) { return pdiff(E, F, G, H); }
    static __device__ __forceinline__ float cross_flux(float E, float v1, float v2, float G, float v3, float v4) {
        return cross_sums(E, v1 + v2, G, v3 + v4);
    }
    static __device__ __forceinline__ float add_vert(float s, float c1, float a, float w1, float w2, float c2, float c,
                                                     float w3, float w4) {
        return s + pdiff(c1 * a, w1 + w2, c2 * c, w3 + w4);
    }
    static __device__ __forceinline__ float add_vself(float s, float d1, float m, float w, float d2, float p) {
        return s + pdiff(d1 * m, w + m, d2 * p, w + p);
    }
};

// Policy of each storage type.
template <typename ST> struct arith_of { using type = ArithKahan; };
template <> struct arith_of<double> { using type = ArithF64; };
template <> struct arith_of<float> { using type = ArithSplit; };
template <> struct arith_of<fx32_t> { using type = ArithF64; };

// Coefficients of one point.  Each output's x and y coefficients are uniform
// over the domain; the vertical pair is per level.  For scaled storage the
// per-field power-of-two scales are folded in (term coefficient x out_scale /
// (scale of its two fields)), so the arithmetic runs on stored values and
// yields stored outputs; the folding is exact.
template <typename CT>
struct PointCoefs {
    CT xu, yu, z1u, z2u;   // su: tcx, tcy, tzc1(k), tzc2(k)
    CT yv, xv, z1v, z2v;   // sv: tcy, tcx, tzc1(k), tzc2(k)
    CT xw, yw, z1w, z2w;   // sw: tcx, tcy, tzd1(k), tzd2(k)
};

// GUARDED: reads above the column top only when k < nz (global-memory
// accessors, where level nz+1 may lie outside the array).  Unguarded (LDS
// windows, where every such read stays inside the staged window): all reads
// are issued unconditionally and the column-top and k = 1 results are picked
// by selects, so the code is straight-line and two points of one thread can
// share their reads.  MAY_BOTTOM / MAY_TOP = false state that k is never 1 /
// never nz for this point (known at compile time for pairs of levels in
// even-height columns), which drops the corresponding select.
//
// xs (unguarded form, policies with kCarrySums, or NULL): the x-face sums of
// the x terms of sv and sw, carried along the x march.  The lower face of
// plane i is the upper face of plane i-1, so on entry xs[0] holds
// u(k, j, i-1) + u(k, j+1, i-1) (sv) and xs[1] holds u(k, j, i-1) +
// u(k+1, j, i-1) (sw), and on return the same sums at plane i.  The sums are
// the same operations on the same values as when formed here, so results do
// not change.  (At the column top xs[1] leaves with the top-zeroed upper
// value; only sw(nz) would read it, and that result is replaced by zero.)
template <typename AR, bool GUARDED, bool MAY_BOTTOM = true, bool MAY_TOP = true, typename Acc,
          typename CT = typename AR::T>
__device__ __forceinline__ void pw_point(const Acc& A, int k, int nz, const PointCoefs<CT>& c, CT& su, CT& sv,
                                         CT& sw, CT* xs = nullptr) {
    if constexpr (GUARDED) {
        if (k < 2) {
            su = CT(0);
            sv = CT(0);
            sw = CT(0);
            return;
        }
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
    // cross terms: coefficient x kCrossScale (loop-invariant) x cross_flux
    CT s = c.xu * AR::self_flux(u_xm, u0, u_xp);
    s = s + (c.yu * AR::kCrossScale) * AR::cross_flux(u_ym, v_ym, A.template v<0, -1, 1>(), u_yp, v0, v_xp);
    // sv: mirror of su, own-direction (y) term first
    CT t = c.yv * AR::self_flux(v_ym, v0, v_yp);
    if constexpr (!GUARDED && AR::kCarrySums) {
        if (xs != nullptr) {
            const CT h = u0 + u_yp;   // upper x face of v, u(k, j, i) + u(k, j+1, i)
            t = t + (c.xv * AR::kCrossScale) * AR::cross_sums(v_xm, xs[0], v_xp, h);
            xs[0] = h;
        } else {
            t = t + (c.xv * AR::kCrossScale) * AR::cross_flux(v_xm, u_xm, A.template u<0, 1, -1>(), v_xp, u0, u_yp);
        }
    } else {
        t = t + (c.xv * AR::kCrossScale) * AR::cross_flux(v_xm, u_xm, A.template u<0, 1, -1>(), v_xp, u0, u_yp);
    }

    const CT w_u_lo = A.template w<-1, 0, 1>();   // w(k-1, j, i+1): lower z face of u
    const CT w_v_lo = A.template w<-1, 1, 0>();   // w(k-1, j+1, i): lower z face of v
    const CT w_xp = A.template w<0, 0, 1>();
    const CT w_yp = A.template w<0, 1, 0>();
    // The three outputs given the three values above the point.
    auto eval = [&](CT u_zp, CT v_zp, CT w_zp, CT& a, CT& b, CT& r) {
        a = AR::add_vert(s, c.z1u, u_zm, w_zm, w_u_lo, c.z2u, u_zp, w0, w_xp);
        b = AR::add_vert(t, c.z1v, v_zm, w_zm, w_v_lo, c.z2v, v_zp, w0, w_yp);
        // sw: x and y terms with u, v summed over levels k, k+1; then w along z
        CT q;
        if constexpr (!GUARDED && AR::kCarrySums) {
            if (xs != nullptr) {
                const CT h = u0 + u_zp;   // upper x face of w, u(k, j, i) + u(k+1, j, i)
                q = (c.xw * AR::kCrossScale) * AR::cross_sums(A.template w<0, 0, -1>(), xs[1], w_xp, h);
                xs[1] = h;
            } else {
                q = (c.xw * AR::kCrossScale) *
                    AR::cross_flux(A.template w<0, 0, -1>(), u_xm, A.template u<1, 0, -1>(), w_xp, u0, u_zp);
            }
        } else {
            q = (c.xw * AR::kCrossScale) *
                AR::cross_flux(A.template w<0, 0, -1>(), u_xm, A.template u<1, 0, -1>(), w_xp, u0, u_zp);
        }
        q = q + (c.yw * AR::kCrossScale) *
                    AR::cross_flux(A.template w<0, -1, 0>(), v_ym, A.template v<1, -1, 0>(), w_yp, v0, v_zp);
        r = AR::add_vself(q, c.z1w, w_zm, w0, c.z2w, w_zp);
    };
    // column top: su and sv without their upper vertical flux (Sec. III)
    auto top = [&](CT& a, CT& b) {
        a = s + c.z1u * u_zm * (w_zm + w_u_lo);
        b = t + c.z1v * v_zm * (w_zm + w_v_lo);
    };
    if constexpr (GUARDED) {
        if (k < nz) {
            eval(A.template u<1, 0, 0>(), A.template v<1, 0, 0>(), A.template w<1, 0, 0>(), su, sv, sw);
        } else {
            top(su, sv);
            sw = CT(0);
        }
    } else {
        // every read is inside the staged window (level nz + 1 of a column is
        // level 1 of the next one)
        CT u_zp = A.template u<1, 0, 0>();
        CT v_zp = A.template v<1, 0, 0>();
        const CT w_zp = A.template w<1, 0, 0>();
        const bool in = k < nz;
        // FP32 compute (the VALU-bound 16-bit kernels): zero values above the
        // top make the upper vertical fluxes exact zeros, the column-top form
        // at no extra cost for finite inputs.  FP64 compute (HBM-bound) takes
        // the column-top form by a select instead, which costs it nothing
        // measurable and keeps the top results independent of the values
        // above the top, finite or not.
        constexpr bool kZeroTop = MAY_TOP && AR::kExactZeroFlux && sizeof(CT) == 4;
        if constexpr (kZeroTop) {
            u_zp = in ? u_zp : CT(0);
            v_zp = in ? v_zp : CT(0);
        }
        CT fa, fb, fr;
        eval(u_zp, v_zp, w_zp, fa, fb, fr);
        if constexpr (MAY_TOP) {
            if constexpr (!kZeroTop) {
                CT ta, tb;
                top(ta, tb);
                fa = in ? fa : ta;
                fb = in ? fb : tb;
            }
            fr = in ? fr : CT(0);
        }
        if constexpr (MAY_BOTTOM) {
            const bool live = k >= 2;
            fa = live ? fa : CT(0);
            fb = live ? fb : CT(0);
            fr = live ? fr : CT(0);
        }
        su = fa;
        sv = fb;
        sw = fr;
    }
}

}  // namespace pw
