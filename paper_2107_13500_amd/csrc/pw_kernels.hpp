// PW advection kernels for gfx950.
//
// direct  one thread per grid point; every operand is a global load, neighbour
//         reuse is left to L1/L2.  Handles any strides; the correctness anchor.
// march   the HBM-streaming kernel.  With packed columns (sy = nz) each x plane
//         is one contiguous run of (ny + 2) * nz elements, so a workgroup owns a
//         contiguous chunk of P points of that (j, k) run and walks along x.  It
//         keeps the three planes i-1, i, i+1 of u, v, w in a ring of LDS slots
//         (the GPU form of the paper's three-slice shift buffer, Sec. III): each
//         step loads one new plane window [p0 - nz, p0 + P + nz) -- the chunk
//         plus one column of y halo on each side -- into registers while the
//         current plane is computed, so every input element crosses HBM about
//         once and the loads of plane i+2 overlap the arithmetic of plane i.
#pragma once

#include <type_traits>

#include "pw_stencil.hpp"

namespace pw {

constexpr int kMarchMaxNz = 256;   // largest column the march variant accepts
constexpr int kNumXcd = 8;         // MI355X: 8 accelerator complex dies, one L2 each

// Everything a kernel needs about one domain (passed by value).
struct DomainArgs {
    const void* u;
    const void* v;
    const void* w;
    void* su;
    void* sv;
    void* sw;
    const double* tzc1;
    const double* tzc2;
    const double* tzd1;
    const double* tzd2;
    double tcx, tcy;
    float in_inv[3];     // 1 / in_scale (16-bit storage only)
    float out_scale[3];  // out_scale (16-bit storage only)
    int32_t nx, ny, nz;
    int32_t pad_;
    int64_t sy, sx;
};

// Geometry of a march launch over one domain.
struct MarchGeom {
    int32_t nchunks;   // chunks of P points over the interior (j, k) run
    int32_t nseg;      // x segments
    int32_t seg;       // planes per segment
    int32_t wpad;      // LDS elements per field per slot
};

template <typename ST> struct is16 { static constexpr bool value = false; };
template <> struct is16<bf16_t> { static constexpr bool value = true; };
template <> struct is16<f16_t> { static constexpr bool value = true; };

template <typename ST>
__device__ __forceinline__ typename compute_of<ST>::type load_in(const ST* p, float inv) {
    auto x = to_compute(*p);
    if constexpr (is16<ST>::value) x *= inv;
    return x;
}

template <typename ST>
__device__ __forceinline__ void store_out(ST* p, typename compute_of<ST>::type x, float scale) {
    if constexpr (is16<ST>::value) x *= scale;
    ST y = from_compute<ST>(x);
    if constexpr (sizeof(ST) == 2) {
        uint16_t bits;
        __builtin_memcpy(&bits, &y, 2);
        __builtin_nontemporal_store(bits, reinterpret_cast<uint16_t*>(p));
    } else {
        __builtin_nontemporal_store(y, p);
    }
}

template <typename ST>
__device__ __forceinline__ LevelCoefs<typename compute_of<ST>::type> level_coefs(const DomainArgs& d, int k) {
    using CT = typename compute_of<ST>::type;
    LevelCoefs<CT> z;
    if (k >= 2) {
        z.c1 = static_cast<CT>(d.tzc1[k - 1]);
        z.c2 = static_cast<CT>(d.tzc2[k - 1]);
        z.d1 = k < d.nz ? static_cast<CT>(d.tzd1[k - 1]) : CT(0);
        z.d2 = k < d.nz ? static_cast<CT>(d.tzd2[k - 1]) : CT(0);
    } else {
        z.c1 = z.c2 = z.d1 = z.d2 = CT(0);
    }
    return z;
}

// ---------------------------------------------------------------------------
// direct variant
// ---------------------------------------------------------------------------
// Accessor wrapper with the u<>/v<>/w<> names the stencil expects.
template <typename ST>
struct GAcc {
    using CT = typename compute_of<ST>::type;
    const ST* pu;
    const ST* pv;
    const ST* pw;
    int64_t sy, sx;
    float iu, iv, iw;
    template <int dk, int dj, int di>
    __device__ __forceinline__ CT u() const { return load_in(pu + (dk + dj * sy + di * sx), iu); }
    template <int dk, int dj, int di>
    __device__ __forceinline__ CT v() const { return load_in(pv + (dk + dj * sy + di * sx), iv); }
    template <int dk, int dj, int di>
    __device__ __forceinline__ CT w() const { return load_in(pw + (dk + dj * sy + di * sx), iw); }
};

// grid: x over the ny*nz points of a plane in blocks of NT, y over x planes.
template <typename ST, int NT>
__global__ __launch_bounds__(NT) void pw_direct_kernel(DomainArgs d) {
    using CT = typename compute_of<ST>::type;
    const int g = blockIdx.x * NT + threadIdx.x;
    if (g >= d.ny * d.nz) return;
    const int k = g % d.nz + 1;
    const int j = g / d.nz + 1;
    const int i = blockIdx.y + 1;
    const int64_t off = (int64_t)(k - 1) + (int64_t)j * d.sy + (int64_t)i * d.sx;
    GAcc<ST> A{static_cast<const ST*>(d.u) + off, static_cast<const ST*>(d.v) + off,
               static_cast<const ST*>(d.w) + off, d.sy, d.sx, d.in_inv[0], d.in_inv[1], d.in_inv[2]};
    const LevelCoefs<CT> z = level_coefs<ST>(d, k);
    CT su, sv, sw;
    pw_point<CT>(A, k, d.nz, static_cast<CT>(d.tcx), static_cast<CT>(d.tcy), z, su, sv, sw);
    store_out(static_cast<ST*>(d.su) + off, su, d.out_scale[0]);
    store_out(static_cast<ST*>(d.sv) + off, sv, d.out_scale[1]);
    store_out(static_cast<ST*>(d.sw) + off, sw, d.out_scale[2]);
}

// ---------------------------------------------------------------------------
// march variant
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the XCDs.  Renumber them so that
// each XCD receives a contiguous range of tiles: neighbouring chunks, which
// share their y-halo columns, then run at the same time behind the same L2.
__device__ __forceinline__ int xcd_tile(int b, int G) {
    const int q = G / kNumXcd;
    const int r = G % kNumXcd;
    const int x = b % kNumXcd;
    const int slot = b / kNumXcd;
    return x * q + (x < r ? x : r) + slot;
}

template <typename CT>
struct LdsAcc {
    const CT* m;   // slot of plane i-1, at the point's window index
    const CT* c;   // plane i
    const CT* p;   // plane i+1
    int nz, wp;
    template <int di> __device__ __forceinline__ const CT* sel() const {
        return di < 0 ? m : (di > 0 ? p : c);
    }
    template <int dk, int dj, int di>
    __device__ __forceinline__ CT u() const { return sel<di>()[dk + dj * nz]; }
    template <int dk, int dj, int di>
    __device__ __forceinline__ CT v() const { return sel<di>()[wp + dk + dj * nz]; }
    template <int dk, int dj, int di>
    __device__ __forceinline__ CT w() const { return sel<di>()[2 * wp + dk + dj * nz]; }
};

template <typename ST, int NT, int P, bool VEC>
struct March {
    using CT = typename compute_of<ST>::type;
    static constexpr int VW = VEC ? int(16 / sizeof(ST)) : 1;           // elements per load
    static constexpr int WMAX = P + 2 * kMarchMaxNz;                      // largest window
    static constexpr int NVL = (WMAX + NT * VW - 1) / (NT * VW);         // loads per field per thread
    static constexpr int PPT = P / NT;                                    // points per thread
    using Raw = typename std::conditional<VEC, uint4, ST>::type;
    static_assert(P % NT == 0, "P must be a multiple of the block size");

    struct Stage {
        Raw r[3][NVL];
    };

    // Issue the global loads of window [wb, wb + wlen) of plane ip.
    static __device__ __forceinline__ void load(Stage& st, const DomainArgs& d, int64_t ip, int wb, int wlen) {
        const ST* f[3] = {static_cast<const ST*>(d.u), static_cast<const ST*>(d.v), static_cast<const ST*>(d.w)};
#pragma unroll
        for (int fi = 0; fi < 3; ++fi) {
            const ST* base = f[fi] + ip * d.sx + wb;
#pragma unroll
            for (int r = 0; r < NVL; ++r) {
                const int q = (r * NT + (int)threadIdx.x) * VW;
                if (q < wlen) st.r[fi][r] = *reinterpret_cast<const Raw*>(base + q);
            }
        }
    }

    // Convert staged values to the compute type and write them to an LDS slot.
    static __device__ __forceinline__ void put(const Stage& st, CT* slot, int wpad, int wlen, const DomainArgs& d) {
#pragma unroll
        for (int fi = 0; fi < 3; ++fi) {
#pragma unroll
            for (int r = 0; r < NVL; ++r) {
                const int q = (r * NT + (int)threadIdx.x) * VW;
                if (q < wlen) {
                    union {
                        Raw raw;
                        ST e[VW];
                    } cv;
                    cv.raw = st.r[fi][r];
                    CT out[VW];
#pragma unroll
                    for (int n = 0; n < VW; ++n) {
                        out[n] = to_compute(cv.e[n]);
                        if constexpr (is16<ST>::value) out[n] *= d.in_inv[fi];
                    }
                    CT* dst = slot + fi * wpad + q;
                    if constexpr (VW * sizeof(CT) >= 16) {
#pragma unroll
                        for (int n = 0; n < VW; n += 16 / (int)sizeof(CT)) {
                            *reinterpret_cast<uint4*>(dst + n) = *reinterpret_cast<const uint4*>(out + n);
                        }
                    } else {
#pragma unroll
                        for (int n = 0; n < VW; ++n) dst[n] = out[n];
                    }
                }
            }
        }
    }
};

// One (chunk, segment) tile of the march: chunk c of the interior (j, k) run,
// planes i_begin .. i_end.  Every thread of the workgroup must call this (it
// holds barriers); `lds` must hold 9 * wpad compute-type elements.
template <typename ST, int NT, int P, bool VEC>
__device__ __forceinline__ void march_tile(const DomainArgs& d, int c, int i_begin, int i_end, int wpad,
                                           typename compute_of<ST>::type* lds) {
    using M = March<ST, NT, P, VEC>;
    using CT = typename M::CT;

    const int nz = d.nz;
    const int p0 = nz + c * P;                        // first point of the chunk (j >= 1)
    const int pend = min(p0 + P, (d.ny + 1) * nz);    // one past the last interior point
    const int wb = p0 - nz;                           // window start: one column of y halo
    const int wlen = min(P + 2 * nz, (d.ny + 2) * nz - wb);
    const int slot_elems = 3 * wpad;

    // per-point constants: level, coefficients, window index
    int kk[M::PPT];
    int li[M::PPT];
    bool live[M::PPT];
    LevelCoefs<CT> zc[M::PPT];
#pragma unroll
    for (int r = 0; r < M::PPT; ++r) {
        const int p = p0 + r * NT + (int)threadIdx.x;
        live[r] = p < pend;
        kk[r] = p % nz + 1;
        li[r] = p - wb;
        zc[r] = level_coefs<ST>(d, live[r] ? kk[r] : 1);
    }
    const CT tcx = static_cast<CT>(d.tcx);
    const CT tcy = static_cast<CT>(d.tcy);

    typename M::Stage st;
    // prologue: planes i_begin-1 and i_begin straight into their slots, then
    // plane i_begin+1 into registers
    int sm = 0, sc = 1, sp = 2;                       // slots of planes i-1, i, i+1
    M::load(st, d, (int64_t)(i_begin - 1), wb, wlen);
    M::put(st, lds + sm * slot_elems, wpad, wlen, d);
    M::load(st, d, (int64_t)i_begin, wb, wlen);
    M::put(st, lds + sc * slot_elems, wpad, wlen, d);
    M::load(st, d, (int64_t)(i_begin + 1), wb, wlen);

    for (int i = i_begin; i <= i_end; ++i) {
        M::put(st, lds + sp * slot_elems, wpad, wlen, d);
        __syncthreads();
        if (i + 2 <= i_end + 1) M::load(st, d, (int64_t)(i + 2), wb, wlen);

        const int64_t obase = (int64_t)i * d.sx;
#pragma unroll
        for (int r = 0; r < M::PPT; ++r) {
            if (!live[r]) continue;
            const int l = li[r];
            LdsAcc<CT> A{lds + sm * slot_elems + l, lds + sc * slot_elems + l, lds + sp * slot_elems + l, nz, wpad};
            CT su, sv, sw;
            pw_point<CT>(A, kk[r], nz, tcx, tcy, zc[r], su, sv, sw);
            const int64_t o = obase + (wb + l);
            store_out(static_cast<ST*>(d.su) + o, su, d.out_scale[0]);
            store_out(static_cast<ST*>(d.sv) + o, sv, d.out_scale[1]);
            store_out(static_cast<ST*>(d.sw) + o, sw, d.out_scale[2]);
        }
        __syncthreads();
        const int t = sm;
        sm = sc;
        sc = sp;
        sp = t;
    }
}

// Single domain: one workgroup per (chunk, segment) tile.
template <typename ST, int NT, int P, bool VEC>
__global__ __launch_bounds__(NT) void pw_march_kernel(DomainArgs d, MarchGeom g) {
    using CT = typename compute_of<ST>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    CT* lds = reinterpret_cast<CT*>(smem_raw);
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int c = tile % g.nchunks;
    const int s = tile / g.nchunks;
    const int i_begin = 1 + s * g.seg;
    const int i_end = min(i_begin + g.seg - 1, d.nx);
    march_tile<ST, NT, P, VEC>(d, c, i_begin, i_end, g.wpad, lds);
}

}  // namespace pw
