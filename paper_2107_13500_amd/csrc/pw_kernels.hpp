// PW advection kernels for gfx950.
//
// direct  one thread per grid point; every operand is a global load, neighbour
//         reuse is left to L1/L2.  Handles any strides; the correctness anchor.
// march   the HBM-streaming kernel.  With packed columns (sy = nz) each x plane
//         is one contiguous run of (ny + 2) * nz elements, so a workgroup owns a
//         contiguous chunk of P points of that (j, k) run and walks along x.  It
//         keeps the planes i-1, i, i+1 of u, v, w in a ring of LDS slots (the
//         GPU form of the paper's three-slice shift buffer, Sec. III; a fourth
//         slot for FP32 compute saves one barrier per plane).  The window of a
//         plane is [p0 - nz, p0 + P + nz) -- the chunk plus one column of y
//         halo on each side -- so every input element crosses HBM about once.
//         Two or three later planes are in flight in registers while a plane
//         is computed.  With a compile-time column height every LDS offset is
//         an immediate, the ring rotation is unrolled so slots and register
//         sets are compile-time too, and each thread computes two consecutive
//         levels, sharing their neighbour reads and storing both results with
//         one vector store.
#pragma once

#include <type_traits>

#include "pw_stencil.hpp"

namespace pw {

constexpr int kMarchMaxNz = 256;   // largest column the march variant accepts
constexpr int kLdsPerCu = 160 * 1024;           // gfx950 LDS per CU (and per workgroup)
constexpr int kMaxDynamicLds = kLdsPerCu - 1024;   // leaves room for a kernel's small static LDS
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
    // Per output (su, sv, sw): x and y coefficients and the factor applied to
    // the per-level vertical coefficients, with the storage scales of 16-bit
    // and int32 storage folded in (all exact powers of two); plain tcx, tcy,
    // 1 otherwise.
    double cx[3], cy[3], cz[3];
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
    int32_t cpx;       // compact tile order: chunk slots per XCD and segment (0: XCD-contiguous order)
};

// Storage types that carry per-field power-of-two scales.
template <typename ST> struct scaled_type { static constexpr bool value = false; };
template <> struct scaled_type<bf16_t> { static constexpr bool value = true; };
template <> struct scaled_type<f16_t> { static constexpr bool value = true; };
template <> struct scaled_type<fx16_t> { static constexpr bool value = true; };
template <> struct scaled_type<fx32_t> { static constexpr bool value = true; };

// Folded coefficients (see DomainArgs) from tcx, tcy and the storage scales.
__host__ __device__ inline void fold_coefficients(double tcx, double tcy, const float in_scale[3],
                                                  const float out_scale[3], double cx[3], double cy[3],
                                                  double cz[3]) {
    const double su = in_scale[0], sv = in_scale[1], sw = in_scale[2];
    const double o[3] = {out_scale[0], out_scale[1], out_scale[2]};
    const double own[3] = {su, sv, sw};
    for (int f = 0; f < 3; ++f) {
        cx[f] = tcx * o[f] / (own[f] * su);
        cy[f] = tcy * o[f] / (own[f] * sv);
        cz[f] = o[f] / (own[f] * sw);
    }
}

// One load of a Raw value (2, 4, 8 or 16 bytes) through a global pointer, as
// a plain integer vector (HIP's vector structs cannot be assigned from an
// address-space-qualified lvalue), copied bit for bit.
template <typename Raw>
__device__ __forceinline__ Raw load_global(global_ptr<const char> p) {
    typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));
    typedef uint32_t u32x2v __attribute__((ext_vector_type(2)));
    Raw r;
    if constexpr (sizeof(Raw) == 16) {
        const u32x4v x = *reinterpret_cast<global_ptr<const u32x4v>>(p);
        __builtin_memcpy(&r, &x, 16);
    } else if constexpr (sizeof(Raw) == 8) {
        const u32x2v x = *reinterpret_cast<global_ptr<const u32x2v>>(p);
        __builtin_memcpy(&r, &x, 8);
    } else if constexpr (sizeof(Raw) == 4) {
        const uint32_t x = *reinterpret_cast<global_ptr<const uint32_t>>(p);
        __builtin_memcpy(&r, &x, 4);
    } else {
        static_assert(sizeof(Raw) == 2, "2, 4, 8 or 16 bytes");
        const uint16_t x = *reinterpret_cast<global_ptr<const uint16_t>>(p);
        __builtin_memcpy(&r, &x, 2);
    }
    return r;
}

template <typename ST>
__device__ __forceinline__ void store_out(global_ptr<ST> p, typename compute_of<ST>::type x) {
    ST y = from_compute<ST>(x);
    if constexpr (sizeof(ST) == 2) {
        uint16_t bits;
        __builtin_memcpy(&bits, &y, 2);
        __builtin_nontemporal_store(bits, reinterpret_cast<global_ptr<uint16_t>>(p));
    } else if constexpr (std::is_same<ST, fx32_t>::value) {
        __builtin_nontemporal_store(y.v, reinterpret_cast<global_ptr<int32_t>>(p));
    } else {
        __builtin_nontemporal_store(y, p);
    }
}

// Two consecutive outputs p[0], p[1] with one store (p aligned to 2 elements).
// BF16 and FP16 pairs are rounded by one packed conversion (v_cvt_pk_bf16_f32,
// v_cvt_pk_f16_f32: round to nearest even, as from_compute).
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
template <typename ST>
__device__ __forceinline__ void store_pair(global_ptr<ST> p, typename compute_of<ST>::type a, typename compute_of<ST>::type b) {
    if constexpr (std::is_same<ST, double>::value) {
        __builtin_nontemporal_store(f64x2{a, b}, reinterpret_cast<global_ptr<f64x2>>(p));
    } else if constexpr (std::is_same<ST, float>::value) {
        __builtin_nontemporal_store(f32x2{a, b}, reinterpret_cast<global_ptr<f32x2>>(p));
    } else if constexpr (std::is_same<ST, fx32_t>::value) {
        typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
        __builtin_nontemporal_store(i32x2{from_compute<ST>(a).v, from_compute<ST>(b).v}, reinterpret_cast<global_ptr<i32x2>>(p));
    } else if constexpr (std::is_same<ST, bf16_t>::value || std::is_same<ST, f16_t>::value) {
        using H2 = typename std::conditional<std::is_same<ST, bf16_t>::value, bf16x2, f16x2>::type;
        const H2 h = __builtin_convertvector(f32x2{a, b}, H2);
        uint32_t bits;
        __builtin_memcpy(&bits, &h, 4);
        __builtin_nontemporal_store(bits, reinterpret_cast<global_ptr<uint32_t>>(p));
    } else {
        // int16, the result of from_compute in fewer instructions: clamp to
        // the int16 range (NaN becomes -32768), then add 1.5 * 2^23.  The sum
        // lies in [2^23, 2^24), where FP32 values are the integers, so the
        // addition itself rounds to the nearest integer, ties to even (the
        // offset is even); the offset is a multiple of 2^16, so the low 16
        // bits of the sum are that integer in two's complement.  One byte
        // permutation packs the two low halves.  (Clamping before rounding
        // gives the same result: the bounds are integers.)
        static_assert(std::is_same<ST, fx16_t>::value, "int16 fixed point");
        constexpr float kRoundOffset = 12582912.0f;   // 1.5 * 2^23
        const float ra = __builtin_fminf(__builtin_fmaxf(a, -32768.0f), 32767.0f) + kRoundOffset;
        const float rb = __builtin_fminf(__builtin_fmaxf(b, -32768.0f), 32767.0f) + kRoundOffset;
        // bytes 0, 1 of ra, then bytes 0, 1 of rb
        const uint32_t bits = __builtin_amdgcn_perm(__float_as_uint(rb), __float_as_uint(ra), 0x05040100u);
        __builtin_nontemporal_store(bits, reinterpret_cast<global_ptr<uint32_t>>(p));
    }
}

template <typename ST>
__device__ __forceinline__ PointCoefs<typename compute_of<ST>::type> point_coefs(const DomainArgs& d, int k) {
    using CT = typename compute_of<ST>::type;
    PointCoefs<CT> c;
    c.xu = static_cast<CT>(d.cx[0]);
    c.yu = static_cast<CT>(d.cy[0]);
    c.xv = static_cast<CT>(d.cx[1]);
    c.yv = static_cast<CT>(d.cy[1]);
    c.xw = static_cast<CT>(d.cx[2]);
    c.yw = static_cast<CT>(d.cy[2]);
    double z1 = 0.0, z2 = 0.0, e1 = 0.0, e2 = 0.0;
    if (k >= 2) {
        z1 = as_global(d.tzc1)[k - 1];
        z2 = as_global(d.tzc2)[k - 1];
        if (k < d.nz) {
            e1 = as_global(d.tzd1)[k - 1];
            e2 = as_global(d.tzd2)[k - 1];
        }
    }
    c.z1u = static_cast<CT>(z1 * d.cz[0]);
    c.z2u = static_cast<CT>(z2 * d.cz[0]);
    c.z1v = static_cast<CT>(z1 * d.cz[1]);
    c.z2v = static_cast<CT>(z2 * d.cz[1]);
    c.z1w = static_cast<CT>(e1 * d.cz[2]);
    c.z2w = static_cast<CT>(e2 * d.cz[2]);
    return c;
}

// ---------------------------------------------------------------------------
// direct variant
// ---------------------------------------------------------------------------
template <typename ST>
struct GAcc {
    using CT = typename compute_of<ST>::type;
    const ST* pu;
    const ST* pv;
    const ST* pw;
    int64_t sy, sx;
    template <int dk, int dj, int di>
    __device__ __forceinline__ CT u() const { return to_compute(pu[dk + dj * sy + di * sx]); }
    template <int dk, int dj, int di>
    __device__ __forceinline__ CT v() const { return to_compute(pv[dk + dj * sy + di * sx]); }
    template <int dk, int dj, int di>
    __device__ __forceinline__ CT w() const { return to_compute(pw[dk + dj * sy + di * sx]); }
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
               static_cast<const ST*>(d.w) + off, d.sy, d.sx};
    const PointCoefs<CT> c = point_coefs<ST>(d, k);
    CT su, sv, sw;
    pw_point<typename arith_of<ST>::type, true>(A, k, d.nz, c, su, sv, sw);
    store_out(as_global(static_cast<ST*>(d.su) + off), su);
    store_out(as_global(static_cast<ST*>(d.sv) + off), sv);
    store_out(as_global(static_cast<ST*>(d.sw) + off), sw);
}

// ---------------------------------------------------------------------------
// march variant
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the XCDs (workgroup b runs on
// XCD b mod 8), in order of b.  Two tile orders follow from that.
//
// Compact order (march_compact_tile), used when a plane has at least 8
// chunks: XCD x owns the contiguous chunk range [x nc / 8, (x + 1) nc / 8)
// of every segment and walks it segment by segment, so at any time all XCDs
// work on the same one or two segments -- the HBM traffic of the whole chip
// stays in a narrow band of x planes -- while the chunks that share a y-halo
// column still meet in one XCD's L2.  Each XCD gets cpx = ceil(nc / 8) slots
// per segment; with nc not a multiple of 8 some slots are empty and their
// workgroups exit at once.  Measured on 2048 x 2048 x 64 against the
// XCD-contiguous order: FP64 3-4% faster, BF16 2-3%; on 512 x 512 x 64 FP64
// with 16-plane segments 14% faster.
//
// XCD-contiguous order (xcd_tile), for fewer than 8 chunks per plane: each
// XCD receives a contiguous range of the chunk-fastest tile list.
__device__ __forceinline__ bool march_compact_tile(int b, int nchunks, int cpx, int& c, int& s) {
    const int x = b % kNumXcd;
    const int slot = b / kNumXcd;
    s = slot / cpx;
    const int lo = x * nchunks / kNumXcd;
    const int hi = (x + 1) * nchunks / kNumXcd;
    c = lo + slot % cpx;
    return c < hi;
}
__device__ __forceinline__ int xcd_tile(int b, int G) {
    const int q = G / kNumXcd;
    const int r = G % kNumXcd;
    const int x = b % kNumXcd;
    const int slot = b / kNumXcd;
    return x * q + (x < r ? x : r) + slot;
}

// LDS reads around one point; NZ > 0 makes every offset an immediate.
template <typename CT, int NZ, int WPAD>
struct LdsAcc {
    const CT* m;   // plane i-1 at the point's window index
    const CT* c;   // plane i
    const CT* p;   // plane i+1
    int nz_rt, wp_rt;
    __device__ __forceinline__ int nz() const { return NZ > 0 ? NZ : nz_rt; }
    __device__ __forceinline__ int wp() const { return NZ > 0 ? WPAD : wp_rt; }
    template <int di> __device__ __forceinline__ const CT* sel() const {
        return di < 0 ? m : (di > 0 ? p : c);
    }
    template <int dk, int dj, int di>
    __device__ __forceinline__ CT u() const { return sel<di>()[dk + dj * nz()]; }
    template <int dk, int dj, int di>
    __device__ __forceinline__ CT v() const { return sel<di>()[wp() + dk + dj * nz()]; }
    template <int dk, int dj, int di>
    __device__ __forceinline__ CT w() const { return sel<di>()[2 * wp() + dk + dj * nz()]; }
};

constexpr int round_up4(int x) { return (x + 3) / 4 * 4; }
constexpr int gcd_int(int a, int b) { return b == 0 ? a : gcd_int(b, a % b); }

template <typename CT> struct vec2_of;
template <> struct vec2_of<double> { using type = f64x2; };
template <> struct vec2_of<float> { using type = f32x2; };

// LDS reads for point O (0 or 1) of a pair of consecutive levels whose first
// point sits at an even window index: every read is an aligned two-element
// load (8 or 16 bytes per lane, so lanes at an 8- or 16-byte stride hit the
// LDS banks without conflicts), and the two points' identical loads are
// shared.
template <typename CT, int NZ, int WPAD, int O>
struct PairAcc {
    // field F of plane i-1, i, i+1 at the pair's (even) window index
    const CT* m[3];
    const CT* c[3];
    const CT* p[3];
    template <int F, int di> __device__ __forceinline__ const CT* sel() const {
        return di < 0 ? m[F] : (di > 0 ? p[F] : c[F]);
    }
    template <int F, int dk, int dj, int di>
    __device__ __forceinline__ CT get() const {
        constexpr int e = O + dk;                              // -1 .. 2 from the pair start
        constexpr int start = e < 0 ? -2 : (e >= 2 ? 2 : 0);   // aligned two-element block
        using V2 = typename vec2_of<CT>::type;
        const V2 val = *reinterpret_cast<const V2*>(sel<F, di>() + dj * NZ + start);
        return val[e - start];
    }
    template <int dk, int dj, int di> __device__ __forceinline__ CT u() const { return get<0, dk, dj, di>(); }
    template <int dk, int dj, int di> __device__ __forceinline__ CT v() const { return get<1, dk, dj, di>(); }
    template <int dk, int dj, int di> __device__ __forceinline__ CT w() const { return get<2, dk, dj, di>(); }
};

// Planes held in the LDS ring: four for FP32 compute (one barrier per plane),
// three for FP64, whose larger slots would otherwise cost occupancy.
template <typename CT> constexpr int march_slots() { return sizeof(CT) == 4 ? 4 : 3; }

// The aligned two-level blocks a pair of levels reads: field F, row offset dj,
// plane offset di, block b in {-2, 0, 2} levels from the pair's start.  The
// stencil's reads (pw_point) per (field, dj, di) as a mask of level offsets
// dk (bit 0: dk = -1, bit 1: dk = 0, bit 2: dk = +1); a read at dk touches
// block -2 (dk = -1, first point), block 0 (every dk) and block 2 (dk = +1,
// second point).
constexpr int pair_dk_mask(int F, int dj, int di) {
    // [field][dj + 1][di + 1]
    constexpr int mask[3][3][3] = {{{0, 2, 0}, {6, 7, 2}, {2, 2, 0}},    // u
                                   {{0, 6, 2}, {2, 7, 2}, {0, 2, 0}},    // v
                                   {{0, 2, 0}, {2, 7, 3}, {0, 3, 0}}};   // w
    return mask[F][dj + 1][di + 1];
}
constexpr bool pair_block_used(int F, int dj, int di, int b) {
    return b == -2 ? (pair_dk_mask(F, dj, di) & 1) != 0
                   : (b == 0 ? pair_dk_mask(F, dj, di) != 0 : (pair_dk_mask(F, dj, di) & 4) != 0);
}
constexpr int pair_key(int F, int dj, int di, int b) { return ((F * 3 + dj + 1) * 3 + di + 1) * 3 + b / 2 + 1; }
constexpr int pair_carry_key(int F, int dj, int b) { return (F * 3 + dj + 1) * 3 + b / 2 + 1; }

// Pair reads from blocks already held in registers (indexed by pair_key).
template <typename CT, int O>
struct CachedPairAcc {
    using V2 = typename vec2_of<CT>::type;
    const V2* blk;
    template <int F, int dk, int dj, int di>
    __device__ __forceinline__ CT get() const {
        constexpr int e = O + dk;
        constexpr int start = e < 0 ? -2 : (e >= 2 ? 2 : 0);
        static_assert(pair_block_used(F, dj, di, start), "block missing from the pair block table");
        return blk[pair_key(F, dj, di, start)][e - start];
    }
    template <int dk, int dj, int di> __device__ __forceinline__ CT u() const { return get<0, dk, dj, di>(); }
    template <int dk, int dj, int di> __device__ __forceinline__ CT v() const { return get<1, dk, dj, di>(); }
    template <int dk, int dj, int di> __device__ __forceinline__ CT w() const { return get<2, dk, dj, di>(); }
};

// One (chunk, segment) tile of the march: chunk c of the interior (j, k) run,
// planes i_begin .. i_end.  Every thread of the workgroup must run it (it
// holds barriers); `lds` must hold 3 * march_slots<CT>() * wpad compute-type
// elements.
// NZ > 0: the domain's nz equals NZ and wpad equals round_up4(P + 2 NZ).
template <typename ST, int NT, int P, bool VEC, int NZ, int DIST = 2, bool FORCE_EXACT = false>
struct MarchTile {
    using CT = typename compute_of<ST>::type;
    // Elements per load: as many as fill 16 bytes of LDS in the compute type,
    // so each lane's write of a converted vector is one conflict-free 16-byte
    // store (16-bit and int32 storage then load 8 bytes per lane).
    static constexpr int VW = VEC ? int(16 / sizeof(CT)) : 1;
    static constexpr int WMAX = P + 2 * (NZ > 0 ? NZ : kMarchMaxNz);      // largest window
    static constexpr int NVR = (3 * (WMAX / VW) + NT - 1) / NT;           // load rounds per thread (3 fields)
    static constexpr int PPT = P / NT;                                     // points per thread
    static constexpr bool PAIR = VEC && NZ > 0 && NZ % 2 == 0 && P % (2 * NT) == 0;
    static constexpr int WPAD = NZ > 0 ? round_up4(P + 2 * NZ) : 0;
    // Branch-free data movement (see the constructor) where storage is
    // narrower than the compute type: those kernels are bound by instruction
    // issue, and exact load counting lets two planes stay in flight.  FP32
    // and FP64 storage are bound by HBM and keep the branches, which cost
    // fewer registers (measured: 4% faster for them, 4-23% slower for the
    // converting types).
    static constexpr bool EXACT = NZ > 0 && (FORCE_EXACT || sizeof(ST) < sizeof(CT));
    static constexpr int NSLOT = march_slots<CT>();                       // planes in the LDS ring
    static_assert(!VEC || VW * sizeof(ST) == 16 || VW * sizeof(ST) == 8, "8- or 16-byte loads");
    using Raw = typename std::conditional<VEC, typename std::conditional<VW * sizeof(ST) == 16, uint4, uint2>::type,
                                          ST>::type;
    static_assert(P % NT == 0, "P must be a multiple of the block size");

    const DomainArgs& d;
    CT* lds;
    int nz_rt, wpad_rt, wb, wlen, pend;
    int li[PPT];
    int kk[PPT];
    bool live[PPT];          // point lies in the chunk (always true when EXACT)
    CT hx[3], hy[3];       // uniform x and y coefficients of su, sv, sw
    CT zc[PPT][6];         // per-level vertical coefficients of each point
    // CARRY (with the branch-free data movement): blocks read at plane i as
    // "this plane" or "next plane" are kept in registers and reused at plane
    // i+1 as "previous plane" or "this plane", so a pair reads 17 of its 27
    // blocks from LDS instead of all of them.  cm: blocks for di = -1, c0:
    // blocks for di = 0, both indexed by pair_carry_key.  (FP32 storage,
    // bound by HBM, measured 4% slower with it: the carried registers cost a
    // resident workgroup per CU.)
    static constexpr bool CARRY = PAIR && EXACT;
    using V2 = typename vec2_of<CT>::type;
    V2 cm[CARRY ? PPT / 2 : 1][27];
    V2 c0[CARRY ? PPT / 2 : 1][27];
    // CARRY: the x-face sums of sv's and sw's x terms, carried from plane to
    // plane (pw_point's xs), so each is formed once instead of twice
    CT xs[CARRY ? PPT : 1][2];
    // ZEND (fixed-point storage with the register carry, policies where a
    // zero product is an exact zero): the column's end points get zero
    // coefficients instead of selects -- all of them at k = 1, and at the top
    // the upper vertical coefficients of su and sv and the horizontal ones of
    // sw (tzd1, tzd2 are zero there already).  With finite operands that gives
    // a zero at k = 1, the column-top forms at k = nz and sw(nz) = 0; the zero
    // may carry either sign, which the integer output does not keep.  Floating
    // storage keeps the selects: its k = 1 outputs are +0 bit for bit, and no
    // value above the column top (level 1 of the next column) can reach a
    // result through 0 x Inf.  ph: per-point copies of the horizontal
    // coefficients xu, yu, yv, xv, xw, yw.
    static constexpr bool ZEND = CARRY && arith_of<ST>::type::kExactZeroFlux && is_fixed_point<ST>;
    CT ph[ZEND ? PPT : 1][6];
    // The window vectors of all three fields are spread over the workgroup:
    // round r of this thread moves vector t + r NT -- field fsel[r] (-1: none),
    // element pointer gp[r] into the window of the next plane to load, LDS
    // offset loff[r].  Planes are loaded in order, so each load advances gp
    // by one plane (a 64-bit add of a uniform stride instead of a multiply).
    int fsel[NVR];
    global_ptr<const char> gp[NVR];
    int loff[NVR];
    // DIST planes in flight: plane p lives in register set (p - i_begin + 1) % DIST
    static_assert(DIST == 2 || DIST == 3, "two or three planes in flight");
    static constexpr int UNROLL = NSLOT * DIST / gcd_int(NSLOT, DIST);   // steps until slots and sets repeat
    static_assert(UNROLL <= 6, "unrolled block too long");
    Raw st[DIST][NVR];

    __device__ __forceinline__ int nz() const { return NZ > 0 ? NZ : nz_rt; }
    __device__ __forceinline__ int wpad() const { return NZ > 0 ? WPAD : wpad_rt; }
    __device__ __forceinline__ int slot_elems() const { return 3 * wpad(); }

    __device__ __forceinline__ MarchTile(const DomainArgs& dd, int c, int wpad_in, CT* l)
        : d(dd), lds(l), nz_rt(dd.nz), wpad_rt(wpad_in) {
        const int n = nz();
        const int p0 = n + c * P;                       // first point of the chunk (j >= 1)
        pend = min(p0 + P, (d.ny + 1) * n);             // one past the last interior point
        wb = p0 - n;                                    // window start: one column of y halo
        wlen = min(P + 2 * n, (d.ny + 2) * n - wb);
        const int nvec = wlen / VW;   // vectors per field (wlen is a multiple of VW)
#pragma unroll
        for (int r = 0; r < NVR; ++r) {
            // With a compile-time height the rounds fit the window exactly but
            // for the last round's tail; those lanes wrap round and move a
            // duplicate of an early vector (identical data to the same LDS
            // place), so loads and LDS writes need no branch and the compiler
            // can count outstanding loads exactly instead of waiting for all.
            const int v = EXACT ? ((int)threadIdx.x + r * NT) % (3 * nvec) : (int)threadIdx.x + r * NT;
            const int f = v < 3 * nvec ? v / nvec : -1;
            const int q = (v - (f < 0 ? 0 : f) * nvec) * VW;
            fsel[r] = f;
            const ST* base = static_cast<const ST*>(f == 0 ? d.u : (f == 1 ? d.v : d.w));
            gp[r] = as_global(reinterpret_cast<const char*>(base + (wb + q)));   // plane 0
            loff[r] = (f < 0 ? 0 : f) * wpad() + q;
        }
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int t = (int)threadIdx.x;
            int p = PAIR ? p0 + 2 * (t + NT * (q / 2)) + (q % 2) : p0 + t + NT * q;
            live[q] = p < pend;
            // EXACT: points past the chunk's end (last chunk of a domain)
            // recompute the chunk's last point or pair and store the
            // identical result again, so stores need no branch either.
            if (EXACT && !live[q]) {
                p = PAIR ? pend - 2 + (q % 2) : pend - 1;
                live[q] = true;
            }
            kk[q] = p % n + 1;
            li[q] = p - wb;
            const PointCoefs<CT> c = point_coefs<ST>(d, live[q] ? kk[q] : 1);
            zc[q][0] = c.z1u;
            zc[q][1] = c.z2u;
            zc[q][2] = c.z1v;
            zc[q][3] = c.z2v;
            zc[q][4] = c.z1w;
            zc[q][5] = c.z2w;
        }
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            hx[f] = static_cast<CT>(d.cx[f]);
            hy[f] = static_cast<CT>(d.cy[f]);
        }
        if constexpr (ZEND) {
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const CT h[6] = {hx[0], hy[0], hy[1], hx[1], hx[2], hy[2]};
                const bool bottom = q % 2 == 0 && kk[q] == 1;   // first level of a pair: odd k
                const bool top = q % 2 == 1 && kk[q] == n;      // second level: even k
#pragma unroll
                for (int e = 0; e < 6; ++e) ph[q][e] = (bottom || (top && e >= 4)) ? CT(0) : h[e];
                if (bottom) {
#pragma unroll
                    for (int e = 0; e < 6; ++e) zc[q][e] = CT(0);
                }
                if (top) {
                    zc[q][1] = CT(0);   // tzc2 of su
                    zc[q][3] = CT(0);   // tzc2 of sv
                }
            }
        }
    }

    // Move the load pointers to plane ip.
    __device__ __forceinline__ void seek(int64_t ip) {
        const int64_t po = ip * d.sx * (int64_t)sizeof(ST);
#pragma unroll
        for (int r = 0; r < NVR; ++r) gp[r] += po;
    }
    // Issue the global loads of the window of the next plane into `dst`.
    __device__ __forceinline__ void load_next(Raw* dst) {
        const int64_t ps = d.sx * (int64_t)sizeof(ST);   // uniform plane stride in bytes
#pragma unroll
        for (int r = 0; r < NVR; ++r) {
            if (EXACT || fsel[r] >= 0) dst[r] = load_global<Raw>(gp[r]);
            gp[r] += ps;
        }
    }

    // Convert staged values to the compute type and write them to a slot.
    __device__ __forceinline__ void put_from(const Raw* src, int sidx) {
        CT* slot = lds + sidx * slot_elems();
#pragma unroll
        for (int r = 0; r < NVR; ++r) {
            if (EXACT || fsel[r] >= 0) {
                union {
                    Raw raw;
                    ST e[VW];
                } cv;
                cv.raw = src[r];
                CT out[VW];
                if constexpr (std::is_same<ST, bf16_t>::value && VEC) {
                    // a BF16 value is the upper half of its FP32 value: per
                    // 32-bit word, shift the low element up, mask the high one
                    uint32_t wd[sizeof(Raw) / 4];
                    __builtin_memcpy(wd, &cv.raw, sizeof(Raw));
#pragma unroll
                    for (int n = 0; n < VW / 2; ++n) {
                        out[2 * n] = __uint_as_float(wd[n] << 16);
                        out[2 * n + 1] = __uint_as_float(wd[n] & 0xffff0000u);
                    }
                } else {
#pragma unroll
                    for (int n = 0; n < VW; ++n) out[n] = to_compute(cv.e[n]);
                }
                CT* dst = slot + loff[r];
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

    // LDS address of field F of ring slot `slot` at pair pq's window index.
    __device__ __forceinline__ const CT* block_base(int pq, int slot, int F) const {
        return lds + slot * slot_elems() + F * WPAD + li[2 * pq];
    }

    // CARRY: this step's blocks of pair pq, from the carried registers where
    // the previous step read them, else from LDS (slots sm, sc, sp hold planes
    // i-1, i, i+1).  Compile-time loop over all 81 keys; unused keys vanish.
    // Each LDS read is a single 8-byte read at an immediate offset from the
    // pair's one base address (every slot, field and row lies within the
    // 64 KiB offset range).  A scheduling barrier after each read keeps the
    // compiler from pairing reads into two-address reads, whose 2 KiB offset
    // range would cost a vector add for a new base address nearly every
    // time: in these VALU-bound kernels five such adds per plane and thread
    // measured slower than the extra LDS instructions.
    template <int K>
    __device__ __forceinline__ void gather_blocks(V2* blk, int pq, int sm, int sc, int sp) {
        if constexpr (K < 81) {
            constexpr int F = K / 27, dj = (K / 9) % 3 - 1, di = (K / 3) % 3 - 1, b = (K % 3 - 1) * 2;
            if constexpr (pair_block_used(F, dj, di, b)) {
                if constexpr (di == -1 && pair_block_used(F, dj, 0, b)) {
                    blk[K] = cm[pq][pair_carry_key(F, dj, b)];
                } else if constexpr (di == 0 && pair_block_used(F, dj, 1, b)) {
                    blk[K] = c0[pq][pair_carry_key(F, dj, b)];
                } else {
                    const int slot = di < 0 ? sm : (di > 0 ? sp : sc);
                    blk[K] = *reinterpret_cast<const V2*>(block_base(pq, slot, F) + dj * NZ + b);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            gather_blocks<K + 1>(blk, pq, sm, sc, sp);
        }
    }
    // CARRY: keep this step's blocks that the next step reuses.
    template <int K>
    __device__ __forceinline__ void keep_blocks(const V2* blk, int pq) {
        if constexpr (K < 27) {
            constexpr int F = K / 9, dj = (K / 3) % 3 - 1, b = (K % 3 - 1) * 2;
            if constexpr (pair_block_used(F, dj, -1, b) && pair_block_used(F, dj, 0, b))
                cm[pq][K] = blk[pair_key(F, dj, 0, b)];
            if constexpr (pair_block_used(F, dj, 0, b) && pair_block_used(F, dj, 1, b))
                c0[pq][K] = blk[pair_key(F, dj, 1, b)];
            keep_blocks<K + 1>(blk, pq);
        }
    }
    // CARRY: before a tile's first step, load the carried blocks from planes
    // i_begin - 1 (slot 0) and i_begin (slot 1).
    template <int K>
    __device__ __forceinline__ void prime_blocks(int pq) {
        if constexpr (K < 27) {
            constexpr int F = K / 9, dj = (K / 3) % 3 - 1, b = (K % 3 - 1) * 2;
            if constexpr (pair_block_used(F, dj, -1, b) && pair_block_used(F, dj, 0, b))
                cm[pq][K] = *reinterpret_cast<const V2*>(block_base(pq, 0, F) + dj * NZ + b);
            if constexpr (pair_block_used(F, dj, 0, b) && pair_block_used(F, dj, 1, b))
                c0[pq][K] = *reinterpret_cast<const V2*>(block_base(pq, 1, F) + dj * NZ + b);
            prime_blocks<K + 1>(pq);
        }
    }

    // CARRY: the x-face sums at plane i_begin - 1 from the carried blocks of
    // that plane (cm, just primed), in the order pw_point forms them.
    __device__ __forceinline__ void prime_sums(int pq) {
        constexpr int kU0 = pair_carry_key(0, 0, 0), kU0b = pair_carry_key(0, 0, 2), kU1 = pair_carry_key(0, 1, 0);
        static_assert(pair_block_used(0, 0, -1, 0) && pair_block_used(0, 0, 0, 0) && pair_block_used(0, 0, -1, 2) &&
                          pair_block_used(0, 0, 0, 2) && pair_block_used(0, 1, -1, 0) && pair_block_used(0, 1, 0, 0),
                      "sum blocks must be carried");
        const V2 a = cm[pq][kU0], b = cm[pq][kU0b], r = cm[pq][kU1];
        xs[2 * pq][0] = a[0] + r[0];       // u(k, j) + u(k, j+1)
        xs[2 * pq][1] = a[0] + a[1];       // u(k) + u(k+1)
        xs[2 * pq + 1][0] = a[1] + r[1];
        xs[2 * pq + 1][1] = a[1] + b[0];
    }

    // Compute plane i from the slots sm (plane i-1), sc (plane i), sp (plane i+1).
    __device__ __forceinline__ void compute(int i, int sm, int sc, int sp) {
        const int64_t obase = (int64_t)i * d.sx + wb;
        const int se = slot_elems();
        using AR = typename arith_of<ST>::type;
        CT res[PPT][3];
        V2 blk[CARRY ? PPT / 2 : 1][81];   // CARRY: this step's blocks, indexed by pair_key
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int l = li[q];
            const PointCoefs<CT> c = ZEND ? PointCoefs<CT>{ph[q][0], ph[q][1], zc[q][0], zc[q][1],
                                                           ph[q][2], ph[q][3], zc[q][2], zc[q][3],
                                                           ph[q][4], ph[q][5], zc[q][4], zc[q][5]}
                                          : PointCoefs<CT>{hx[0], hy[0], zc[q][0], zc[q][1], hy[1], hx[1],
                                                           zc[q][2], zc[q][3], hx[2], hy[2], zc[q][4], zc[q][5]};
            if constexpr (CARRY) {
                if (q % 2 == 0) gather_blocks<0>(blk[q / 2], q / 2, sm, sc, sp);
                if (q % 2 == 0) {
                    CachedPairAcc<CT, 0> A{blk[q / 2]};
                    pw_point<AR, false, !ZEND, false>(A, kk[q], nz(), c, res[q][0], res[q][1], res[q][2], xs[q]);
                } else {
                    CachedPairAcc<CT, 1> A{blk[q / 2]};
                    pw_point<AR, false, false, !ZEND>(A, kk[q], nz(), c, res[q][0], res[q][1], res[q][2], xs[q]);
                    keep_blocks<0>(blk[q / 2], q / 2);
                }
            } else if constexpr (PAIR) {
                const CT *m[3], *cc[3], *pp[3];
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const int l0 = li[q & ~1];   // the pair's first (even) index
                    m[f] = lds + sm * se + f * WPAD + l0;
                    cc[f] = lds + sc * se + f * WPAD + l0;
                    pp[f] = lds + sp * se + f * WPAD + l0;
                }
                // the pair's first level is odd (k = 1 possible, never the
                // top); the second is even (never k = 1, the top possible)
                if (q % 2 == 0) {
                    PairAcc<CT, NZ, WPAD, 0> A{{m[0], m[1], m[2]}, {cc[0], cc[1], cc[2]}, {pp[0], pp[1], pp[2]}};
                    pw_point<AR, false, true, false>(A, kk[q], nz(), c, res[q][0], res[q][1], res[q][2]);
                } else {
                    PairAcc<CT, NZ, WPAD, 1> A{{m[0], m[1], m[2]}, {cc[0], cc[1], cc[2]}, {pp[0], pp[1], pp[2]}};
                    pw_point<AR, false, false, true>(A, kk[q], nz(), c, res[q][0], res[q][1], res[q][2]);
                }
            } else {
                LdsAcc<CT, NZ, WPAD> A{lds + sm * se + l, lds + sc * se + l, lds + sp * se + l, nz_rt, wpad()};
                pw_point<AR, false>(A, kk[q], nz(), c, res[q][0], res[q][1], res[q][2]);
            }
        }
        global_ptr<ST> outs[3] = {as_global(static_cast<ST*>(d.su) + obase), as_global(static_cast<ST*>(d.sv) + obase),
                                  as_global(static_cast<ST*>(d.sw) + obase)};
        if constexpr (PAIR) {
#pragma unroll
            for (int q = 0; q < PPT; q += 2) {
                if (!EXACT && !live[q]) continue;   // a pair never straddles the chunk end (P, nz even)
#pragma unroll
                for (int f = 0; f < 3; ++f) store_pair(outs[f] + (uint32_t)li[q], res[q][f], res[q + 1][f]);
            }
        } else {
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                if (!EXACT && !live[q]) continue;
#pragma unroll
                for (int f = 0; f < 3; ++f) store_out(outs[f] + (uint32_t)li[q], res[q][f]);
            }
        }
    }

    // One march step: publish plane i+1, prefetch plane i+1+DIST, compute
    // plane i.  DIST register sets keep DIST planes in flight, so each load
    // has DIST steps to arrive; SET = (i - i_begin) % DIST holds plane i+1
    // and then receives plane i+1+DIST.  With three slots the slot of plane
    // i-1 is refilled by the next step, so a second barrier keeps it until
    // every wave has computed plane i; with four slots that refill happens
    // one step later, behind the next step's barrier, and one barrier per
    // plane suffices.
    template <int SET>
    __device__ __forceinline__ void step(int i, int i_end, int sm, int sc, int sp) {
        put_from(st[SET], sp);
        __syncthreads();
        if (i + 1 + DIST <= i_end + 1) load_next(st[SET]);   // plane i + 1 + DIST
        compute(i, sm, sc, sp);
        if constexpr (NSLOT == 3) __syncthreads();
    }

    // Steps R .. UNROLL-1 of one unrolled block starting at plane i; slots and
    // register sets are compile-time constants.  Returns false past i_end.
    template <int R>
    __device__ __forceinline__ bool block(int i, int i_end) {
        if constexpr (R == UNROLL) {
            return true;
        } else {
            if (i + R > i_end) return false;
            step<R % DIST>(i + R, i_end, R % NSLOT, (R + 1) % NSLOT, (R + 2) % NSLOT);
            return block<R + 1>(i, i_end);
        }
    }

    // Run-time slots (any column height): DIST steps per iteration so the
    // register sets stay compile-time.
    template <int R>
    __device__ __forceinline__ bool block_rt(int i, int i_end, int& sm, int& sc, int& sp) {
        if constexpr (R == DIST) {
            return true;
        } else {
            if (i + R > i_end) return false;
            step<R>(i + R, i_end, sm, sc, sp);
            sm = sc;
            sc = sp;
            sp = sp + 1 == NSLOT ? 0 : sp + 1;
            return block_rt<R + 1>(i, i_end, sm, sc, sp);
        }
    }

    __device__ __forceinline__ void run(int i_begin, int i_end) {
        // the first planes are requested together, so a tile's start waits
        // for one memory latency, not several
        {
            // planes i_begin - 1, i_begin, i_begin + 1 (<= nx + 1, always
            // there), then up to i_begin + DIST; the steps continue in order
            // with plane i + 1 + DIST, and once one plane lies past i_end + 1
            // every later one does too
            Raw a[NVR], b[NVR];
            seek((int64_t)(i_begin - 1));
            load_next(a);
            load_next(b);
            load_next(st[0]);
#pragma unroll
            for (int q = 1; q < DIST; ++q) {
                if (i_begin + 1 + q <= i_end + 1) load_next(st[q]);
            }
            put_from(a, 0);
            put_from(b, 1);
        }
        if constexpr (CARRY) {
            __syncthreads();
#pragma unroll
            for (int pq = 0; pq < PPT / 2; ++pq) {
                prime_blocks<0>(pq);
                prime_sums(pq);
            }
        }
        if constexpr (NZ > 0) {
            for (int i = i_begin;; i += UNROLL) {
                if (!block<0>(i, i_end)) break;
            }
        } else {
            int sm = 0, sc = 1, sp = 2;
            for (int i = i_begin;; i += DIST) {
                if (!block_rt<0>(i, i_end, sm, sc, sp)) break;
            }
        }
        // the next tile of a persistent workgroup refills slots 0 and 1
        if constexpr (NSLOT == 4) __syncthreads();
    }
};

template <typename ST, int NT, int P, bool VEC, int NZ, int DIST = 2, bool FORCE_EXACT = false>
__device__ __forceinline__ void march_tile(const DomainArgs& d, int c, int i_begin, int i_end, int wpad,
                                           typename compute_of<ST>::type* lds) {
    MarchTile<ST, NT, P, VEC, NZ, DIST, FORCE_EXACT> t(d, c, wpad, lds);
    t.run(i_begin, i_end);
}

// Resident waves per SIMD the single-domain march kernel may reach: FP64
// storage is held at two (two workgroups per CU, each with two planes in
// flight): three workgroups per CU, with more planes in flight or without,
// measured 10% slower on 2048 x 2048 x 64 -- more concurrent streams cost
// the HBM more than the extra bytes in flight gain.  Other storage types are
// not capped.
template <typename ST> constexpr int march_max_waves() { return std::is_same<ST, double>::value ? 2 : 8; }

// Single domain: one workgroup per (chunk, segment) tile.
template <typename ST, int NT, int P, bool VEC, int NZ>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, march_max_waves<ST>())))
void pw_march_kernel(DomainArgs d, MarchGeom g) {
    using CT = typename compute_of<ST>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    CT* lds = reinterpret_cast<CT*>(smem_raw);
    int c, s;
    if (g.cpx > 0) {
        if (!march_compact_tile((int)blockIdx.x, g.nchunks, g.cpx, c, s)) return;   // empty slot, whole workgroup
    } else {
        const int tile = xcd_tile(blockIdx.x, gridDim.x);
        c = tile % g.nchunks;
        s = tile / g.nchunks;
    }
    const int i_begin = 1 + s * g.seg;
    const int i_end = min(i_begin + g.seg - 1, d.nx);
    march_tile<ST, NT, P, VEC, NZ>(d, c, i_begin, i_end, g.wpad, lds);
}

}  // namespace pw
