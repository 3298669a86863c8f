// Batched PW advection: many uneven subdomains in one launch, plus the
// periodic halo fill and the field perturbation used between repeated
// timestep calls.
//
// The plan flattens every domain's (chunk, segment) tiles into one global
// tile range (prefix sums in a device table).  By default one workgroup runs
// each tile (longest tiles first, handed to the XCDs in runs of neighbouring
// tiles); on request a persistent grid sized to the GPU walks the range
// instead (each XCD a contiguous share).  Each workgroup maps a tile to its
// domain (a binary search, then a forward scan) and runs the per-tile code
// of the single-domain march kernel.  The per-point arithmetic
// is the same source, and the library is built with FMA formed only within
// a source expression, so each domain's result is bit-identical to a
// pw_advect call (the result of a point does not depend on the tiling).
//
// Each domain splits its x range into segments of even length (at most the
// plan's segment length) rather than full segments and a short last one:
// tiles of equal length keep the workgroups that run neighbouring chunks in
// step, so the y-halo columns and boundary planes they share are still in L2
// when the second one reads them (measured on the 384-domain batch: 3-6%
// faster for FP64, FP32 and BF16).
//
// The tile list takes the domains longest tiles first (by segment length,
// then in the caller's order; each domain's tiles stay together), so the
// short tiles fill the end of the launch instead of a few long ones running
// alone.  The table row of a domain keeps the index of its record.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "pw_plan.hpp"

namespace pw {

namespace {

__device__ __forceinline__ bool shape_matches(const pw_shape& a, const BatchDomain& b) {
    const int64_t sy = a.sy ? a.sy : a.nz;
    const int64_t sx = a.sx ? a.sx : (int64_t)(a.ny + 2) * sy;
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.reserved == 0 && sy == b.sy && sx == b.sx;
}

__device__ __forceinline__ float scale_or_one(float s) { return s > 0.0f ? s : 1.0f; }

// A record's scale must be 0 (meaning 1) or a finite positive power of two
// (normal or subnormal), as pw_advect requires of its scales; folding such
// scales into the coefficients is exact.
__device__ __forceinline__ bool scale_ok(float s) {
    const uint32_t b = __float_as_uint(s);
    if (b == 0u) return true;                       // +0: default scale
    if (b >> 31) return false;                      // negative or -0
    const uint32_t e = (b >> 23) & 0xffu, m = b & 0x7fffffu;
    if (e == 0xffu) return false;                   // Inf or NaN
    return e != 0u ? m == 0u : __popc(m) == 1;
}

__device__ __forceinline__ bool scales_ok(const pw_scales& sc) {
    bool ok = true;
#pragma unroll
    for (int f = 0; f < 3; ++f) ok = ok && scale_ok(sc.in_scale[f]) && scale_ok(sc.out_scale[f]);
    return ok;
}

template <typename ST>
__device__ __forceinline__ DomainArgs domain_from(const pw_domain_args& a, const BatchDomain& b) {
    DomainArgs d{};
    d.u = a.u;
    d.v = a.v;
    d.w = a.w;
    d.su = a.su;
    d.sv = a.sv;
    d.sw = a.sw;
    d.tzc1 = a.tzc1;
    d.tzc2 = a.tzc2;
    d.tzd1 = a.tzd1;
    d.tzd2 = a.tzd2;
    float in_s[3], out_s[3];
    for (int f = 0; f < 3; ++f) {
        in_s[f] = scaled_type<ST>::value ? scale_or_one(a.scales.in_scale[f]) : 1.0f;
        out_s[f] = scaled_type<ST>::value ? scale_or_one(a.scales.out_scale[f]) : 1.0f;
    }
    fold_coefficients(a.tcx, a.tcy, in_s, out_s, d.cx, d.cy, d.cz);
    d.nx = b.nx;
    d.ny = b.ny;
    d.nz = b.nz;
    d.sy = b.sy;
    d.sx = b.sx;
    return d;
}

__device__ __forceinline__ int find_domain(const BatchDomain* table, int ndom, int64_t t) {
    int lo = 0, hi = ndom - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (table[mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Which per-tile code paths a batched kernel carries.  Every path inlined
// into the batched kernel counts towards its register allocation, so a
// plan launches the narrowest kind its shapes allow:
//   kFixedNz  vector loads, column heights 64 / 96 / 128 only;
//   kVector   vector loads, any column height;
//   kAny      also element-wise loads (shapes without vector alignment).
// The vector kinds need every field pointer 16-byte aligned; a record that
// is not is skipped and counted like a shape mismatch.
enum BatchKind { kFixedNz = 0, kVector = 1, kAny = 2 };

// gate: NULL, or a device word that must be nonzero for the launch to run
// (the allocation-free entry point's table check); if it is zero, workgroup
// 0 counts every domain as skipped and all workgroups exit.
// Tile order of one workgroup per tile (kOneTileRuns): XCD x of block g of
// the tile list takes tiles g 8R + x R .. g 8R + x R + R - 1, one per
// workgroup in dispatch order, so all XCDs work in the same window of the
// list at a time while runs of R neighbouring chunks meet in one XCD's L2;
// the grid is padded to whole blocks and workgroups past the last tile exit.
// Measured on the 384-domain batch against plain dispatch order: as fast or
// up to 1% faster, and the y-halo re-reads of neighbouring chunks hit L2.
constexpr int kOneTileRuns = 8;

// wg_per_cu 0 (the default) or PW_WG_ONE_PER_TILE: one workgroup per tile;
// 1..8: a persistent grid of that many workgroups per CU.
inline bool batched_one_per_tile(const pw_tuning& t) { return t.wg_per_cu <= 0; }

template <typename ST, int NT, int P, int KIND>
__global__ __launch_bounds__(NT) void pw_batched_kernel(const BatchDomain* __restrict__ table, int ndom,
                                                        int64_t ntiles, const pw_domain_args* __restrict__ args,
                                                        unsigned long long* errors,
                                                        int vec_shapes, int one_per_tile, const int32_t* __restrict__ order,
                                                        const uint32_t* gate) {
    using CT = typename compute_of<ST>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    CT* lds = reinterpret_cast<CT*>(smem_raw);
    if (gate != nullptr && *gate == 0u) {   // uniform over the grid
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(errors, (unsigned long long)ndom);
        return;
    }
    // Persistent grid: workgroups are dispatched round-robin over the XCDs;
    // each XCD gets a contiguous share of the tile range, walked by its own
    // workgroups, so the tiles in flight on one XCD are neighbouring chunks
    // and segments of the same domains and share their halo columns and
    // planes in its L2.
    const int G = (int)gridDim.x;
    const int x = (int)blockIdx.x % kNumXcd;
    const int slot = (int)blockIdx.x / kNumXcd;
    const int q = G / kNumXcd, r = G % kNumXcd;
    const int wgs = q + (x < r ? 1 : 0);                 // workgroups on this XCD
    const int before = x * q + (x < r ? x : r);          // workgroups on lower XCDs
    int64_t t_begin = ntiles * before / G + slot, t_end = ntiles * (before + wgs) / G, t_step = wgs;
    if (one_per_tile) {
        int64_t t;
        if (order != nullptr) {
            t = order[blockIdx.x];   // the plan's dispatch order; -1: no tile
        } else {
            const int64_t sl = blockIdx.x / kNumXcd;
            t = (sl / kOneTileRuns) * (kNumXcd * kOneTileRuns) + (int64_t)x * kOneTileRuns + sl % kOneTileRuns;
        }
        t_begin = t < 0 ? 0 : t;
        t_end = (t >= 0 && t < ntiles) ? t + 1 : t_begin;   // no tile: empty range
        t_step = 1;
    }
    int dom = -1;
    for (int64_t t = t_begin; t < t_end; t += t_step) {
        // tiles only move forward: after the first binary search a short
        // forward scan finds the domain (usually zero or one step)
        if (dom < 0) {
            dom = find_domain(table, ndom, t);
        } else {
            while (dom + 1 < ndom && table[dom + 1].tile_begin <= t) ++dom;
        }
        const BatchDomain b = table[dom];
        const int64_t local = t - b.tile_begin;
        const int c = (int)(local % b.nchunks);
        const int s = (int)(local / b.nchunks);
        const pw_domain_args& a = args[b.rec];
        if (!shape_matches(a.shape, b) || !a.u || !a.v || !a.w || !a.su || !a.sv || !a.sw ||
            (scaled_type<ST>::value && !scales_ok(a.scales))) {
            if (threadIdx.x == 0 && local == 0) atomicAdd(errors, 1ull);
            continue;   // uniform over the workgroup
        }
        const DomainArgs d = domain_from<ST>(a, b);
        const int i_begin = 1 + s * b.seg;   // <= nx: (nseg - 1) * seg < nx
        const int i_end = min(i_begin + b.seg - 1, b.nx);
        const bool vec = vec_shapes && aligned16(a.u) && aligned16(a.v) && aligned16(a.w) && aligned16(a.su) &&
                         aligned16(a.sv) && aligned16(a.sw);
        if (KIND != kAny && !vec) {
            if (threadIdx.x == 0 && local == 0) atomicAdd(errors, 1ull);
            continue;   // uniform over the workgroup
        }
        const int wpad = round_up4(P + 2 * b.nz);
        // Short tiles leave less time to hide a plane's latency: FP64
        // compute (three LDS slots) keeps three planes in flight, and every
        // storage type takes the branch-free data movement, whose exact
        // outstanding-load counts keep those planes in flight (measured on
        // the 384-domain batch: FP64 1.45 -> 1.22 ms, FP32 0.75 -> 0.64 ms).
        constexpr int D = march_slots<CT>() == 3 ? 3 : 2;
        constexpr bool X = true;
        if (vec && b.nz == 64) march_tile<ST, NT, P, true, 64, D, X>(d, c, i_begin, i_end, wpad, lds);
        else if (vec && b.nz == 96) march_tile<ST, NT, P, true, 96, D, X>(d, c, i_begin, i_end, wpad, lds);
        else if (vec && b.nz == 128) march_tile<ST, NT, P, true, 128, D, X>(d, c, i_begin, i_end, wpad, lds);
        else if constexpr (KIND != kFixedNz) {
            if (vec) march_tile<ST, NT, P, true, 0, D>(d, c, i_begin, i_end, wpad, lds);
            else if constexpr (KIND == kAny) march_tile<ST, NT, P, false, 0, D>(d, c, i_begin, i_end, wpad, lds);
        }
    }
}

// Storage elements moved as raw bits through global pointers (the storage
// structs cannot be assigned through an address-space-qualified lvalue).
template <int N> struct bits_of;
template <> struct bits_of<2> { using type = uint16_t; };
template <> struct bits_of<4> { using type = uint32_t; };
template <> struct bits_of<8> { using type = uint64_t; };
template <typename ST> using storage_bits = typename bits_of<sizeof(ST)>::type;
template <typename ST> __device__ __forceinline__ ST from_bits(storage_bits<ST> u) {
    ST x;
    __builtin_memcpy(&x, &u, sizeof(ST));
    return x;
}
template <typename ST> __device__ __forceinline__ storage_bits<ST> to_bits(ST x) {
    storage_bits<ST> u;
    __builtin_memcpy(&u, &x, sizeof(ST));
    return u;
}

// Periodic x-y halo of u, v, w.  Each halo column (i, j) copies interior
// column (wrap(i), wrap(j)) with wrap(0) = n, wrap(n + 1) = 1 -- the same
// result as filling x faces first and then y faces over the halo'd x range.
// grid: y over domains, x a number of workgroups sized to the mean domain's
// halo; each workgroup strides over its domain's halo elements (every
// element is written once, from an interior source, so the order is free).
template <typename ST>
__global__ __launch_bounds__(256) void pw_halo_kernel(const BatchDomain* __restrict__ table,
                                                      const pw_domain_args* __restrict__ args) {
    const BatchDomain b = table[blockIdx.y];
    const pw_domain_args& a = args[b.rec];
    if (!shape_matches(a.shape, b)) return;
    const int nhalo = 2 * (b.nx + 2) + 2 * b.ny;
    using U = storage_bits<ST>;
    global_ptr<U> f[3] = {as_global((U*)a.u), as_global((U*)a.v), as_global((U*)a.w)};
    const int64_t n = (int64_t)nhalo * b.nz;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (int64_t)gridDim.x * 256) {
        const int k = (int)(g % b.nz);
        const int h = (int)(g / b.nz);
        int i, j;
        if (h < b.nx + 2) {
            i = h;
            j = 0;
        } else if (h < 2 * (b.nx + 2)) {
            i = h - (b.nx + 2);
            j = b.ny + 1;
        } else if (h < 2 * (b.nx + 2) + b.ny) {
            i = 0;
            j = 1 + h - 2 * (b.nx + 2);
        } else {
            i = b.nx + 1;
            j = 1 + h - 2 * (b.nx + 2) - b.ny;
        }
        const int si = i == 0 ? b.nx : (i == b.nx + 1 ? 1 : i);
        const int sj = j == 0 ? b.ny : (j == b.ny + 1 ? 1 : j);
        const int64_t dst = k + (int64_t)j * b.sy + (int64_t)i * b.sx;
        const int64_t src = k + (int64_t)sj * b.sy + (int64_t)si * b.sx;
#pragma unroll
        for (int q = 0; q < 3; ++q) f[q][dst] = f[q][src];
    }
}

// SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014).
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

// 32-bit integer hash "lowbias32" (C. Wellons, "Prospecting for Hash
// Functions", 2018).
__device__ __forceinline__ uint32_t lowbias32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// u += amp * r, v += amp * r' on the interior, r uniform in [-1, 1) from a
// counter-based hash of (seed, call, domain, field, point); `call` is read
// from device memory so a captured graph perturbs differently on each replay.
// The (seed, call, domain) key is mixed once by SplitMix64; each element then
// costs one 32-bit hash of its field and its point index g = k + nz ((j - 1) +
// ny (i - 1)), so the values do not depend on how the work is split.
// One workgroup per tile of the plan (the batched kernel's split: a chunk of
// the (j, k) points of a plane times a segment of x planes), so every
// workgroup of the grid has work whatever the spread of domain sizes; each
// thread reads the points of kPerturbPlanes planes before it writes them.
constexpr int kPerturbPlanes = 4;

template <typename ST>
__global__ __launch_bounds__(256) void pw_perturb_kernel(const BatchDomain* __restrict__ table, int ndom, int chunk,
                                                         const pw_domain_args* __restrict__ args, uint64_t seed,
                                                         const unsigned long long* __restrict__ call, double amp) {
    using CT = typename compute_of<ST>::type;
    const int64_t t = blockIdx.x;
    const BatchDomain b = table[find_domain(table, ndom, t)];
    const int dom = b.rec;   // the caller's domain index keys the hash
    const pw_domain_args& a = args[dom];
    if (!shape_matches(a.shape, b)) return;
    const int64_t local = t - b.tile_begin;
    const int c = (int)(local % b.nchunks);
    const int sg = (int)(local / b.nchunks);
    const int i0 = 1 + sg * b.seg;                 // <= nx: segments start at or before plane nx
    const int i1 = min(i0 + b.seg - 1, b.nx);
    const uint32_t nz = (uint32_t)b.nz, nyz = (uint32_t)b.ny * (uint32_t)b.nz;   // nx ny nz < 2^31 (plan time)
    const uint32_t pend = min((uint32_t)(c + 1) * (uint32_t)chunk, nyz);
    const uint64_t key64 = splitmix64(seed ^ splitmix64((uint64_t)(*call) * 0x100000001b3ull + (uint64_t)dom));
    const uint32_t key = (uint32_t)key64 ^ (uint32_t)(key64 >> 32);
    using U = storage_bits<ST>;
    global_ptr<U> f[2] = {as_global((U*)a.u), as_global((U*)a.v)};
    const CT sc[2] = {static_cast<CT>(scaled_type<ST>::value ? scale_or_one(a.scales.in_scale[0]) : 1.0f),
                      static_cast<CT>(scaled_type<ST>::value ? scale_or_one(a.scales.in_scale[1]) : 1.0f)};
    uint32_t p = 0;
    // x + amp r (times the field's scale) at plane i of point p, field q
    auto perturbed = [&](CT x, int i, int q) {
        const uint32_t g = (uint32_t)(i - 1) * nyz + p;
        const uint32_t h = lowbias32(key ^ lowbias32(2u * g + (uint32_t)q));
        const float r = (float)(h >> 8) * 0x1.0p-23f - 1.0f;   // [-1, 1)
        return x + static_cast<CT>(amp * (double)r) * sc[q];
    };
    for (p = (uint32_t)c * (uint32_t)chunk + threadIdx.x; p < pend; p += 256) {
        const uint32_t k = p % nz;
        const uint32_t j = p / nz + 1;
        const int64_t col = k + (int64_t)j * b.sy;
        // full groups of kPerturbPlanes planes without conditions (so the
        // compiler keeps all their loads in flight), then the rest one by one
        int i = i0;
        for (; i + kPerturbPlanes - 1 <= i1; i += kPerturbPlanes) {
            CT x[kPerturbPlanes][2];
#pragma unroll
            for (int u = 0; u < kPerturbPlanes; ++u)
#pragma unroll
                for (int q = 0; q < 2; ++q) x[u][q] = to_compute(from_bits<ST>(f[q][col + (int64_t)(i + u) * b.sx]));
#pragma unroll
            for (int u = 0; u < kPerturbPlanes; ++u)
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    f[q][col + (int64_t)(i + u) * b.sx] = to_bits(from_compute<ST>(perturbed(x[u][q], i + u, q)));
        }
        for (; i <= i1; ++i) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const CT x = to_compute(from_bits<ST>(f[q][col + (int64_t)i * b.sx]));
                f[q][col + (int64_t)i * b.sx] = to_bits(from_compute<ST>(perturbed(x, i, q)));
            }
        }
    }
}

__global__ void pw_bump_kernel(unsigned long long* call) { *call += 1ull; }

// Everything one launch of the batched kernel needs besides the records.
struct BatchedLaunch {
    const BatchDomain* table;
    int32_t ndomains;
    int64_t tiles;
    int64_t workgroups;
    int64_t lds_bytes;
    unsigned long long* errors;
    const uint32_t* gate;
    bool vec_shapes;
    bool one_per_tile;
    const int32_t* order;   // one workgroup per tile: the plan's dispatch order, or NULL (runs of kOneTileRuns)
};

template <typename ST, int P, int KIND>
hipError_t launch_batched(const BatchedLaunch& bl, const pw_domain_args* args, hipStream_t stream) {
    auto kern = pw_batched_kernel<ST, 256, P, KIND>;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [&] {
        attr_err = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynamicLds);
    });
    if (attr_err != hipSuccess) return attr_err;
    hipLaunchKernelGGL(kern, dim3((unsigned)bl.workgroups), dim3(256), (size_t)bl.lds_bytes, stream, bl.table,
                       bl.ndomains, bl.tiles, args, bl.errors, bl.vec_shapes ? 1 : 0, bl.one_per_tile ? 1 : 0,
                       bl.order, bl.gate);
    return hipGetLastError();
}

template <typename ST, int P, int KIND>
int occupancy_of(int64_t lds_bytes) {
    int n = 0;
    auto kern = pw_batched_kernel<ST, 256, P, KIND>;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              kMaxDynamicLds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, 256, (size_t)lds_bytes) != hipSuccess) return 0;
    return n;
}

template <typename ST, int P>
int occupancy_kind(int32_t kind, int64_t lds_bytes) {
    switch (kind) {
        case kFixedNz: return occupancy_of<ST, P, kFixedNz>(lds_bytes);
        case kVector: return occupancy_of<ST, P, kVector>(lds_bytes);
        case kAny: return occupancy_of<ST, P, kAny>(lds_bytes);
        default: return 0;
    }
}

template <typename ST>
int occupancy_typed(int32_t chunk, int32_t kind, int64_t lds_bytes) {
    switch (chunk) {
        case 256: return occupancy_kind<ST, 256>(kind, lds_bytes);
        case 512: return occupancy_kind<ST, 512>(kind, lds_bytes);
        case 1024: return occupancy_kind<ST, 1024>(kind, lds_bytes);
        default: return 0;
    }
}

// Resident workgroups per CU of the batched kernel (registers and LDS).
int batched_occupancy(int32_t storage, int32_t chunk, int32_t kind, int64_t lds_bytes) {
    switch (storage) {
        case PW_F64: return occupancy_typed<double>(chunk, kind, lds_bytes);
        case PW_F32: return occupancy_typed<float>(chunk, kind, lds_bytes);
        case PW_BF16: return occupancy_typed<bf16_t>(chunk, kind, lds_bytes);
        case PW_F16: return occupancy_typed<f16_t>(chunk, kind, lds_bytes);
        case PW_I16: return occupancy_typed<fx16_t>(chunk, kind, lds_bytes);
        case PW_I32: return occupancy_typed<fx32_t>(chunk, kind, lds_bytes);
        default: return 0;
    }
}

template <typename ST, int P>
hipError_t dispatch_kind(int32_t kind, const BatchedLaunch& bl, const pw_domain_args* args, hipStream_t stream) {
    switch (kind) {
        case kFixedNz: return launch_batched<ST, P, kFixedNz>(bl, args, stream);
        case kVector: return launch_batched<ST, P, kVector>(bl, args, stream);
        case kAny: return launch_batched<ST, P, kAny>(bl, args, stream);
        default: return hipErrorInvalidValue;
    }
}

template <typename ST>
hipError_t dispatch_chunk(int32_t chunk, int32_t kind, const BatchedLaunch& bl, const pw_domain_args* args,
                          hipStream_t stream) {
    switch (chunk) {
        case 256: return dispatch_kind<ST, 256>(kind, bl, args, stream);
        case 512: return dispatch_kind<ST, 512>(kind, bl, args, stream);
        case 1024: return dispatch_kind<ST, 1024>(kind, bl, args, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t dispatch_batched(int32_t storage, int32_t chunk, int32_t kind, const BatchedLaunch& bl,
                            const pw_domain_args* args, hipStream_t stream) {
    switch (storage) {
        case PW_F64: return dispatch_chunk<double>(chunk, kind, bl, args, stream);
        case PW_F32: return dispatch_chunk<float>(chunk, kind, bl, args, stream);
        case PW_BF16: return dispatch_chunk<bf16_t>(chunk, kind, bl, args, stream);
        case PW_F16: return dispatch_chunk<f16_t>(chunk, kind, bl, args, stream);
        case PW_I16: return dispatch_chunk<fx16_t>(chunk, kind, bl, args, stream);
        case PW_I32: return dispatch_chunk<fx32_t>(chunk, kind, bl, args, stream);
        default: return hipErrorInvalidValue;
    }
}

// Workgroups per domain of the halo fill: the mean domain's halo in blocks
// of 256 elements (larger domains loop), at most the largest domain's.
int64_t halo_blocks(const pw_plan* p) {
    int64_t m = 0, sum = 0;
    for (const pw_shape& s : p->shapes) {
        const int64_t e = (int64_t)(2 * (s.nx + 2) + 2 * s.ny) * s.nz;
        m = std::max<int64_t>(m, e);
        sum += e;
    }
    const int64_t mean = sum / std::max<int64_t>(1, (int64_t)p->shapes.size());
    return std::max<int64_t>(1, std::min((m + 255) / 256, (mean + 255) / 256));
}

}  // namespace

// Tile split of one domain: nchunks chunks of `chunk` points per plane, x
// range split into nseg segments of even length (at most seg_max planes:
// nseg = ceil(nx / seg_max) parts of ceil(nx / nseg) planes, which start at or
// before plane nx and cover every plane).
__host__ __device__ inline void domain_tiles(int32_t nx, int32_t ny, int32_t nz, int32_t chunk, int32_t seg_max,
                                             BatchDomain* b) {
    b->nx = nx;
    b->ny = ny;
    b->nz = nz;
    b->nchunks = (int32_t)(((int64_t)ny * nz + chunk - 1) / chunk);
    b->nseg = (nx + seg_max - 1) / seg_max;
    b->seg = (nx + b->nseg - 1) / b->nseg;
}

// Launch shape of the batched kernel for a list of (normalised) shapes:
// chunk, segment bound, LDS, code-path kind, total tiles and grid.  Allocates
// nothing.  Returns PW_OK with L->tiles == 0 if a shape cannot use the
// batched kernel (march variant impossible, or 2^31 points or more).
int32_t batched_launch_shape(int32_t storage, const pw_shape* shapes, int32_t n, const pw_tuning& t, Launch* L,
                             int32_t* kind, bool* vec_out) {
    *L = Launch{};
    for (int32_t d = 0; d < n; ++d) {
        pw_shape s;
        const int32_t rc = normalize_shape(shapes[d], &s);
        if (rc != PW_OK) return rc;
        if (!march_possible(s) || (int64_t)s.nx * s.ny * s.nz >= (int64_t(1) << 31)) return PW_OK;
    }
    const int32_t chunk = t.chunk ? t.chunk : 512;
    if (chunk != 256 && chunk != 512 && chunk != 1024) return PW_ERR_INVALID_ARG;
    if (t.seg < 0 || t.wg_per_cu < PW_WG_ONE_PER_TILE || t.wg_per_cu > 8) return PW_ERR_INVALID_ARG;
    // default segment length: short tiles balance the uneven domains of a
    // batch for the 4- and 8-byte types; the 16-bit types, with more
    // arithmetic per byte, gain from longer marches (measured on the
    // 384-domain batch: FP64 and FP32 fastest at 12-16 planes, BF16 at 48+)
    const int32_t seg_max = t.seg ? t.seg : (elem_bytes(storage) >= 4 ? 16 : 64);
    const int64_t vw = 16 / elem_bytes(storage);
    int32_t nzmax = 0;
    int64_t tiles = 0;
    bool vec = true, fixed_nz = true;
    for (int32_t d = 0; d < n; ++d) {
        pw_shape s;
        (void)normalize_shape(shapes[d], &s);   // checked above
        BatchDomain b{};
        domain_tiles(s.nx, s.ny, s.nz, chunk, seg_max, &b);
        tiles += (int64_t)b.nchunks * b.nseg;
        nzmax = std::max(nzmax, s.nz);
        if (s.nz % vw || s.sx % vw || s.sy % vw) vec = false;
        fixed_nz = fixed_nz && (s.nz == 64 || s.nz == 96 || s.nz == 128);
    }
    Launch r{};
    r.variant = PW_VARIANT_MARCH;
    r.chunk = chunk;
    r.seg = seg_max;
    r.block = 256;
    r.wpad = ((chunk + 2 * nzmax) + 3) / 4 * 4;
    r.lds_bytes = march_lds_bytes(storage, r.wpad);
    if (r.lds_bytes > kMaxDynamicLds) return PW_ERR_UNSUPPORTED;
    r.tiles = tiles;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return report_hip(e);
    const int32_t k = !vec ? kAny : (fixed_nz ? kFixedNz : kVector);
    const int64_t by_lds = std::max<int64_t>(1, kLdsPerCu / std::max<int64_t>(r.lds_bytes, 1));
    int64_t per_cu = std::min<int64_t>(by_lds, 8);
    const int occ = batched_occupancy(storage, chunk, k, r.lds_bytes);
    if (occ > 0) per_cu = std::min<int64_t>(per_cu, occ);
    if (t.wg_per_cu > 0) per_cu = std::min<int64_t>(per_cu, t.wg_per_cu);
    r.workgroups = std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)cus * per_cu));
    // One workgroup per tile: the kernel's tile loop then runs once per
    // workgroup, and the hardware dispatches tiles in order as workgroups
    // retire, so the workgroups on neighbouring chunks stay in step (their
    // shared halo columns meet in L2) where a persistent grid's fixed
    // round-robin shares drift apart.  Measured on the 384-domain batch: 2-3%
    // faster than the best persistent grid for FP64, FP32 and BF16, and 11-18%
    // faster than a persistent grid at full occupancy; hence the default.
    if (batched_one_per_tile(t)) {
        constexpr int64_t block = (int64_t)kNumXcd * kOneTileRuns;   // padded to whole blocks (kernel comment)
        const int64_t g = (tiles + block - 1) / block * block;
        if (g >= (int64_t(1) << 31)) return PW_ERR_UNSUPPORTED;
        r.workgroups = g;
    }
    *L = r;
    *kind = k;
    *vec_out = vec;
    return PW_OK;
}

// Dispatch order of a plan's one-workgroup-per-tile launch.  Each domain's
// chunks form groups of kOneTileRuns neighbours (they share y-halo columns),
// and every segment of a group runs on one XCD; the groups are spread over
// the XCDs by their points, the longest tiles first.  An XCD's queue takes
// its groups in windows of about as many tiles as the XCD keeps resident
// and runs segment 0 of every group of the window, then segment 1, and so on
// -- the march kernel's compact order within each window -- so the tile of
// segment s + 1 of a group starts as the window's segment-s tiles retire and
// finds the planes they share still in the XCD's L2.  Workgroups go
// round-robin over the XCDs: order[k * 8 + x] is the tile of the k-th
// workgroup of XCD x, -1 past the end of that XCD's queue.
std::vector<int32_t> one_tile_order(const std::vector<BatchDomain>& table, int32_t chunk, int64_t resident_per_xcd) {
    struct Group {
        int d, c0, c1;
    };
    std::vector<std::vector<Group>> groups(kNumXcd);
    std::vector<int64_t> load(kNumXcd, 0);
    for (int d = 0; d < (int)table.size(); ++d) {
        const BatchDomain& b = table[d];
        for (int c0 = 0; c0 < b.nchunks; c0 += kOneTileRuns) {
            const int c1 = std::min(b.nchunks, c0 + kOneTileRuns);
            const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            groups[x].push_back(Group{d, c0, c1});
            load[x] += (int64_t)(c1 - c0) * chunk * b.nx;
        }
    }
    const size_t window = (size_t)std::max<int64_t>(1, resident_per_xcd / kOneTileRuns);   // groups in flight
    std::vector<std::vector<int32_t>> queue(kNumXcd);
    for (int x = 0; x < kNumXcd; ++x) {
        const std::vector<Group>& gs = groups[x];
        for (size_t w0 = 0; w0 < gs.size(); w0 += window) {
            const size_t w1 = std::min(gs.size(), w0 + window);
            int nseg = 0;
            for (size_t i = w0; i < w1; ++i) nseg = std::max(nseg, table[gs[i].d].nseg);
            for (int sg = 0; sg < nseg; ++sg)
                for (size_t i = w0; i < w1; ++i) {
                    const BatchDomain& b = table[gs[i].d];
                    if (sg >= b.nseg) continue;
                    for (int c = gs[i].c0; c < gs[i].c1; ++c)
                        queue[x].push_back((int32_t)(b.tile_begin + (int64_t)sg * b.nchunks + c));
                }
        }
    }
    size_t len = 0;
    for (const std::vector<int32_t>& q : queue) len = std::max(len, q.size());
    std::vector<int32_t> order(len * kNumXcd, -1);
    for (int x = 0; x < kNumXcd; ++x)
        for (size_t k = 0; k < queue[x].size(); ++k) order[k * kNumXcd + x] = queue[x][k];
    return order;
}

int32_t batched_plan_init(pw_plan* p) {
    BatchState& B = p->batch;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(nullptr, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return PW_ERR_CAPTURE;
    Launch L{};
    int32_t kind = kAny;
    bool vec = false;
    int32_t rc = batched_launch_shape(p->storage, p->shapes.data(), p->ndomains, p->tuning, &L, &kind, &vec);
    if (rc != PW_OK) return rc;
    if (L.tiles == 0) return PW_OK;   // batched entry points will report PW_ERR_UNSUPPORTED

    std::vector<BatchDomain> rows(p->ndomains);
    for (int32_t d = 0; d < p->ndomains; ++d) {
        const pw_shape& s = p->shapes[d];
        BatchDomain& b = rows[d];
        domain_tiles(s.nx, s.ny, s.nz, L.chunk, L.seg, &b);
        b.sy = s.sy;
        b.sx = s.sx;
        b.rec = d;
    }
    // One workgroup per tile: longest tiles first (stable: equal lengths keep
    // the caller's order), so long tiles start early and short ones fill the
    // end.  A persistent grid keeps the caller's order: its XCDs walk
    // contiguous shares of the list, which a sorted list would leave
    // unbalanced (measured 9-16% slower on the 384-domain batch).
    if (batched_one_per_tile(p->tuning))
        std::stable_sort(rows.begin(), rows.end(),
                         [](const BatchDomain& x, const BatchDomain& y) { return x.seg > y.seg; });
    std::vector<BatchDomain>& table = rows;
    int64_t tiles = 0;
    for (BatchDomain& b : table) {
        b.tile_begin = tiles;
        tiles += (int64_t)b.nchunks * b.nseg;
    }
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return report_hip(e);
    std::vector<int32_t> order;
    // The grouped order (one_tile_order) measured 6-11% faster than runs of
    // kOneTileRuns for BF16 and FP16 batches, whose kernels are bound by
    // instruction issue and gain from the L2 hits; 4-7% slower for FP64 and
    // FP32, bound by HBM, which gain more from all XCDs streaming neighbouring
    // tiles of the list at once, and 0.5-1% slower for int16.  So only BF16
    // and FP16 use it.
    if (batched_one_per_tile(p->tuning) && (p->storage == PW_BF16 || p->storage == PW_F16) &&
        tiles < (int64_t(1) << 31)) {
        // workgroups one XCD keeps resident: its CUs times the occupancy
        const int64_t by_lds = std::max<int64_t>(1, kLdsPerCu / std::max<int64_t>(L.lds_bytes, 1));
        int64_t per_cu = std::min<int64_t>(by_lds, 8);
        const int occ = batched_occupancy(p->storage, L.chunk, kind, L.lds_bytes);
        if (occ > 0) per_cu = std::min<int64_t>(per_cu, occ);
        order = one_tile_order(table, L.chunk, std::max<int64_t>(1, cus / kNumXcd) * per_cu);
        if ((int64_t)order.size() >= (int64_t(1) << 31)) order.clear();
        if (!order.empty()) L.workgroups = (int64_t)order.size();
    }
    void* mem = nullptr;
    const size_t tbytes = sizeof(BatchDomain) * table.size();
    // one allocation: the tile table, the error count, then the dispatch order
    const size_t off_err = (tbytes + 63) / 64 * 64;
    const size_t off_order = off_err + 64;
    e = hipMalloc(&mem, off_order + sizeof(int32_t) * order.size());
    if (e == hipErrorOutOfMemory) return PW_ERR_OUT_OF_MEMORY;
    if (e != hipSuccess) return report_hip(e);
    B.d_table = static_cast<BatchDomain*>(mem);
    B.d_errors = reinterpret_cast<unsigned long long*>(static_cast<char*>(mem) + off_err);
    B.d_order = order.empty() ? nullptr : reinterpret_cast<const int32_t*>(static_cast<char*>(mem) + off_order);
    e = hipMemcpy(B.d_table, table.data(), tbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess && !order.empty())
        e = hipMemcpy(static_cast<char*>(mem) + off_order, order.data(), sizeof(int32_t) * order.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(B.d_errors, 0, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);   // zeroed before any launch on another stream
    if (e != hipSuccess) {
        (void)hipFree(mem);
        B.d_table = nullptr;
        B.d_errors = nullptr;
        B.d_order = nullptr;
        return report_hip(e);
    }
    B.launch = L;
    B.device = dev;
    B.vec_shapes = vec;
    B.kind = kind;
    return PW_OK;
}

int32_t batched_plan_free(pw_plan* p) {
    if (p->batch.d_table) {
        hipError_t e = hipFree(p->batch.d_table);
        p->batch.d_table = nullptr;
        p->batch.d_errors = nullptr;
        p->batch.d_order = nullptr;
        if (e != hipSuccess) return report_hip(e);
    }
    return PW_OK;
}

}  // namespace pw

using namespace pw;

extern "C" {

int32_t pw_advect_batched(const pw_plan* plan, int32_t ndomains, const pw_domain_args* d_args, void* stream) {
    if (!plan || !d_args) return PW_ERR_INVALID_ARG;
    if (ndomains != plan->ndomains) return PW_ERR_PLAN_MISMATCH;
    if (!plan->batch.d_table) return PW_ERR_UNSUPPORTED;
    if (elem_bytes(plan->storage) == 0) return PW_ERR_UNSUPPORTED;
    const BatchState& B = plan->batch;
    const BatchedLaunch bl{B.d_table, plan->ndomains, B.launch.tiles, B.launch.workgroups, B.launch.lds_bytes,
                           B.d_errors, nullptr, B.vec_shapes, batched_one_per_tile(plan->tuning),
                           B.d_order};
    hipError_t e = dispatch_batched(plan->storage, B.launch.chunk, B.kind, bl, d_args, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return report_hip(e);
    return PW_OK;
}

int32_t pw_fill_halo_batched(const pw_plan* plan, int32_t ndomains, const pw_domain_args* d_args, void* stream) {
    if (!plan || !d_args) return PW_ERR_INVALID_ARG;
    if (ndomains != plan->ndomains) return PW_ERR_PLAN_MISMATCH;
    if (!plan->batch.d_table) return PW_ERR_UNSUPPORTED;
    dim3 grid((unsigned)halo_blocks(plan), (unsigned)ndomains);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const BatchDomain* tb = plan->batch.d_table;
    switch (plan->storage) {
        case PW_F64: hipLaunchKernelGGL(pw_halo_kernel<double>, grid, dim3(256), 0, s, tb, d_args); break;
        case PW_F32: hipLaunchKernelGGL(pw_halo_kernel<float>, grid, dim3(256), 0, s, tb, d_args); break;
        case PW_BF16: hipLaunchKernelGGL(pw_halo_kernel<bf16_t>, grid, dim3(256), 0, s, tb, d_args); break;
        case PW_F16: hipLaunchKernelGGL(pw_halo_kernel<f16_t>, grid, dim3(256), 0, s, tb, d_args); break;
        case PW_I16: hipLaunchKernelGGL(pw_halo_kernel<fx16_t>, grid, dim3(256), 0, s, tb, d_args); break;
        case PW_I32: hipLaunchKernelGGL(pw_halo_kernel<fx32_t>, grid, dim3(256), 0, s, tb, d_args); break;
        default: return PW_ERR_UNSUPPORTED;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return report_hip(e);
    return PW_OK;
}

int32_t pw_perturb_batched(const pw_plan* plan, int32_t ndomains, const pw_domain_args* d_args, uint64_t seed,
                           unsigned long long* d_call, double amplitude, void* stream) {
    if (!plan || !d_args || !d_call || !std::isfinite(amplitude)) return PW_ERR_INVALID_ARG;
    if (ndomains != plan->ndomains) return PW_ERR_PLAN_MISMATCH;
    if (!plan->batch.d_table) return PW_ERR_UNSUPPORTED;
    const Launch& L = plan->batch.launch;
    if (L.tiles >= (int64_t(1) << 31)) return PW_ERR_UNSUPPORTED;
    const dim3 grid((unsigned)L.tiles);   // one workgroup per tile
    hipStream_t s = static_cast<hipStream_t>(stream);
    const BatchDomain* tb = plan->batch.d_table;
    const int nd = plan->ndomains, ch = L.chunk;
    switch (plan->storage) {
        case PW_F64:
            hipLaunchKernelGGL(pw_perturb_kernel<double>, grid, dim3(256), 0, s, tb, nd, ch, d_args, seed, d_call, amplitude);
            break;
        case PW_F32:
            hipLaunchKernelGGL(pw_perturb_kernel<float>, grid, dim3(256), 0, s, tb, nd, ch, d_args, seed, d_call, amplitude);
            break;
        case PW_BF16:
            hipLaunchKernelGGL(pw_perturb_kernel<bf16_t>, grid, dim3(256), 0, s, tb, nd, ch, d_args, seed, d_call, amplitude);
            break;
        case PW_F16:
            hipLaunchKernelGGL(pw_perturb_kernel<f16_t>, grid, dim3(256), 0, s, tb, nd, ch, d_args, seed, d_call, amplitude);
            break;
        case PW_I16:
            hipLaunchKernelGGL(pw_perturb_kernel<fx16_t>, grid, dim3(256), 0, s, tb, nd, ch, d_args, seed, d_call, amplitude);
            break;
        case PW_I32:
            hipLaunchKernelGGL(pw_perturb_kernel<fx32_t>, grid, dim3(256), 0, s, tb, nd, ch, d_args, seed, d_call, amplitude);
            break;
        default: return PW_ERR_UNSUPPORTED;
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(pw_bump_kernel, dim3(1), dim3(1), 0, s, d_call);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return report_hip(e);
    return PW_OK;
}

int32_t pw_plan_error_count(const pw_plan* plan, unsigned long long* count) {
    if (!plan || !count) return PW_ERR_INVALID_ARG;
    *count = 0;
    if (!plan->batch.d_errors) return PW_OK;
    hipError_t e = hipMemcpy(count, plan->batch.d_errors, sizeof(unsigned long long), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return report_hip(e);
    return PW_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free batched call.  The tile table and the error word live in
// `scratch`, one array per GPU (file scope, allocated with the code object);
// a small kernel builds the table from the device records on every call.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace pw {
namespace {

constexpr int kNoAllocMaxDomains = 4096;
constexpr int kNoAllocHeader = 64;   // gate word, tile count, error word
constexpr size_t kNoAllocScratchBytes = kNoAllocHeader + sizeof(BatchDomain) * kNoAllocMaxDomains;   // 229,440 B
static_assert(kNoAllocScratchBytes == 229440, "scratch size stated in the header");
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

struct ScratchSlot {
    std::once_flag once;
    hipError_t err = hipSuccess;
    unsigned char* ptr = nullptr;   // device address of this GPU's scratch
};
ScratchSlot g_scratch[kMaxDevices];

// Device address of the current GPU's `scratch`, looked up once per device
// (with that device current).  The host-side symbol is only a stand-in for
// the device array and must never be passed to a kernel or a copy.
int32_t scratch_of_current_device(unsigned char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return report_hip(e);
    if (dev < 0 || dev >= kMaxDevices) return PW_ERR_UNSUPPORTED;
    ScratchSlot& sl = g_scratch[dev];
    std::call_once(sl.once, [&] {
        void* p = nullptr;
        sl.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        sl.ptr = static_cast<unsigned char*>(p);
    });
    if (sl.err != hipSuccess) return report_hip(sl.err);
    if (!sl.ptr) return PW_ERR_HIP;
    *out = sl.ptr;
    return PW_OK;
}

// One term of the shape digest: a hash of (domain index, normalised shape).
// The digest of a batch is the sum of its terms (mod 2^64), so the device can
// form it with a parallel reduction and compare it with the host's.
__host__ __device__ inline uint64_t shape_digest_term(int32_t d, int32_t nx, int32_t ny, int32_t nz, int32_t reserved,
                                                      int64_t sy, int64_t sx) {
    uint64_t h = splitmix64(((uint64_t)(uint32_t)d << 32) ^ (uint64_t)(uint32_t)nx);
    h = splitmix64(h ^ (uint64_t)(uint32_t)ny);
    h = splitmix64(h ^ ((uint64_t)(uint32_t)nz | ((uint64_t)(uint32_t)reserved << 32)));
    h = splitmix64(h ^ (uint64_t)sy);
    return splitmix64(h ^ (uint64_t)sx);
}

constexpr int kTableThreads = 1024;
constexpr int kTablePerThread = kNoAllocMaxDomains / kTableThreads;

// Table row of domain d from its record (an empty row if the shape is out of
// range: the digest of such a batch cannot match a valid one).
__device__ __forceinline__ BatchDomain record_row(const pw_domain_args* args, int d, int chunk, int seg_max,
                                                  uint64_t* term) {
    const pw_shape s = args[d].shape;
    const int64_t sy = s.sy ? s.sy : s.nz;
    const int64_t sx = s.sx ? s.sx : (int64_t)(s.ny + 2) * sy;
    *term = shape_digest_term(d, s.nx, s.ny, s.nz, s.reserved, sy, sx);
    BatchDomain b{};
    if (s.nx >= 1 && s.ny >= 1 && s.nz >= 2 && s.nx <= (1 << 30) && (int64_t)s.ny * s.nz < (int64_t(1) << 31))
        domain_tiles(s.nx, s.ny, s.nz, chunk, seg_max, &b);
    b.sy = sy;
    b.sx = sx;
    return b;
}

// Builds the tile table of a batch from its device records into scratch (one
// workgroup): thread t takes domains 4t .. 4t+3, a workgroup scan of the
// per-thread tile counts gives every domain its first tile, and a reduction
// forms the shape digest.  The gate word is set only if the digest and the
// tile total equal the host's, i.e. the records carry the shapes the launch
// was shaped for.  The error word is cleared.
__global__ __launch_bounds__(kTableThreads) void pw_noalloc_table_kernel(const pw_domain_args* __restrict__ args,
                                                                         int ndom, int chunk, int seg_max,
                                                                         uint64_t digest_host, int64_t tiles_host,
                                                                         unsigned char* scr) {
    __shared__ int64_t part[kTableThreads];
    __shared__ uint64_t hsum[kTableThreads];
    BatchDomain* table = reinterpret_cast<BatchDomain*>(scr + kNoAllocHeader);
    const int t = (int)threadIdx.x;
    int64_t mine = 0;
    uint64_t h = 0;
    for (int q = 0; q < kTablePerThread; ++q) {
        const int d = t * kTablePerThread + q;
        if (d < ndom) {
            uint64_t term;
            const BatchDomain b = record_row(args, d, chunk, seg_max, &term);
            h += term;
            mine += (int64_t)b.nchunks * b.nseg;
        }
    }
    part[t] = mine;
    hsum[t] = h;
    __syncthreads();
    // inclusive scan of the tile counts (Hillis-Steele) and tree reduction of
    // the digest terms into hsum[0]
    for (int off = 1; off < kTableThreads; off <<= 1) {
        const int64_t a = t >= off ? part[t - off] : 0;
        const uint64_t g = (t & (2 * off - 1)) == 0 ? hsum[t + off] : 0;
        __syncthreads();
        part[t] += a;
        hsum[t] += g;
        __syncthreads();
    }
    int64_t first = part[t] - mine;
    for (int q = 0; q < kTablePerThread; ++q) {
        const int d = t * kTablePerThread + q;
        if (d < ndom) {
            uint64_t term;
            BatchDomain b = record_row(args, d, chunk, seg_max, &term);
            b.rec = d;   // the caller's order (no reordering on the device)
            b.tile_begin = first;
            first += (int64_t)b.nchunks * b.nseg;
            table[d] = b;
        }
    }
    if (t == 0) {
        const bool ok = hsum[0] == digest_host && part[kTableThreads - 1] == tiles_host;
        *reinterpret_cast<int64_t*>(scr + 8) = part[kTableThreads - 1];
        *reinterpret_cast<unsigned long long*>(scr + 16) = 0ull;
        *reinterpret_cast<uint32_t*>(scr) = ok ? 1u : 0u;
    }
}

}  // namespace
}  // namespace pw

extern "C" {

int32_t pw_advect_batched_noalloc(int32_t storage, const pw_shape* shapes, int32_t ndomains,
                                  const pw_domain_args* d_args, const pw_tuning* tuning,
                                  unsigned long long* d_skipped, void* stream) {
    if (!shapes || !d_args || ndomains < 1) return PW_ERR_INVALID_ARG;
    if (ndomains > kNoAllocMaxDomains) return PW_ERR_INVALID_ARG;
    if (elem_bytes(storage) == 0) return PW_ERR_UNSUPPORTED;
    const pw_tuning t = tuning ? *tuning : pw_tuning{};
    if (t.variant != PW_VARIANT_AUTO && t.variant != PW_VARIANT_MARCH) return PW_ERR_UNSUPPORTED;
    // digest of the normalised shapes, then the launch shape; nothing here allocates
    uint64_t digest = 0;
    for (int32_t d = 0; d < ndomains; ++d) {
        pw_shape s;
        int32_t rc = normalize_shape(shapes[d], &s);
        if (rc != PW_OK) return rc;
        digest += shape_digest_term(d, s.nx, s.ny, s.nz, s.reserved, s.sy, s.sx);
    }
    Launch L{};
    int32_t kind = 0;
    bool vec = false;
    int32_t rc = batched_launch_shape(storage, shapes, ndomains, t, &L, &kind, &vec);
    if (rc != PW_OK) return rc;
    if (L.tiles == 0) return PW_ERR_UNSUPPORTED;
    unsigned char* scr = nullptr;
    rc = scratch_of_current_device(&scr);
    if (rc != PW_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(pw_noalloc_table_kernel, dim3(1), dim3(kTableThreads), 0, st, d_args, ndomains, L.chunk,
                       L.seg, digest, L.tiles, scr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return report_hip(e);
    unsigned long long* errors = d_skipped ? d_skipped : reinterpret_cast<unsigned long long*>(scr + 16);
    const BatchedLaunch bl{reinterpret_cast<const BatchDomain*>(scr + kNoAllocHeader), ndomains, L.tiles,
                           L.workgroups, L.lds_bytes, errors, reinterpret_cast<const uint32_t*>(scr), vec,
                           batched_one_per_tile(t), nullptr};
    e = dispatch_batched(storage, L.chunk, kind, bl, d_args, st);
    if (e != hipSuccess) return report_hip(e);
    return PW_OK;
}

}  // extern "C"
