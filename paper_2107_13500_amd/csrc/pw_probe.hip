// HBM calibration probes: plain streaming reads, writes and copies over
// 0..3 source and 0..3 destination buffers with 16-byte accesses (the
// stencil kernels' width).  They move a known number of bytes, so their
// times give the attainable read-only, write-only and mixed read+write
// bandwidth of the card, and their profiler counters give the scale factor
// between the counters and true bytes.
//
// The main loop covers whole blocks of 256 x U words per buffer and carries
// no per-lane condition, so the compiler waits for each load only where its
// value is used (a guarded load or store would make it wait for every
// outstanding memory operation).  The ragged tail is one guarded block run
// by the last workgroup after its main loop.  Variants (flags): loads plain
// or non-temporal, stores non-temporal or plain, one or four words per lane
// and buffer; with one word and one block per workgroup (the fastest mixed
// read+write form measured on MI355X) each workgroup moves one 4 KiB block
// of every buffer and exits.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pw_advect.h"
#include "pw_plan.hpp"

namespace pw {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct ProbeArgs {
    const u32x4* src[3];
    u32x4* dst[3];
    u32x4* sink;   // read-only probes: one word per workgroup, written only if the XOR of all loads hits a marker
    int64_t n16;   // 16-byte words per buffer
};

// One block of U words per lane and buffer at word `base` (+ u * 256).
template <int NIN, int NOUT, int U, bool NTL, bool TS, bool GUARD>
__device__ __forceinline__ void probe_block(const ProbeArgs& a, int64_t base, u32x4& acc) {
    u32x4 r[NIN > 0 ? NIN : 1][U];
    if constexpr (NIN > 0) {
#pragma unroll
        for (int s = 0; s < NIN; ++s)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = base + (int64_t)u * 256;
                if (!GUARD || q < a.n16) {
                    if constexpr (NTL) r[s][u] = __builtin_nontemporal_load(a.src[s] + q);
                    else r[s][u] = a.src[s][q];
                }
            }
    }
    if constexpr (NOUT > 0) {
#pragma unroll
        for (int s = 0; s < NOUT; ++s)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = base + (int64_t)u * 256;
                u32x4 val;
                if constexpr (NIN > 0) {
                    val = r[s % NIN][u];
                } else {
                    val = u32x4{(unsigned)q, (unsigned)(q >> 32), (unsigned)s, 0u};
                }
                if (!GUARD || q < a.n16) {
                    if constexpr (TS) a.dst[s][q] = val;
                    else __builtin_nontemporal_store(val, a.dst[s] + q);
                }
            }
    } else {
#pragma unroll
        for (int s = 0; s < NIN; ++s)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = base + (int64_t)u * 256;
                if (!GUARD || q < a.n16) acc ^= r[s][u];
            }
    }
}

template <int NIN, int NOUT, int U, bool NTL, bool TS>
__global__ __launch_bounds__(256) void pw_probe_kernel(ProbeArgs a) {
    constexpr int64_t W = 256 * U;
    const int64_t nblk = a.n16 / W;
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x)
        probe_block<NIN, NOUT, U, NTL, TS, false>(a, b * W + threadIdx.x, acc);
    if (blockIdx.x == gridDim.x - 1 && nblk * W < a.n16)
        probe_block<NIN, NOUT, U, NTL, TS, true>(a, nblk * W + threadIdx.x, acc);
    if constexpr (NOUT == 0) {
        // keeps the loads alive; the marker is not a XOR of the probe's data
        if (acc.x == 0x9e3779b9u && acc.y == 0x7f4a7c15u && acc.z == 0xbf58476du && acc.w == 0x1ce4e5b9u)
            a.sink[blockIdx.x] = acc;
    }
}

template <int NIN, int NOUT, int U, bool NTL, bool TS>
void launch_probe(const ProbeArgs& a, int64_t grid, hipStream_t s) {
    hipLaunchKernelGGL((pw_probe_kernel<NIN, NOUT, U, NTL, TS>), dim3((unsigned)grid), dim3(256), 0, s, a);
}

template <int NIN, int NOUT>
void launch_probe_flags(const ProbeArgs& a, int32_t flags, int64_t grid, hipStream_t s) {
    const bool ntl = flags & PW_PROBE_NT_LOADS, ts = flags & PW_PROBE_CACHED_STORES;
    if (flags & PW_PROBE_UNROLL4) {
        if (ntl) ts ? launch_probe<NIN, NOUT, 4, true, true>(a, grid, s) : launch_probe<NIN, NOUT, 4, true, false>(a, grid, s);
        else ts ? launch_probe<NIN, NOUT, 4, false, true>(a, grid, s) : launch_probe<NIN, NOUT, 4, false, false>(a, grid, s);
    } else {
        if (ntl) ts ? launch_probe<NIN, NOUT, 1, true, true>(a, grid, s) : launch_probe<NIN, NOUT, 1, true, false>(a, grid, s);
        else ts ? launch_probe<NIN, NOUT, 1, false, true>(a, grid, s) : launch_probe<NIN, NOUT, 1, false, false>(a, grid, s);
    }
}

template <int NIN>
void launch_probe_in(const ProbeArgs& a, int32_t nout, int32_t flags, int64_t grid, hipStream_t s) {
    switch (nout) {
        case 0: launch_probe_flags<NIN, 0>(a, flags, grid, s); break;
        case 1: launch_probe_flags<NIN, 1>(a, flags, grid, s); break;
        case 2: launch_probe_flags<NIN, 2>(a, flags, grid, s); break;
        default: launch_probe_flags<NIN, 3>(a, flags, grid, s); break;
    }
}

}  // namespace
}  // namespace pw

using namespace pw;

extern "C" int32_t pw_probe_bandwidth(const void* const* src, int32_t nsrc, void* const* dst, int32_t ndst,
                                      int64_t bytes, int32_t workgroups, int32_t flags, void* sink, void* stream) {
    if (nsrc < 0 || nsrc > 3 || ndst < 0 || ndst > 3 || nsrc + ndst == 0) return PW_ERR_INVALID_ARG;
    if ((nsrc > 0 && !src) || (ndst > 0 && !dst) || bytes <= 0 || bytes % 16 || workgroups < 0)
        return PW_ERR_INVALID_ARG;
    if (flags & ~(PW_PROBE_NT_LOADS | PW_PROBE_CACHED_STORES | PW_PROBE_UNROLL4)) return PW_ERR_INVALID_ARG;
    if (ndst == 0 && !sink) return PW_ERR_INVALID_ARG;
    ProbeArgs a{};
    for (int s = 0; s < nsrc; ++s) {
        if (!src[s]) return PW_ERR_INVALID_ARG;
        if (reinterpret_cast<uintptr_t>(src[s]) % 16) return PW_ERR_ALIGNMENT;
        a.src[s] = static_cast<const u32x4*>(src[s]);
    }
    for (int s = 0; s < ndst; ++s) {
        if (!dst[s]) return PW_ERR_INVALID_ARG;
        if (reinterpret_cast<uintptr_t>(dst[s]) % 16) return PW_ERR_ALIGNMENT;
        a.dst[s] = static_cast<u32x4*>(dst[s]);
    }
    if (sink && reinterpret_cast<uintptr_t>(sink) % 16) return PW_ERR_ALIGNMENT;
    a.sink = static_cast<u32x4*>(sink);
    a.n16 = bytes / 16;
    const int64_t unroll = (flags & PW_PROBE_UNROLL4) ? 4 : 1;
    const int64_t need = std::max<int64_t>(1, (a.n16 + 256 * unroll - 1) / (256 * unroll));
    int64_t grid = workgroups > 0 ? std::min<int64_t>(workgroups, need) : need;
    if (grid >= (int64_t(1) << 31)) return PW_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (nsrc) {
        case 0: launch_probe_in<0>(a, ndst, flags, grid, s); break;
        case 1: launch_probe_in<1>(a, ndst, flags, grid, s); break;
        case 2: launch_probe_in<2>(a, ndst, flags, grid, s); break;
        default: launch_probe_in<3>(a, ndst, flags, grid, s); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return report_hip(e);
    return PW_OK;
}

extern "C" int32_t pw_probe_copy(const void* const* src, void* const* dst, int32_t nstreams, int64_t bytes,
                                 int32_t workgroups, void* stream) {
    if (!src || !dst || nstreams < 1 || nstreams > 3) return PW_ERR_INVALID_ARG;
    // four words per lane, grid-stride over the blocks (16 workgroups per CU by default)
    return pw_probe_bandwidth(src, nstreams, dst, nstreams, bytes, workgroups > 0 ? workgroups : 256 * 16,
                              PW_PROBE_UNROLL4, nullptr, stream);
}
