// HBM calibration probe: a plain streaming copy of 1..3 buffers with the same
// access width (16-byte loads, non-temporal 16-byte stores) as the stencil
// kernels.  It moves a known number of bytes, so its time gives the
// attainable read+write bandwidth of the card and its profiler counters give
// the scale factor between the counters and true bytes.
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
    int64_t n16;   // 16-byte words per buffer
};

template <int NS, int UNROLL>
__global__ __launch_bounds__(256) void pw_probe_copy_kernel(ProbeArgs a) {
    const int64_t stride = (int64_t)gridDim.x * 256 * UNROLL;
    for (int64_t base = (int64_t)blockIdx.x * 256 * UNROLL + threadIdx.x; base < a.n16; base += stride) {
        u32x4 r[NS][UNROLL];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const int64_t q = base + (int64_t)u * 256;
                if (q < a.n16) r[s][u] = a.src[s][q];
            }
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const int64_t q = base + (int64_t)u * 256;
                if (q < a.n16) __builtin_nontemporal_store(r[s][u], a.dst[s] + q);
            }
    }
}

}  // namespace
}  // namespace pw

using namespace pw;

extern "C" int32_t pw_probe_copy(const void* const* src, void* const* dst, int32_t nstreams, int64_t bytes,
                                 int32_t workgroups, void* stream) {
    if (!src || !dst || nstreams < 1 || nstreams > 3 || bytes <= 0 || bytes % 16 || workgroups < 0)
        return PW_ERR_INVALID_ARG;
    ProbeArgs a{};
    for (int s = 0; s < nstreams; ++s) {
        if (!src[s] || !dst[s]) return PW_ERR_INVALID_ARG;
        if (reinterpret_cast<uintptr_t>(src[s]) % 16 || reinterpret_cast<uintptr_t>(dst[s]) % 16)
            return PW_ERR_ALIGNMENT;
        a.src[s] = static_cast<const u32x4*>(src[s]);
        a.dst[s] = static_cast<u32x4*>(dst[s]);
    }
    a.n16 = bytes / 16;
    constexpr int UNROLL = 4;
    const int64_t need = (a.n16 + 256 * UNROLL - 1) / (256 * UNROLL);
    int64_t grid = workgroups > 0 ? workgroups : std::min<int64_t>(need, 256 * 16);
    grid = std::max<int64_t>(1, std::min<int64_t>(grid, need));
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (nstreams) {
        case 1: hipLaunchKernelGGL((pw_probe_copy_kernel<1, UNROLL>), dim3((unsigned)grid), dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL((pw_probe_copy_kernel<2, UNROLL>), dim3((unsigned)grid), dim3(256), 0, s, a); break;
        default: hipLaunchKernelGGL((pw_probe_copy_kernel<3, UNROLL>), dim3((unsigned)grid), dim3(256), 0, s, a); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return report_hip(e);
    return PW_OK;
}
