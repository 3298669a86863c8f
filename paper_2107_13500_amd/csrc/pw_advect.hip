// Host side of the C ABI in include/pw_advect.h: plans, argument checks and
// kernel dispatch.  No entry point except pw_advect_plan allocates, and none
// synchronises.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "pw_advect.h"
#include "pw_kernels.hpp"
#include "pw_plan.hpp"

namespace {

thread_local int32_t g_last_hip_error = 0;

int32_t hip_fail(hipError_t e) {
    g_last_hip_error = static_cast<int32_t>(e);
    return PW_ERR_HIP;
}

}  // namespace

namespace pw {

int64_t elem_bytes(int32_t storage) {
    switch (storage) {
        case PW_F64: return 8;
        case PW_F32:
        case PW_I32: return 4;
        case PW_BF16:
        case PW_F16:
        case PW_I16: return 2;
        default: return 0;
    }
}

int64_t compute_bytes(int32_t storage) { return storage == PW_F64 || storage == PW_I32 ? 8 : 4; }

// LDS of one march workgroup: three fields per ring slot (march_slots<CT>()).
int64_t march_lds_bytes(int32_t storage, int32_t wpad) {
    const int64_t slots = compute_bytes(storage) == 8 ? march_slots<double>() : march_slots<float>();
    return 3 * slots * (int64_t)wpad * compute_bytes(storage);
}

bool scaled_storage(int32_t storage) {
    return storage == PW_BF16 || storage == PW_F16 || storage == PW_I16 || storage == PW_I32;
}

int32_t normalize_shape(const pw_shape& in, pw_shape* out) {
    pw_shape s = in;
    if (s.nx < 1 || s.ny < 1 || s.nz < 2 || s.reserved != 0) return PW_ERR_INVALID_ARG;
    const int64_t nx = s.nx, ny = s.ny, nz = s.nz;
    // 32-bit in-plane indexing in the kernels; plane indices up to nx + 1
    if ((ny + 2) * nz >= (int64_t(1) << 31) || nx + 2 >= (int64_t(1) << 31)) return PW_ERR_INVALID_ARG;
    // strides: every element offset stays below 2^48 (far beyond any device
    // memory), so element and byte offsets never overflow 64 bits
    constexpr int64_t kMaxElems = int64_t(1) << 48;
    if (s.sy == 0) s.sy = nz;
    if (s.sy < nz || s.sy > kMaxElems / (ny + 2)) return PW_ERR_INVALID_ARG;
    if (s.sx == 0) s.sx = (ny + 2) * s.sy;
    if (s.sx < (ny + 2) * s.sy || s.sx > kMaxElems / (nx + 2)) return PW_ERR_INVALID_ARG;
    *out = s;
    return PW_OK;
}

int64_t extent_elems(const pw_shape& s) {
    return (int64_t)(s.nz - 1) + ((int64_t)s.ny + 1) * s.sy + ((int64_t)s.nx + 1) * s.sx + 1;
}

bool march_possible(const pw_shape& s) {
    return s.sy == s.nz && s.nz <= kMarchMaxNz && s.nx <= (1 << 30);
}

int32_t auto_seg(int32_t storage, const pw_shape& s, int32_t nchunks) {
    // Many tiles (the boundary planes each tile re-reads stay a few percent
    // of its traffic only with segments of 16 planes or more), all segments
    // of nearly equal length.  Measured with the compact tile order on
    // 512 x 512 x 64 and 2048 x 2048 x 64 over chunks 512/1024 and segments
    // of 16..256 planes for every storage type: 16 planes are best on the
    // small grid for all types; on the large grid FP64 and the 16-bit types
    // are best at about 8192 tiles (64 planes) and the 4-byte types at about
    // 2048 (256 planes), 0.5-1% ahead of 128 planes; an uneven split (such as
    // 192 planes over 2048) costs 7%.
    const int64_t target = elem_bytes(storage) == 4 ? 2048 : 8192;
    int64_t seg = (int64_t)s.nx * nchunks / target;
    seg = std::max<int64_t>(seg, 16);
    seg = std::min<int64_t>(seg, 256);
    seg = std::min<int64_t>(seg, s.nx);
    seg = std::max<int64_t>(seg, 1);
    const int64_t nseg = (s.nx + seg - 1) / seg;
    return (int32_t)((s.nx + nseg - 1) / nseg);
}

int32_t resolve_launch(int32_t storage, const pw_shape& s, const pw_tuning& t, Launch* L) {
    Launch r{};
    int32_t variant = t.variant;
    if (variant == PW_VARIANT_AUTO) variant = march_possible(s) ? PW_VARIANT_MARCH : PW_VARIANT_DIRECT;
    if (variant != PW_VARIANT_MARCH && variant != PW_VARIANT_DIRECT) return PW_ERR_UNSUPPORTED;
    if (variant == PW_VARIANT_MARCH && !march_possible(s)) return PW_ERR_UNSUPPORTED;
    r.variant = variant;
    if (variant == PW_VARIANT_MARCH) {
        const int32_t chunk = t.chunk ? t.chunk : 512;
        if (chunk != 256 && chunk != 512 && chunk != 1024) return PW_ERR_INVALID_ARG;
        if (t.seg < 0) return PW_ERR_INVALID_ARG;
        r.chunk = chunk;
        r.block = 256;
        r.nchunks = (int32_t)(((int64_t)s.ny * s.nz + chunk - 1) / chunk);
        r.seg = t.seg ? std::min(t.seg, s.nx) : auto_seg(storage, s, r.nchunks);
        r.nseg = (s.nx + r.seg - 1) / r.seg;
        r.wpad = ((chunk + 2 * s.nz) + 3) / 4 * 4;
        r.lds_bytes = march_lds_bytes(storage, r.wpad);
        if (r.lds_bytes > kMaxDynamicLds) return PW_ERR_UNSUPPORTED;
        r.tiles = (int64_t)r.nchunks * r.nseg;
        // compact tile order (pw_march_kernel) when every XCD owns a chunk
        r.cpx = r.nchunks >= kNumXcd ? (r.nchunks + kNumXcd - 1) / kNumXcd : 0;
        r.workgroups = r.cpx > 0 ? (int64_t)kNumXcd * r.cpx * r.nseg : r.tiles;
        if (r.workgroups >= (int64_t(1) << 31)) return PW_ERR_INVALID_ARG;
    } else {
        const int32_t block = t.block ? t.block : 256;
        if (block != 64 && block != 128 && block != 256 && block != 512) return PW_ERR_INVALID_ARG;
        if (s.nx > 65535) return PW_ERR_INVALID_ARG;   // x planes ride on grid.y
        r.block = block;
        r.chunk = 0;
        r.seg = 1;
        r.nchunks = (int32_t)(((int64_t)s.ny * s.nz + block - 1) / block);
        r.nseg = s.nx;
        r.workgroups = (int64_t)r.nchunks * s.nx;
        r.lds_bytes = 0;
        r.tiles = r.workgroups;
    }
    *L = r;
    return PW_OK;
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
template <typename ST, int P, bool VEC, int NZ>
hipError_t launch_march(const DomainArgs& d, const Launch& L, hipStream_t stream) {
    auto kern = pw_march_kernel<ST, 256, P, VEC, NZ>;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [&] {
        attr_err = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynamicLds);
    });
    if (attr_err != hipSuccess) return attr_err;
    MarchGeom g{L.nchunks, L.nseg, L.seg, L.wpad, L.cpx};
    hipLaunchKernelGGL(kern, dim3((unsigned)L.workgroups), dim3(256), (size_t)L.lds_bytes, stream, d, g);
    return hipGetLastError();
}

// Column heights 64 (the paper's and MONC's default), 96 and 128 get kernels
// with the height compiled in; other heights use the general one.
template <typename ST, bool VEC, int NZ>
hipError_t dispatch_march_p(const DomainArgs& d, const Launch& L, hipStream_t stream) {
    switch (L.chunk) {
        case 256: return launch_march<ST, 256, VEC, NZ>(d, L, stream);
        case 512: return launch_march<ST, 512, VEC, NZ>(d, L, stream);
        case 1024: return launch_march<ST, 1024, VEC, NZ>(d, L, stream);
        default: return hipErrorInvalidValue;
    }
}

template <typename ST>
hipError_t launch_direct(const DomainArgs& d, const Launch& L, hipStream_t stream) {
    dim3 grid((unsigned)L.nchunks, (unsigned)d.nx);
    switch (L.block) {
        case 64: hipLaunchKernelGGL((pw_direct_kernel<ST, 64>), grid, dim3(64), 0, stream, d); break;
        case 128: hipLaunchKernelGGL((pw_direct_kernel<ST, 128>), grid, dim3(128), 0, stream, d); break;
        case 256: hipLaunchKernelGGL((pw_direct_kernel<ST, 256>), grid, dim3(256), 0, stream, d); break;
        case 512: hipLaunchKernelGGL((pw_direct_kernel<ST, 512>), grid, dim3(512), 0, stream, d); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename ST>
hipError_t launch_typed(const DomainArgs& d, const Launch& L, bool vec, hipStream_t stream) {
    if (L.variant == PW_VARIANT_MARCH) {
        if (vec) {
            switch (d.nz) {
                case 64: return dispatch_march_p<ST, true, 64>(d, L, stream);
                case 96: return dispatch_march_p<ST, true, 96>(d, L, stream);
                case 128: return dispatch_march_p<ST, true, 128>(d, L, stream);
                default: return dispatch_march_p<ST, true, 0>(d, L, stream);
            }
        }
        return dispatch_march_p<ST, false, 0>(d, L, stream);
    }
    return launch_direct<ST>(d, L, stream);
}

hipError_t launch_domain(int32_t storage, const DomainArgs& d, const Launch& L, bool vec, hipStream_t stream) {
    switch (storage) {
        case PW_F64: return launch_typed<double>(d, L, vec, stream);
        case PW_F32: return launch_typed<float>(d, L, vec, stream);
        case PW_BF16: return launch_typed<bf16_t>(d, L, vec, stream);
        case PW_F16: return launch_typed<f16_t>(d, L, vec, stream);
        case PW_I16: return launch_typed<fx16_t>(d, L, vec, stream);
        case PW_I32: return launch_typed<fx32_t>(d, L, vec, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pw

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace pw;

extern "C" {

const char* pw_status_string(int32_t status) {
    switch (status) {
        case PW_OK: return "ok";
        case PW_ERR_INVALID_ARG: return "invalid argument";
        case PW_ERR_UNSUPPORTED: return "unsupported";
        case PW_ERR_ALIAS: return "an output overlaps an input or another output";
        case PW_ERR_ALIGNMENT: return "misaligned pointer";
        case PW_ERR_OUT_OF_MEMORY: return "out of device memory";
        case PW_ERR_HIP: return "HIP runtime error";
        case PW_ERR_CAPTURE: return "allocation requested during stream capture";
        case PW_ERR_PLAN_MISMATCH: return "arguments do not match the plan";
        default: return "unknown status";
    }
}

int32_t pw_last_hip_error(void) { return g_last_hip_error; }

int32_t pw_advect_plan(pw_plan** plan, int32_t storage, const pw_shape* shapes, int32_t ndomains,
                       const pw_tuning* tuning) {
    if (!plan || !shapes || ndomains < 1) return PW_ERR_INVALID_ARG;
    *plan = nullptr;
    if (elem_bytes(storage) == 0) return PW_ERR_UNSUPPORTED;
    pw_tuning t{};
    if (tuning) t = *tuning;
    std::unique_ptr<pw_plan> p(new (std::nothrow) pw_plan());
    if (!p) return PW_ERR_OUT_OF_MEMORY;
    p->storage = storage;
    p->ndomains = ndomains;
    p->tuning = t;
    p->shapes.resize(ndomains);
    for (int32_t d = 0; d < ndomains; ++d) {
        int32_t rc = normalize_shape(shapes[d], &p->shapes[d]);
        if (rc != PW_OK) return rc;
        p->points += (int64_t)p->shapes[d].nx * p->shapes[d].ny * p->shapes[d].nz;
    }
    if (ndomains == 1) {
        int32_t rc = resolve_launch(storage, p->shapes[0], t, &p->single);
        if (rc != PW_OK) return rc;
    }
    int32_t rc = batched_plan_init(p.get());
    if (rc != PW_OK) return rc;
    *plan = p.release();
    return PW_OK;
}

int32_t pw_plan_destroy(pw_plan* plan) {
    if (!plan) return PW_OK;
    int32_t rc = batched_plan_free(plan);
    delete plan;
    return rc;
}

int32_t pw_plan_get_info(const pw_plan* plan, pw_plan_info* info) {
    if (!plan || !info) return PW_ERR_INVALID_ARG;
    pw_plan_info r{};
    r.storage = plan->storage;
    r.ndomains = plan->ndomains;
    const Launch& L = plan->ndomains == 1 ? plan->single : plan->batch.launch;
    if (plan->ndomains == 1) {
        r.batched_workgroups = plan->batch.launch.workgroups;
    } else {
        r.batched_workgroups = L.workgroups;
    }
    r.variant = L.variant;
    r.chunk = L.chunk;
    r.seg = L.seg;
    r.block = L.block;
    r.workgroups = L.workgroups;
    r.tiles = L.tiles;
    r.lds_bytes = L.lds_bytes;
    r.points = plan->points;
    *info = r;
    return PW_OK;
}

int32_t pw_advect(const pw_plan* plan, const void* u, const void* v, const void* w, void* su, void* sv,
                  void* sw, double tcx, double tcy, const double* tzc1, const double* tzc2,
                  const double* tzd1, const double* tzd2, const pw_scales* scales, void* stream) {
    if (!plan) return PW_ERR_INVALID_ARG;
    if (plan->ndomains != 1) return PW_ERR_PLAN_MISMATCH;
    if (!u || !v || !w || !su || !sv || !sw || !tzc1 || !tzc2 || !tzd1 || !tzd2) return PW_ERR_INVALID_ARG;
    if (!std::isfinite(tcx) || !std::isfinite(tcy)) return PW_ERR_INVALID_ARG;
    const pw_shape& s = plan->shapes[0];
    const int64_t eb = elem_bytes(plan->storage);

    const void* ins[3] = {u, v, w};
    void* outs[3] = {su, sv, sw};
    for (const void* q : ins)
        if (reinterpret_cast<uintptr_t>(q) % eb) return PW_ERR_ALIGNMENT;
    for (const void* q : outs)
        if (reinterpret_cast<uintptr_t>(q) % eb) return PW_ERR_ALIGNMENT;
    for (const double* q : {tzc1, tzc2, tzd1, tzd2})
        if (reinterpret_cast<uintptr_t>(q) % 8) return PW_ERR_ALIGNMENT;
    const int64_t ext = extent_elems(s) * eb;
    if (any_overlap(ins, outs, ext)) return PW_ERR_ALIAS;

    DomainArgs d{};
    int32_t rc = fill_domain_args(plan->storage, s, u, v, w, su, sv, sw, tcx, tcy, tzc1, tzc2, tzd1, tzd2,
                                  scales, &d);
    if (rc != PW_OK) return rc;
    const bool vec = vector_ok(plan->storage, s, ins, outs);
    hipError_t e = launch_domain(plan->storage, d, plan->single, vec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e);
    return PW_OK;
}

}  // extern "C"

namespace pw {

int32_t report_hip(hipError_t e) { return hip_fail(e); }

bool any_overlap(const void* const ins[3], void* const outs[3], int64_t ext) {
    auto lo = [](const void* q) { return reinterpret_cast<uintptr_t>(q); };
    for (int a = 0; a < 3; ++a) {
        const uintptr_t oa = lo(outs[a]);
        for (int b = 0; b < 3; ++b) {
            const uintptr_t ib = lo(ins[b]);
            if (oa < ib + ext && ib < oa + ext) return true;
        }
        for (int b = a + 1; b < 3; ++b) {
            const uintptr_t ob = lo(outs[b]);
            if (oa < ob + ext && ob < oa + ext) return true;
        }
    }
    return false;
}

bool vector_ok(int32_t storage, const pw_shape& s, const void* const ins[3], void* const outs[3]) {
    const int64_t vw = 16 / elem_bytes(storage);
    if (s.nz % vw || s.sx % vw || s.sy % vw) return false;
    for (int a = 0; a < 3; ++a) {
        if (reinterpret_cast<uintptr_t>(ins[a]) % 16 || reinterpret_cast<uintptr_t>(outs[a]) % 16) return false;
    }
    return true;
}

int32_t fill_domain_args(int32_t storage, const pw_shape& s, const void* u, const void* v, const void* w,
                         void* su, void* sv, void* sw, double tcx, double tcy, const double* tzc1,
                         const double* tzc2, const double* tzd1, const double* tzd2, const pw_scales* scales,
                         DomainArgs* out) {
    DomainArgs d{};
    d.u = u;
    d.v = v;
    d.w = w;
    d.su = su;
    d.sv = sv;
    d.sw = sw;
    d.tzc1 = tzc1;
    d.tzc2 = tzc2;
    d.tzd1 = tzd1;
    d.tzd2 = tzd2;
    float in_s[3] = {1.0f, 1.0f, 1.0f};
    float out_s[3] = {1.0f, 1.0f, 1.0f};
    if (scales && scaled_storage(storage)) {
        for (int f = 0; f < 3; ++f) {
            const float a = scales->in_scale[f];
            const float b = scales->out_scale[f];
            if (!(a > 0.0f) || !std::isfinite(a) || !(b > 0.0f) || !std::isfinite(b)) return PW_ERR_INVALID_ARG;
            int ea, eb;
            if (std::frexp(a, &ea) != 0.5f || std::frexp(b, &eb) != 0.5f) return PW_ERR_INVALID_ARG;
            in_s[f] = a;
            out_s[f] = b;
        }
    }
    fold_coefficients(tcx, tcy, in_s, out_s, d.cx, d.cy, d.cz);
    d.nx = s.nx;
    d.ny = s.ny;
    d.nz = s.nz;
    d.sy = s.sy;
    d.sx = s.sx;
    *out = d;
    return PW_OK;
}

}  // namespace pw
