// Internal plan layout and host helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "pw_advect.h"
#include "pw_kernels.hpp"

namespace pw {

// Resolved launch shape of one domain (or of the batched kernel).
struct Launch {
    int32_t variant = 0;
    int32_t chunk = 0;     // march: points per workgroup chunk
    int32_t seg = 0;       // march: planes per segment
    int32_t block = 0;     // threads per workgroup
    int32_t nchunks = 0;   // march: chunks per plane; direct: blocks per plane
    int32_t nseg = 0;      // march: segments; direct: planes
    int32_t wpad = 0;      // march: LDS elements per field per slot
    int32_t cpx = 0;       // march: compact tile order, chunk slots per XCD and segment (0: not used)
    int64_t workgroups = 0;
    int64_t tiles = 0;
    int64_t lds_bytes = 0;
};

// Device table of a batched plan (one entry per domain).
struct BatchDomain {
    int32_t nx, ny, nz;
    int32_t nchunks;
    int32_t nseg;
    int32_t seg;          // planes per segment: nx split into nseg even parts
    int64_t sy, sx;
    int64_t tile_begin;   // first global tile of this domain
    int32_t rec;          // index of the domain's record in the caller's pw_domain_args array
    int32_t pad_;
};

struct BatchState {
    Launch launch;               // shared kernel shape (chunk, seg, wpad for the largest nz)
    BatchDomain* d_table = nullptr;
    unsigned long long* d_errors = nullptr;
    const int32_t* d_order = nullptr;   // one workgroup per tile: each workgroup's tile (-1: none), or NULL
    int device = -1;
    bool vec_shapes = false;     // every shape allows 16-byte loads
    int32_t kind = 2;            // code paths of the batched kernel (BatchKind in pw_batched.hip)
};

}  // namespace pw

struct pw_plan {
    int32_t storage = 0;
    int32_t ndomains = 0;
    pw_tuning tuning{};
    std::vector<pw_shape> shapes;   // strides normalised
    int64_t points = 0;
    pw::Launch single;              // ndomains == 1
    pw::BatchState batch;           // ndomains >= 1 (batched entry point)
};

namespace pw {

int64_t elem_bytes(int32_t storage);
int64_t compute_bytes(int32_t storage);
int64_t march_lds_bytes(int32_t storage, int32_t wpad);
bool scaled_storage(int32_t storage);   // 16-bit and int32 types: per-field scales
int32_t normalize_shape(const pw_shape& in, pw_shape* out);
int64_t extent_elems(const pw_shape& s);
bool march_possible(const pw_shape& s);
int32_t auto_seg(int32_t storage, const pw_shape& s, int32_t nchunks);
int32_t resolve_launch(int32_t storage, const pw_shape& s, const pw_tuning& t, Launch* L);
bool any_overlap(const void* const ins[3], void* const outs[3], int64_t ext);
bool vector_ok(int32_t storage, const pw_shape& s, const void* const ins[3], void* const outs[3]);
int32_t fill_domain_args(int32_t storage, const pw_shape& s, const void* u, const void* v, const void* w,
                         void* su, void* sv, void* sw, double tcx, double tcy, const double* tzc1,
                         const double* tzc2, const double* tzd1, const double* tzd2, const pw_scales* scales,
                         DomainArgs* out);
int32_t report_hip(hipError_t e);

// batched plans (pw_batched.hip)
int32_t batched_plan_init(pw_plan* p);
int32_t batched_plan_free(pw_plan* p);

}  // namespace pw
