// Launch-shape autotuner: times candidate tunings on the caller's buffers
// with HIP events and returns the fastest.
//
// For one domain it times pw_advect; for a batch it times pw_advect_batched.
// Each candidate gets its own plan; a candidate the shape cannot use (for
// example the march variant on padded columns) is skipped, not an error.
// The outputs are overwritten by every timed call.  This entry point
// allocates (plans, events, a stream) and synchronises, so it must not be
// called while a stream is being captured.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "pw_advect.h"
#include "pw_plan.hpp"

namespace {

std::vector<pw_tuning> default_candidates(bool batched) {
    std::vector<pw_tuning> c;
    const int chunks[] = {256, 512, 1024};
    const int segs[] = {8, 16, 32, 64, 128, 256};
    for (int ch : chunks)
        for (int sg : segs) {
            if (batched) {
                for (int wpc : {8, 2, 4, PW_WG_ONE_PER_TILE}) c.push_back(pw_tuning{PW_VARIANT_MARCH, ch, sg, 0, wpc});
            } else {
                c.push_back(pw_tuning{PW_VARIANT_MARCH, ch, sg, 0, 0});
            }
        }
    if (!batched) {
        for (int b : {128, 256, 512}) c.push_back(pw_tuning{PW_VARIANT_DIRECT, 0, 0, b, 0});
    }
    return c;
}

}  // namespace

extern "C" int32_t pw_autotune_candidates(int32_t batched, pw_tuning* out, int32_t capacity) {
    const std::vector<pw_tuning> c = default_candidates(batched != 0);
    if (out) {
        for (int32_t i = 0; i < capacity && i < (int32_t)c.size(); ++i) out[i] = c[i];
    }
    return (int32_t)c.size();
}

extern "C" int32_t pw_autotune(int32_t storage, const pw_shape* shapes, int32_t ndomains,
                               const pw_domain_args* h_args, const pw_domain_args* d_args,
                               const pw_tuning* candidates, int32_t ncandidates, int32_t reps,
                               pw_tuning* best, float* best_ms, float* all_ms) {
    if (!shapes || ndomains < 1 || !best || reps < 1 || ncandidates < 0) return PW_ERR_INVALID_ARG;
    if (ndomains == 1 && !h_args) return PW_ERR_INVALID_ARG;
    if (ndomains > 1 && !d_args) return PW_ERR_INVALID_ARG;
    if (ncandidates > 0 && !candidates) return PW_ERR_INVALID_ARG;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(nullptr, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return PW_ERR_CAPTURE;

    const bool batched = ndomains > 1;
    std::vector<pw_tuning> cand = ncandidates > 0 ? std::vector<pw_tuning>(candidates, candidates + ncandidates)
                                                  : default_candidates(batched);
    // the caller's buffers may still be written by work queued on other streams
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return pw::report_hip(e);
    hipStream_t stream = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        if (stream) (void)hipStreamDestroy(stream);
        return pw::report_hip(e);
    }

    int32_t rc = PW_OK;
    float best_t = -1.0f;
    for (size_t c = 0; c < cand.size() && rc == PW_OK; ++c) {
        if (all_ms) all_ms[c] = -1.0f;
        pw_plan* plan = nullptr;
        if (pw_advect_plan(&plan, storage, shapes, ndomains, &cand[c]) != PW_OK) continue;   // not usable
        auto run = [&]() -> int32_t {
            if (batched) return pw_advect_batched(plan, ndomains, d_args, stream);
            const pw_domain_args& a = h_args[0];
            const pw_scales* sc = pw::scaled_storage(storage) ? &a.scales : nullptr;
            return pw_advect(plan, a.u, a.v, a.w, a.su, a.sv, a.sw, a.tcx, a.tcy, a.tzc1, a.tzc2, a.tzd1, a.tzd2,
                             sc, stream);
        };
        int32_t r = run();   // warm-up (also validates the arguments)
        if (r == PW_ERR_UNSUPPORTED) {
            pw_plan_destroy(plan);
            continue;
        }
        if (r != PW_OK) {
            rc = r;
            pw_plan_destroy(plan);
            break;
        }
        std::vector<float> t(reps);
        for (int i = 0; i < reps && rc == PW_OK; ++i) {
            e = hipEventRecord(e0, stream);
            if (e == hipSuccess && (r = run()) != PW_OK) rc = r;
            if (e == hipSuccess && rc == PW_OK) e = hipEventRecord(e1, stream);
            if (e == hipSuccess && rc == PW_OK) e = hipEventSynchronize(e1);
            if (e == hipSuccess && rc == PW_OK) e = hipEventElapsedTime(&t[i], e0, e1);
            if (e != hipSuccess) rc = pw::report_hip(e);
        }
        pw_plan_destroy(plan);
        if (rc != PW_OK) break;
        std::nth_element(t.begin(), t.begin() + reps / 2, t.end());
        const float med = t[reps / 2];
        if (all_ms) all_ms[c] = med;
        if (best_t < 0.0f || med < best_t) {
            best_t = med;
            *best = cand[c];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(stream);
    if (rc != PW_OK) return rc;
    if (best_t < 0.0f) return PW_ERR_UNSUPPORTED;
    if (best_ms) *best_ms = best_t;
    return PW_OK;
}
