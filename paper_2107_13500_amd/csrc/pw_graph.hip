// HIP graphs of library calls: the repeated timestep of the batched form
// (perturb u and v, refill the periodic halos, compute su, sv, sw of every
// domain) recorded once and replayed per call, so a call costs one graph
// launch instead of three kernel launches per step.
//
// Recording is plain stream capture.  The recorded entry points launch
// kernels only: they never allocate, never synchronise and issue no memset
// (counters and flags are written by kernels), so every replay redoes
// exactly the recorded work.
#include <hip/hip_runtime.h>

#include <new>

#include "pw_advect.h"
#include "pw_plan.hpp"

struct pw_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int32_t hip_status(hipError_t e) { return e == hipSuccess ? PW_OK : pw::report_hip(e); }

// End the capture on `s` and instantiate it into a new pw_graph.
int32_t finish_capture(hipStream_t s, pw_graph** out) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return pw::report_hip(e);
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return pw::report_hip(e);
    }
    pw_graph* r = new (std::nothrow) pw_graph();
    if (!r) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        return PW_ERR_OUT_OF_MEMORY;
    }
    r->graph = g;
    r->exec = x;
    *out = r;
    return PW_OK;
}

}  // namespace

extern "C" {

int32_t pw_graph_begin(void** stream) {
    if (!stream) return PW_ERR_INVALID_ARG;
    *stream = nullptr;
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return pw::report_hip(e);
    // thread-local mode: an allocation by this thread during the recording
    // is an error instead of a silently recorded side effect
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(s);
        return pw::report_hip(e);
    }
    *stream = s;
    return PW_OK;
}

int32_t pw_graph_end(void* stream, pw_graph** graph) {
    if (!stream || !graph) return PW_ERR_INVALID_ARG;
    *graph = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess) return pw::report_hip(e);
    if (cs == hipStreamCaptureStatusNone) return PW_ERR_CAPTURE;
    const int32_t rc = finish_capture(s, graph);
    // the recording stream goes away with the recording: a stream left alive
    // after a capture has been seen to keep the asynchronous copies of
    // other streams in the process from overlapping with kernels
    e = hipStreamDestroy(s);
    if (rc != PW_OK) return rc;
    if (e != hipSuccess) {
        pw_graph_destroy(*graph);
        *graph = nullptr;
        return pw::report_hip(e);
    }
    return PW_OK;
}

int32_t pw_graph_capture_timestep(const pw_plan* plan, int32_t ndomains, const pw_domain_args* d_args,
                                  uint64_t seed, unsigned long long* d_call, double amplitude, int32_t nsteps,
                                  pw_graph** graph) {
    if (!graph) return PW_ERR_INVALID_ARG;
    *graph = nullptr;
    if (!plan || !d_args || !d_call || nsteps < 1) return PW_ERR_INVALID_ARG;
    if (ndomains != plan->ndomains) return PW_ERR_PLAN_MISMATCH;
    if (!plan->batch.d_table) return PW_ERR_UNSUPPORTED;
    void* s = nullptr;
    int32_t rc = pw_graph_begin(&s);
    if (rc != PW_OK) return rc;
    for (int32_t step = 0; step < nsteps && rc == PW_OK; ++step) {
        rc = pw_perturb_batched(plan, ndomains, d_args, seed, d_call, amplitude, s);
        if (rc == PW_OK) rc = pw_fill_halo_batched(plan, ndomains, d_args, s);
        if (rc == PW_OK) rc = pw_advect_batched(plan, ndomains, d_args, s);
    }
    if (rc == PW_OK) return pw_graph_end(s, graph);
    pw_graph* abandoned = nullptr;
    (void)pw_graph_end(s, &abandoned);   // ends the recording and frees its stream
    pw_graph_destroy(abandoned);
    return rc;
}

int32_t pw_graph_launch(const pw_graph* graph, void* stream) {
    if (!graph || !graph->exec) return PW_ERR_INVALID_ARG;
    return hip_status(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)));
}

int32_t pw_graph_destroy(pw_graph* graph) {
    if (!graph) return PW_OK;
    hipError_t e1 = graph->exec ? hipGraphExecDestroy(graph->exec) : hipSuccess;
    hipError_t e2 = graph->graph ? hipGraphDestroy(graph->graph) : hipSuccess;
    delete graph;
    if (e1 != hipSuccess) return pw::report_hip(e1);
    return hip_status(e2);
}

}  // extern "C"
