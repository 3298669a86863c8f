// Host-resident domains: PW advection with the host<->device transfers
// included, either as one bulk round trip or as x-slabs whose transfers
// overlap the kernel of the neighbouring slab (paper Sec. IV: chunking along
// x with event dependencies so that, apart from the first and last chunk,
// transfers are in flight while kernels run).
//
// A slab of planes i0..i1 needs input planes i0-1..i1+1 (one plane of x halo
// on each side) and produces output planes i0..i1.  Planes are contiguous in
// the layout, so each slab's inputs are one copy per field; outputs are copied
// back as a 2D copy of the interior columns only, so the host outputs' halo
// columns are never written.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "pw_advect.h"
#include "pw_plan.hpp"

// Copy streams per direction.  Measured on MI355X with pinned host memory:
// one stream each way moves 57 GB/s host-to-device or device-to-host alone
// and 97 GB/s with both directions at once; three streams each way drop the
// two-way rate to 82 GB/s.
constexpr int kCopyStreams = 1;

struct pw_stream_plan {
    int32_t storage = 0;
    pw_shape shape{};          // the whole host domain (strides normalised)
    int32_t chunk = 0;         // planes per slab
    int32_t nbuf = 0;          // device slab buffers in the ring
    pw_plan* plan_full = nullptr;   // slab of `chunk` planes
    pw_plan* plan_tail = nullptr;   // last, shorter slab (if any)
    pw_plan* plan_bulk = nullptr;   // the whole domain (bulk mode)
    std::vector<void*> slab_in;     // per buffer: u, v, w inputs ((chunk + 2) planes each), contiguous
    std::vector<void*> slab_out;    // per buffer: su, sv, sw outputs (chunk planes each)
    void* bulk = nullptr;           // bulk mode: 6 whole arrays
    double* coef = nullptr;         // 4 * nz coefficients
    // kCopyStreams copy streams in each direction (field f uses stream
    // f % kCopyStreams), one kernel stream; events per ring buffer and field
    hipStream_t s_in[3] = {nullptr, nullptr, nullptr};
    hipStream_t s_out[3] = {nullptr, nullptr, nullptr};
    hipStream_t s_run = nullptr;
    std::vector<hipEvent_t> ev_in, ev_run, ev_out;   // ev_in, ev_out: 3 per buffer
    int64_t plane_elems = 0;   // sx
    int64_t eb = 0;
};

namespace {

void release(pw_stream_plan* p) {
    if (!p) return;
    for (void* q : p->slab_in) (void)hipFree(q);
    for (void* q : p->slab_out) (void)hipFree(q);
    if (p->bulk) (void)hipFree(p->bulk);
    if (p->coef) (void)hipFree(p->coef);
    for (auto* v : {&p->ev_in, &p->ev_run, &p->ev_out})
        for (hipEvent_t e : *v) (void)hipEventDestroy(e);
    for (hipStream_t s : {p->s_in[0], p->s_in[1], p->s_in[2], p->s_run, p->s_out[0], p->s_out[1], p->s_out[2]})
        if (s) (void)hipStreamDestroy(s);
    pw_plan_destroy(p->plan_full);
    pw_plan_destroy(p->plan_tail);
    pw_plan_destroy(p->plan_bulk);
    delete p;
}

int32_t hip_status(hipError_t e) {
    if (e == hipErrorOutOfMemory) return PW_ERR_OUT_OF_MEMORY;
    return pw::report_hip(e);
}

// An error return first waits for the copies and kernels already queued on
// the plan's streams: they reference the caller's host buffers, which the
// caller may release once the call has returned.
int32_t fail(pw_stream_plan* p, int32_t rc) {
    for (hipStream_t s : {p->s_in[0], p->s_in[1], p->s_in[2], p->s_run, p->s_out[0], p->s_out[1], p->s_out[2]})
        if (s) (void)hipStreamSynchronize(s);
    return rc;
}

}  // namespace

extern "C" {

int32_t pw_stream_plan_create(pw_stream_plan** out, int32_t storage, const pw_shape* shape, int32_t chunk,
                              int32_t nbuffers, int32_t bulk, const pw_tuning* tuning) {
    if (!out || !shape) return PW_ERR_INVALID_ARG;
    *out = nullptr;
    if (pw::elem_bytes(storage) == 0) return PW_ERR_UNSUPPORTED;
    pw_shape s;
    int32_t rc = pw::normalize_shape(*shape, &s);
    if (rc != PW_OK) return rc;
    if (s.sy != s.nz) return PW_ERR_UNSUPPORTED;   // packed columns: interior rows are contiguous
    if (!bulk && (chunk < 1 || nbuffers < 2 || nbuffers > 8)) return PW_ERR_INVALID_ARG;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(nullptr, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return PW_ERR_CAPTURE;

    pw_stream_plan* p = new (std::nothrow) pw_stream_plan();
    if (!p) return PW_ERR_OUT_OF_MEMORY;
    p->storage = storage;
    p->shape = s;
    p->eb = pw::elem_bytes(storage);
    p->plane_elems = s.sx;
    const int64_t plane_bytes = s.sx * p->eb;
    hipError_t e = hipSuccess;
    if (bulk) {
        p->chunk = s.nx;
        p->nbuf = 1;
        rc = pw_advect_plan(&p->plan_bulk, storage, &s, 1, tuning);
        if (rc == PW_OK) e = hipMalloc(&p->bulk, 6 * (size_t)(s.nx + 2) * plane_bytes);
    } else {
        p->chunk = std::min(chunk, s.nx);
        p->nbuf = nbuffers;
        pw_shape cs_ = s;
        cs_.nx = p->chunk;
        rc = pw_advect_plan(&p->plan_full, storage, &cs_, 1, tuning);
        const int32_t tail = s.nx % p->chunk;
        if (rc == PW_OK && tail) {
            cs_.nx = tail;
            rc = pw_advect_plan(&p->plan_tail, storage, &cs_, 1, tuning);
        }
        for (int b = 0; b < nbuffers && rc == PW_OK && e == hipSuccess; ++b) {
            void* in = nullptr;
            void* o = nullptr;
            e = hipMalloc(&in, 3 * (size_t)(p->chunk + 2) * plane_bytes);
            if (e == hipSuccess) p->slab_in.push_back(in);
            if (e == hipSuccess) e = hipMalloc(&o, 3 * (size_t)(p->chunk + 2) * plane_bytes);
            if (e == hipSuccess) p->slab_out.push_back(o);
        }
    }
    if (rc == PW_OK && e == hipSuccess) e = hipMalloc(&p->coef, 4 * sizeof(double) * s.nz);
    for (int f = 0; f < kCopyStreams && rc == PW_OK && e == hipSuccess; ++f) {
        e = hipStreamCreateWithFlags(&p->s_in[f], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->s_out[f], hipStreamNonBlocking);
    }
    if (rc == PW_OK && e == hipSuccess) e = hipStreamCreateWithFlags(&p->s_run, hipStreamNonBlocking);
    for (int b = 0; b < p->nbuf && rc == PW_OK && e == hipSuccess; ++b) {
        hipEvent_t r;
        e = hipEventCreateWithFlags(&r, hipEventDisableTiming);
        if (e == hipSuccess) p->ev_run.push_back(r);
        for (int f = 0; f < 3 && e == hipSuccess; ++f) {
            hipEvent_t a, o;
            e = hipEventCreateWithFlags(&a, hipEventDisableTiming);
            if (e == hipSuccess) p->ev_in.push_back(a);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&o, hipEventDisableTiming);
            if (e == hipSuccess) p->ev_out.push_back(o);
        }
    }
    if (rc == PW_OK && e != hipSuccess) rc = hip_status(e);
    if (rc != PW_OK) {
        release(p);
        return rc;
    }
    *out = p;
    return PW_OK;
}

int32_t pw_stream_plan_destroy(pw_stream_plan* plan) {
    if (plan) {
        (void)hipDeviceSynchronize();
        release(plan);
    }
    return PW_OK;
}

int32_t pw_advect_host(pw_stream_plan* p, const void* h_u, const void* h_v, const void* h_w, void* h_su,
                       void* h_sv, void* h_sw, double tcx, double tcy, const double* h_tzc1, const double* h_tzc2,
                       const double* h_tzd1, const double* h_tzd2, const pw_scales* scales) {
    if (!p || !h_u || !h_v || !h_w || !h_su || !h_sv || !h_sw || !h_tzc1 || !h_tzc2 || !h_tzd1 || !h_tzd2)
        return PW_ERR_INVALID_ARG;
    const pw_shape& s = p->shape;
    const int64_t eb = p->eb;
    const int64_t pb = p->plane_elems * eb;          // bytes per plane
    const char* hin[3] = {static_cast<const char*>(h_u), static_cast<const char*>(h_v),
                          static_cast<const char*>(h_w)};
    char* hout[3] = {static_cast<char*>(h_su), static_cast<char*>(h_sv), static_cast<char*>(h_sw)};
    const int64_t ext = pw::extent_elems(s) * eb;   // bytes a host array must span
    const void* ins[3] = {h_u, h_v, h_w};
    void* outs[3] = {h_su, h_sv, h_sw};
    if (pw::any_overlap(ins, outs, ext)) return PW_ERR_ALIAS;

    hipError_t e = hipSuccess;
    const double* hc[4] = {h_tzc1, h_tzc2, h_tzd1, h_tzd2};
    for (int q = 0; q < 4 && e == hipSuccess; ++q)
        e = hipMemcpyAsync(p->coef + q * s.nz, hc[q], sizeof(double) * s.nz, hipMemcpyHostToDevice, p->s_run);
    if (e == hipSuccess) e = hipStreamSynchronize(p->s_run);
    if (e != hipSuccess) return fail(p, hip_status(e));
    const double* dc[4] = {p->coef, p->coef + s.nz, p->coef + 2 * s.nz, p->coef + 3 * s.nz};
    // interior columns of one plane: j = 1..ny, contiguous from offset sy
    const size_t row_bytes = (size_t)s.ny * s.sy * eb;
    const size_t row_off = (size_t)s.sy * eb;

    if (p->plan_bulk) {
        char* dev = static_cast<char*>(p->bulk);
        const size_t fb = (size_t)(s.nx + 2) * pb;
        for (int f = 0; f < 3 && e == hipSuccess; ++f)
            e = hipMemcpyAsync(dev + f * fb, hin[f], (size_t)ext, hipMemcpyHostToDevice, p->s_run);
        if (e != hipSuccess) return fail(p, hip_status(e));
        int32_t rc = pw_advect(p->plan_bulk, dev, dev + fb, dev + 2 * fb, dev + 3 * fb, dev + 4 * fb, dev + 5 * fb,
                               tcx, tcy, dc[0], dc[1], dc[2], dc[3], scales, p->s_run);
        if (rc != PW_OK) return fail(p, rc);
        for (int f = 0; f < 3 && e == hipSuccess; ++f)
            e = hipMemcpy2DAsync(hout[f] + pb + row_off, pb, dev + (3 + f) * fb + pb + row_off, pb, row_bytes,
                                 s.nx, hipMemcpyDeviceToHost, p->s_run);
        if (e == hipSuccess) e = hipStreamSynchronize(p->s_run);
        return e == hipSuccess ? PW_OK : fail(p, hip_status(e));
    }

    const int32_t nchunks = (s.nx + p->chunk - 1) / p->chunk;
    for (int32_t c = 0; c < nchunks; ++c) {
        const int b = c % p->nbuf;
        const int32_t i0 = 1 + c * p->chunk;
        const int32_t n = std::min(p->chunk, s.nx - i0 + 1);
        // planes i0-1 .. i0+n; the last plane of the domain may end at the extent
        const size_t in_bytes = (size_t)std::min<int64_t>((int64_t)(n + 2) * pb, ext - (int64_t)(i0 - 1) * pb);
        const size_t fin = (size_t)(p->chunk + 2) * pb;   // field stride inside a slab buffer
        char* din = static_cast<char*>(p->slab_in[b]);
        char* dout = static_cast<char*>(p->slab_out[b]);
        // inputs: the buffer is free once the kernel that last used it ran
        for (int f = 0; f < 3 && e == hipSuccess; ++f) {
            hipStream_t si = p->s_in[f % kCopyStreams];
            if (c >= p->nbuf) e = hipStreamWaitEvent(si, p->ev_run[b], 0);
            if (e == hipSuccess)
                e = hipMemcpyAsync(din + f * fin, hin[f] + (size_t)(i0 - 1) * pb, in_bytes, hipMemcpyHostToDevice, si);
            if (e == hipSuccess) e = hipEventRecord(p->ev_in[3 * b + f], si);
        }
        // kernel: after its inputs arrived and the previous outputs left this buffer
        for (int f = 0; f < 3 && e == hipSuccess; ++f) {
            e = hipStreamWaitEvent(p->s_run, p->ev_in[3 * b + f], 0);
            if (e == hipSuccess && c >= p->nbuf) e = hipStreamWaitEvent(p->s_run, p->ev_out[3 * b + f], 0);
        }
        if (e != hipSuccess) return fail(p, hip_status(e));
        const pw_plan* pl = n == p->chunk ? p->plan_full : p->plan_tail;
        int32_t rc = pw_advect(pl, din, din + fin, din + 2 * fin, dout, dout + fin, dout + 2 * fin, tcx, tcy, dc[0],
                               dc[1], dc[2], dc[3], scales, p->s_run);
        if (rc != PW_OK) return fail(p, rc);
        e = hipEventRecord(p->ev_run[b], p->s_run);
        // outputs: interior columns of planes i0..i0+n-1
        for (int f = 0; f < 3 && e == hipSuccess; ++f) {
            hipStream_t so = p->s_out[f % kCopyStreams];
            e = hipStreamWaitEvent(so, p->ev_run[b], 0);
            if (e == hipSuccess)
                e = hipMemcpy2DAsync(hout[f] + (size_t)i0 * pb + row_off, pb, dout + f * fin + pb + row_off, pb,
                                     row_bytes, n, hipMemcpyDeviceToHost, so);
            if (e == hipSuccess) e = hipEventRecord(p->ev_out[3 * b + f], so);
        }
        if (e != hipSuccess) return fail(p, hip_status(e));
    }
    for (int f = 0; f < kCopyStreams && e == hipSuccess; ++f) e = hipStreamSynchronize(p->s_out[f]);
    return e == hipSuccess ? PW_OK : fail(p, hip_status(e));
}

}  // extern "C"
