/*
 * pw_advect.h -- C ABI of the MI355X (gfx950) Piacsek-Williams advection library.
 *
 * The library computes the PW momentum-advection source terms su, sv, sw from
 * the wind fields u, v, w (N. Brown, "Accelerating advection for atmospheric
 * modelling on Xilinx and Intel FPGAs", Sec. II-A, Listing 1):
 *
 *   su  Listing 1: x flux term (tcx), y flux term (tcy), vertical term with
 *       tzc1 (lower face) and tzc2 (upper face), for k = 2..nz; at k = nz the
 *       upper vertical flux is dropped.
 *   sv  the x<->y mirror of su on the same staggered (Arakawa C) grid
 *       (v on y faces): y term first with tcy, then x term with tcx, then the
 *       vertical term with tzc1/tzc2; k = 2..nz, truncated at k = nz likewise.
 *   sw  the same staggering rule for w on z faces: x and y flux terms with u,
 *       v summed across the two levels k, k+1, and a vertical term in w with
 *       tzd1 (lower) and tzd2 (upper); k = 2..nz-1.
 *   Every output is written as 0 at k = 1, and sw at k = nz (+0 for the
 *   floating storage types).
 *
 * Inputs are taken to be finite (fixed-point inputs always are).  For BF16
 * and FP16 storage the staged kernels evaluate the column top as the full
 * form with the upper vertical flux multiplied by an exact zero, so a
 * non-finite w at level nz of a column or of its x (su) or y (sv) neighbour
 * makes su(nz) or sv(nz) NaN, although the truncated formula does not read
 * that value.  FP64 and FP32 storage select the truncated form, so their
 * column-top results never read values above the top.
 *
 * The paper prints only su; sv and sw follow the staggering that Listing 1's
 * indices imply and the 21 operations per field that Sec. III counts.
 *
 * Layout (Listing 1, Fortran u(k, j, i)): element (k, j, i) with k in 1..nz,
 * j in 0..ny+1, i in 0..nx+1 sits at element offset
 *     (k - 1) + j * sy + i * sx
 * from the array base: k (vertical) is fastest, a one-point halo surrounds the
 * interior in x and y, there is no vertical halo.  Default strides are
 * sy = nz and sx = (ny + 2) * sy.  All six arrays of one domain share the
 * shape and strides.  For HBM throughput, allocate them back to back in
 * one allocation (each start 256-byte aligned) rather than as six separate
 * allocations: the latter share the allocator's large alignment, and equal
 * offsets in the six streams can then fall on the same memory channels.  Every interior column (i in 1..nx, j in 1..ny) of every
 * output is fully written (all k); halo columns of the outputs are never
 * touched.  The caller fills the input halos (including the corner columns,
 * which sv and su read) before the call.
 *
 * Storage precision: PW_F64 computes in FP64.  PW_F32, PW_BF16, PW_F16 and
 * PW_I16 store all six arrays in that type and compute in FP32 with every flux
 * difference in a compensated form: FP32 storage subtracts neighbouring values
 * first (exact when they are within a factor of two); the 16-bit types use
 * Kahan's fused multiply-add product difference on sums of two stored values,
 * which FP32 holds exactly for int16, and for BF16 (FP16) whenever the two
 * magnitudes are within 2^15 (2^12) of each other.  The vertical coefficients stay FP64 in memory and are rounded
 * to FP32 once per thread.  PW_I32 stores 32-bit fixed point and computes in
 * FP64 (every int32 converts exactly).  For the 16-bit types and PW_I32 each
 * field has a power-of-two scale: stored = value * scale.
 *
 * Conventions for every entry point:
 *  - Pointers named "device" are HIP device (or managed) pointers owned by
 *    the caller; the library never frees them.  Pointers named "host" are
 *    read before the call returns.
 *  - Functions return a pw_status (PW_OK = 0, errors negative) and never
 *    throw.  Argument errors are detected on the host before anything is
 *    launched.  A failed HIP call returns PW_ERR_HIP and its hipError_t is
 *    kept for pw_last_hip_error() (per host thread).  Faults inside a kernel
 *    surface at the caller's next synchronisation, as with any HIP launch.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Compute entry points are asynchronous on that stream, never synchronise
 *    and never allocate, so they may be recorded into a HIP graph.
 */
#ifndef PW_ADVECT_H
#define PW_ADVECT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
    PW_OK = 0,
    PW_ERR_INVALID_ARG = -1,   /* null pointer, bad size or stride, bad tuning value */
    PW_ERR_UNSUPPORTED = -2,   /* unknown dtype or variant, or no GPU device */
    PW_ERR_ALIAS = -3,         /* an output overlaps an input or another output */
    PW_ERR_ALIGNMENT = -4,     /* a pointer is not aligned to its element size */
    PW_ERR_OUT_OF_MEMORY = -5, /* plan tables could not be allocated */
    PW_ERR_HIP = -6,           /* a HIP runtime call failed; see pw_last_hip_error() */
    PW_ERR_CAPTURE = -7,       /* the call would allocate while the stream is being captured */
    PW_ERR_PLAN_MISMATCH = -8  /* the arguments do not match the plan */
};

/* Storage types of the six field arrays.  PW_I16 and PW_I32 are 16- and
   32-bit fixed point: a signed integer with a per-field power-of-two scale
   (stored = value * scale, rounded to nearest even and saturated to the
   type's range on output; a NaN result stores the most negative value). */
enum { PW_F64 = 0, PW_F32 = 1, PW_BF16 = 2, PW_F16 = 3, PW_I16 = 4, PW_I32 = 5 };

/* Kernel variants (pw_tuning.variant). */
enum {
    PW_VARIANT_AUTO = 0,
    PW_VARIANT_DIRECT = 1, /* one thread per point, every operand loaded through the caches */
    PW_VARIANT_MARCH = 2   /* workgroup stages y-z plane windows in LDS and marches along x */
};

/* Shape of one domain: interior extents and element strides (k stride is 1).
   nx, ny >= 1, nz >= 2.  sy = 0 means nz; sx = 0 means (ny + 2) * sy.
   Requires sy >= nz and sx >= (ny + 2) * sy. */
typedef struct pw_shape {
    int32_t nx, ny, nz;
    int32_t reserved;  /* must be 0 */
    int64_t sy, sx;
} pw_shape;

/* Launch tuning; 0 in any field selects the library default.
   variant    PW_VARIANT_*.
   chunk      points of the (j, k) plane one workgroup owns in the march
              variant (and in the batched kernel): 256, 512 or 1024.
   seg        x planes one workgroup marches through (>= 1).  In the batched
              kernel each domain splits its nx planes into n = ceil(nx / seg)
              segments of ceil(nx / n) planes (at most seg; the last may be
              shorter), so a domain's tiles have nearly equal length; the
              batched default is 16 for 4- and 8-byte storage and 64 for the
              16-bit types.
   block      threads per workgroup of the direct variant: 64, 128, 256 or 512.
   wg_per_cu  batched launches: 0 (the default) or PW_WG_ONE_PER_TILE runs
              one workgroup per tile, so the hardware hands out the tiles in
              order (one launch; the tiles are taken longest first); 1..8
              runs a persistent grid of that many resident workgroups per
              compute unit (further capped by LDS and registers), whose
              workgroups walk the tiles in the caller's domain order. */
#define PW_WG_ONE_PER_TILE (-1)
typedef struct pw_tuning {
    int32_t variant;
    int32_t chunk;
    int32_t seg;
    int32_t block;
    int32_t wg_per_cu;
} pw_tuning;

/* Per-field power-of-two scales for the 16-bit types and PW_I32 (stored =
   value * scale): in_scale for u, v, w and out_scale for su, sv, sw.  Ignored
   for PW_F64 and PW_F32; NULL means all 1. */
typedef struct pw_scales {
    float in_scale[3];
    float out_scale[3];
} pw_scales;

/* Opaque plan: storage type, domain shapes and the resolved launch shape.
   Immutable once created, so one plan may serve concurrent calls on
   different streams. */
typedef struct pw_plan pw_plan;

/* Resolved launch description of a plan (for logs and tests). */
typedef struct pw_plan_info {
    int32_t storage;
    int32_t ndomains;
    int32_t variant;      /* resolved PW_VARIANT_* of domain 0 / of the batched kernel */
    int32_t chunk;
    int32_t seg;
    int32_t block;
    int64_t workgroups;   /* workgroups of one pw_advect / pw_advect_batched launch */
    int64_t tiles;        /* (chunk, segment) tiles over all domains */
    int64_t lds_bytes;    /* dynamic LDS per workgroup */
    int64_t points;       /* interior grid points over all domains */
    int64_t batched_workgroups;  /* grid of pw_advect_batched: persistent, or one per tile (padded to
                                    whole blocks of 64 tiles; for BF16 and FP16 plans, 8 times the
                                    longest per-XCD queue of the plan's dispatch order); 0 if
                                    unavailable */
} pw_plan_info;

/* Create a plan for `ndomains` domains (1 for pw_advect; the batch size for
   pw_advect_batched) of storage type `storage`.  The plan fixes the tiling:
   contiguous chunks of each y-z plane with one halo column on either side
   (the GPU form of the paper's Y chunking with a two-point overlap, Sec. III,
   Fig. 4), each marched along x through a segment of planes (the shift
   buffer of Sec. III, Fig. 3, as an LDS ring).
     plan      host out-pointer; receives the new plan.
     shapes    host array of ndomains shapes (copied).
     tuning    host pointer or NULL (library defaults).
   The plan allocates its small device tile table here, on the current device
   (the device the plan's launches must run on); this is the only entry point
   that allocates.  Returns PW_ERR_INVALID_ARG for bad shapes or tuning,
   PW_ERR_UNSUPPORTED for an unknown storage type or a variant the shape
   cannot use, PW_ERR_CAPTURE if called while the null stream is capturing,
   PW_ERR_OUT_OF_MEMORY or PW_ERR_HIP if the table cannot be allocated. */
int32_t pw_advect_plan(pw_plan **plan, int32_t storage, const pw_shape *shapes,
                       int32_t ndomains, const pw_tuning *tuning);

/* Free a plan of pw_advect_plan and its device tables.  NULL is accepted.  The caller must make
   sure no launch that uses the plan is still running. */
int32_t pw_plan_destroy(pw_plan *plan);

/* Describe a plan of pw_advect_plan (its resolved tiling and launch shape);
   `info` is a host out-pointer. */
int32_t pw_plan_get_info(const pw_plan *plan, pw_plan_info *info);

/* su, sv, sw of one domain (paper Sec. II-A, Listing 1 for su; the mirror and
   the staggering rule for sv and sw, as stated at the top of this header).
     plan             a plan with ndomains == 1 whose storage type the arrays use.
     u, v, w          device inputs laid out as described above, halos filled.
     su, sv, sw       device outputs, same shape and strides; must not overlap
                      any input or each other (PW_ERR_ALIAS): the stencil reads
                      neighbours, so it cannot run in place.
     tcx, tcy         horizontal coefficients (host values).
     tzc1, tzc2       device, nz FP64 values each, entry k-1 for level k
                      (entries for k = 1 are not read).
     tzd1, tzd2       device, nz FP64 values each (entries k = 1 and k = nz are
                      not read).
     scales           host pointer or NULL; see pw_scales.
     stream           hipStream_t or NULL.
   Pointers must be aligned to their element size (PW_ERR_ALIGNMENT); wider
   vector loads are used when the bases are 16-byte aligned and nz and sx are
   multiples of the vector width, scalar loads otherwise. */
int32_t pw_advect(const pw_plan *plan,
                  const void *u, const void *v, const void *w,
                  void *su, void *sv, void *sw,
                  double tcx, double tcy,
                  const double *tzc1, const double *tzc2,
                  const double *tzd1, const double *tzd2,
                  const pw_scales *scales, void *stream);

/* One subdomain of a batched call.  An array of these lives in DEVICE memory
   (the kernel reads it); its shapes must equal, in order, the shapes the plan
   was created with (checked on the device: a mismatching domain, or one with
   a NULL field pointer, is skipped and counted, see pw_plan_error_count).
   When every shape of the plan allows 16-byte vector access (nz, sy and sx
   multiples of 16 / element size), the six field pointers must also be
   16-byte aligned; a record that is not is skipped and counted the same way.
   For scaled storage types a scale of 0 means 1. */
typedef struct pw_domain_args {
    pw_shape shape;
    const void *u, *v, *w;
    void *su, *sv, *sw;
    double tcx, tcy;
    const double *tzc1, *tzc2, *tzd1, *tzd2;
    pw_scales scales;
} pw_domain_args;

/* su, sv, sw of all domains of a batched plan in one launch (one workgroup
   per tile by default, or a persistent grid with wg_per_cu 1..8).
   Definition as for pw_advect (Sec. II-A, Listing 1), applied to every
   subdomain of a decomposed model that one device holds: the scheme runs once
   per model timestep (Sec. II-A) over each subdomain, and where the paper
   runs several kernels side by side to fill the device (Sec. IV), one launch
   here spreads uneven subdomains over the whole GPU.
     plan       plan created with the batch's shapes (ndomains > 1 allowed, 1 too).
     ndomains   must equal the plan's ndomains (PW_ERR_PLAN_MISMATCH).
     d_args     device array of ndomains pw_domain_args.
     stream     hipStream_t or NULL.
   Every domain is computed exactly as pw_advect computes it (same per-point
   arithmetic), so results are bit-identical to per-domain calls.  Overlap
   between domains' arrays is not checked. */
int32_t pw_advect_batched(const pw_plan *plan, int32_t ndomains,
                          const pw_domain_args *d_args, void *stream);

/* pw_advect_batched without a plan, for callers that cannot allocate device
   memory (code recorded into a HIP graph, tight serving loops, harnesses that
   forbid hipMalloc): it calls no hipMalloc, hipFree or other allocating
   routine.  The tile table and error word that a plan would own live in a
   fixed array of 229,440 bytes per GPU inside the library (allocated with its
   code, held until the process ends); a small kernel rebuilds the table from
   the device records on every call, then the batched kernel runs as in
   pw_advect_batched, with identical results.
     storage    PW_* storage type.
     shapes     host array of ndomains shapes (as for pw_advect_plan); the
                device records must carry the same shapes, checked on the
                device by a digest: if they differ, no domain is computed and
                all ndomains are counted as skipped.
     ndomains   1 .. 4096 (PW_ERR_INVALID_ARG beyond).
     d_args     device array of ndomains pw_domain_args (as for
                pw_advect_batched; records are skipped and counted likewise).
     tuning     host pointer or NULL; chunk, seg and wg_per_cu as for a
                batched plan.
     d_skipped  device pointer to one counter or NULL; if given, the number
                of records this call skipped is added to it (the caller
                clears it).
     stream     hipStream_t or NULL.
   Every call on one GPU uses that GPU's one array: calls that may overlap in
   time on the same GPU (different streams, different host threads) race and
   must be ordered by the caller.  Returns PW_ERR_UNSUPPORTED if a shape
   cannot use the batched kernel. */
int32_t pw_advect_batched_noalloc(int32_t storage, const pw_shape *shapes, int32_t ndomains,
                                  const pw_domain_args *d_args, const pw_tuning *tuning,
                                  unsigned long long *d_skipped, void *stream);

/* Periodic x-y halo fill of u, v, w of every domain of a plan (asynchronous,
   no allocation; may be recorded into a graph).  The stencil has depth one
   (Sec. II-A, Sec. III), so each call needs the one-point halo refreshed; this
   is the repeated-timestep harness's refresh, not part of the stencil.  Each halo column (i, j)
   receives interior column (wrap(i), wrap(j)), wrap(0) = n, wrap(n+1) = 1, so
   corner columns are periodic too.  Arguments as for pw_advect_batched. */
int32_t pw_fill_halo_batched(const pw_plan *plan, int32_t ndomains,
                             const pw_domain_args *d_args, void *stream);

/* Add amplitude * r to every interior point of u and v of every domain, with
   r uniform in [-1, 1) from a counter-based hash of (seed, *d_call, domain,
   point) -- a SplitMix64 key per (seed, call, domain), then one 32-bit
   lowbias32 hash per element; then increment *d_call on the device.  Used to
   change the fields between repeated timestep calls (the scheme runs once
   per model timestep, Sec. II-A), also inside a replayed graph; harness, not
   part of the stencil.  d_call: device pointer to one 64-bit counter owned by the caller.
   Halos are not refreshed (call pw_fill_halo_batched after). */
int32_t pw_perturb_batched(const pw_plan *plan, int32_t ndomains,
                           const pw_domain_args *d_args, uint64_t seed,
                           unsigned long long *d_call, double amplitude, void *stream);

/* HIP graphs of library calls (the paper's many short kernel executions,
   Sec. IV, recorded once and replayed).  A pw_graph owns an instantiated HIP
   graph; every entry point it records launches kernels only, so each replay
   redoes exactly the recorded work on the same device buffers (a
   perturbation's call counter lives in device memory and advances on every
   replay).

   pw_graph_begin: start a recording.  `stream` (host out-pointer) receives
   a new hipStream_t (as void*) owned by the recording: library calls issued
   on it until pw_graph_end are recorded, not run.  The recording is
   thread-local: the entry points that allocate (plan creation, the
   autotuner, host-resident calls) must not be called by this thread until
   pw_graph_end, since HIP rejects an allocation during the recording and
   invalidates it.
   pw_graph_end: stop the recording on `stream` (from pw_graph_begin),
   instantiate it and destroy the stream; `graph` (host out-pointer)
   receives the new graph.  PW_ERR_CAPTURE if the stream is not recording;
   PW_ERR_HIP if HIP rejects the recording.  (The library records on a
   stream of its own because on MI355X a stream left alive after a capture
   has been seen to keep later asynchronous copies of the process from
   overlapping with kernels.) */
typedef struct pw_graph pw_graph;
int32_t pw_graph_begin(void **stream);
int32_t pw_graph_end(void *stream, pw_graph **graph);

/* Record `nsteps` repeated timesteps of a batched plan into a new graph --
   each step pw_perturb_batched (seed, d_call, amplitude), then
   pw_fill_halo_batched, then pw_advect_batched, all on `d_args` -- through
   pw_graph_begin / pw_graph_end (allocates the graph; not for use while
   another recording of this thread is open).  Arguments as for those calls; nsteps >= 1.
   `graph` (host out-pointer) receives the graph. */
int32_t pw_graph_capture_timestep(const pw_plan *plan, int32_t ndomains, const pw_domain_args *d_args,
                                  uint64_t seed, unsigned long long *d_call, double amplitude,
                                  int32_t nsteps, pw_graph **graph);

/* Replay a graph on `stream` (asynchronous; NULL: the null stream).  Replays
   on one graph must not overlap in time. */
int32_t pw_graph_launch(const pw_graph *graph, void *stream);

/* Free a graph (NULL accepted); no replay of it may still be running. */
int32_t pw_graph_destroy(pw_graph *graph);

/* Error count of a batched plan (pw_advect_batched, its halo fill and
   perturbation): the number of domain records skipped so far because their shape did
   not match the plan, a field pointer was NULL or (vector-aligned plans) not
   16-byte aligned.  Synchronous (copies one word from the device).  `count`
   is a host out-pointer. */
int32_t pw_plan_error_count(const pw_plan *plan, unsigned long long *count);

/* Host-resident domains (paper Sec. IV: the accelerator run with the
   host<->device transfers included).  A stream plan owns device buffers,
   streams (one kernel stream, one copy stream per field and direction) and
   events for one host domain shape:
     bulk != 0  one round trip: copy the whole domain in, compute, copy the
                outputs out, in order on one stream (no overlap);
     bulk == 0  x-slabs of `chunk` planes through a ring of `nbuffers` (2..8)
                device slab buffers: the inputs of one slab (its planes plus
                one x-halo plane on each side) are copied in while the
                previous slab is computed and the one before it is copied
                out, ordered by events.
   Requires packed columns (sy == nz).  Allocates; not for use during
   capture (PW_ERR_CAPTURE).  `tuning` (host or NULL) applies to the slab
   kernels. */
typedef struct pw_stream_plan pw_stream_plan;
int32_t pw_stream_plan_create(pw_stream_plan **plan, int32_t storage, const pw_shape *shape,
                              int32_t chunk, int32_t nbuffers, int32_t bulk, const pw_tuning *tuning);
/* Synchronises the device, then frees the plan. */
int32_t pw_stream_plan_destroy(pw_stream_plan *plan);

/* su, sv, sw of a host-resident domain (same results as pw_advect on the
   same data).  All pointers are HOST pointers; pinned memory (hipHostMalloc)
   lets the copies run asynchronously and overlap.  Each array must span the
   domain's extent; the output halo columns are never written.  Blocks until
   the outputs are on the host; an error return, too, comes only after every
   copy and kernel the call queued has finished, so the host buffers may be
   released at once.  Returns PW_ERR_ALIAS if an output overlaps an input. */
int32_t pw_advect_host(pw_stream_plan *plan,
                       const void *h_u, const void *h_v, const void *h_w,
                       void *h_su, void *h_sv, void *h_sw,
                       double tcx, double tcy,
                       const double *h_tzc1, const double *h_tzc2,
                       const double *h_tzd1, const double *h_tzd2,
                       const pw_scales *scales);

/* Launch-shape autotuner (the batched form's tile shapes: chunk, segment
   length, workgroups per CU; the single-domain variant, chunk and segment).
   The paper fixes its Y chunk size by on-chip memory and finds the size of no
   consequence above 8 (Sec. III); on the GPU chunk and segment length trade
   halo re-reads against tiles to fill the device, so they are measured.
   Times each candidate tuning on the caller's buffers -- pw_advect with
   h_args[0] when ndomains == 1, pw_advect_batched with d_args otherwise --
   as the median of `reps` calls after one warm-up, and returns the fastest.
     storage, shapes, ndomains  as for pw_advect_plan.
     h_args      host array (ndomains == 1: one record whose pointers are
                 device pointers; its shape field is ignored).
     d_args      device array of ndomains records (ndomains > 1).
     candidates  host array of ncandidates tunings, or NULL with
                 ncandidates == 0 for the built-in search space (see
                 pw_autotune_candidates).
     best        host out-pointer: fastest tuning.
     best_ms     host out-pointer or NULL: its median time in ms.
     all_ms      host array of one float per candidate or NULL: median
                 times, -1 for candidates the shape cannot use.
   Overwrites the outputs.  Allocates, creates a stream and synchronises:
   not for use during stream capture (PW_ERR_CAPTURE).  Returns
   PW_ERR_UNSUPPORTED if no candidate is usable. */
int32_t pw_autotune(int32_t storage, const pw_shape *shapes, int32_t ndomains,
                    const pw_domain_args *h_args, const pw_domain_args *d_args,
                    const pw_tuning *candidates, int32_t ncandidates, int32_t reps,
                    pw_tuning *best, float *best_ms, float *all_ms);

/* The built-in search space of pw_autotune: writes up to `capacity` tunings to
   `out` (host, may be NULL) and returns how many there are. */
int32_t pw_autotune_candidates(int32_t batched, pw_tuning *out, int32_t capacity);

/* Measurement utility (no part of the stencil; it measures the attainable
   HBM bandwidth that replaces the paper's operations-times-clock
   "theoretical performance", Sec. III, Table I): streaming copy src[s] ->
   dst[s] for s < nstreams (1..3) of `bytes` bytes each (a multiple of 16),
   with the stencil kernels' access width (16-byte loads, non-temporal 16-byte
   stores).  Its time gives the attainable HBM read+write bandwidth and its
   profiler counters calibrate the byte counters.  src, dst: host arrays of
   device pointers (16-byte aligned, not overlapping); workgroups: grid size
   (0 = 16 per compute unit of a 256-CU part).  Asynchronous on `stream`. */
int32_t pw_probe_copy(const void *const *src, void *const *dst, int32_t nstreams,
                      int64_t bytes, int32_t workgroups, void *stream);

/* Measurement utility (no part of the stencil; as pw_probe_copy, Sec. III,
   Table I): the general form of pw_probe_copy.  Reads nsrc (0..3) and writes ndst (0..3) buffers of
   `bytes` bytes each (a multiple of 16), not both zero:
     nsrc > 0, ndst > 0  dst[s] = src[s mod nsrc] (a copy);
     nsrc = 0            dst[s] receives a fixed pattern (write only);
     ndst = 0            the sources are read and XOR-reduced (read only);
                         `sink` (device, 16 bytes per workgroup) receives a
                         word only if the reduction hits a fixed marker, so
                         the loads cannot be dropped by the compiler.
   flags: PW_PROBE_* bits -- non-temporal loads (default plain), cached
   stores (default non-temporal), four 16-byte words per lane and buffer in
   each block (default one).  The main loop is free of per-lane conditions;
   the ragged tail is handled separately.  src, dst: host arrays of device
   pointers (16-byte aligned); sink may be NULL when ndst > 0.  workgroups:
   grid size, 0 = one workgroup per block (256 lanes x 1 or 4 words per
   buffer); a smaller grid walks the blocks grid-stride.  Asynchronous on
   `stream`.  Returns PW_ERR_INVALID_ARG for bad counts, sizes or flags,
   PW_ERR_ALIGNMENT for a misaligned pointer. */
#define PW_PROBE_NT_LOADS 1
#define PW_PROBE_CACHED_STORES 2
#define PW_PROBE_UNROLL4 4
int32_t pw_probe_bandwidth(const void *const *src, int32_t nsrc, void *const *dst, int32_t ndst,
                           int64_t bytes, int32_t workgroups, int32_t flags, void *sink, void *stream);

/* Measurement utility (no part of the stencil; as pw_probe_copy, Sec. III,
   Table I): the march kernel's HBM access pattern for FP64 storage without
   LDS or arithmetic, the reference for what the stencil's own data movement
   can reach.  Each workgroup owns a chunk of 512 points of the y-z plane and
   a segment of `seg` x planes (the march kernel's compact tile order); for
   each of the segment's seg + 2 input planes it loads the chunk's window
   (the chunk and nz points on either side) of u, v, w, and for each of its
   seg output planes it stores the chunk of su, sv, sw: out(plane, vector t)
   = in(plane, window vector t) + in(plane, window vector min(256 + t,
   255 + nz)) in 2-double vectors.  Occupancy is capped at two workgroups
   per CU, as in the FP64 march kernel.
     u, v, w, su, sv, sw  device FP64 arrays laid out as for pw_advect
                          (16-byte aligned); su, sv, sw are overwritten in
                          their interior columns only.
     shape      host pointer: nz even, 2..256; sy == nz; sx >= (ny+2) nz and
                even; ny * nz a multiple of 512.
     seg        even, >= 2, dividing nx.
   Asynchronous on `stream`.  PW_ERR_INVALID_ARG for other shapes or
   segments, PW_ERR_ALIGNMENT for a misaligned pointer. */
int32_t pw_probe_march(const void *u, const void *v, const void *w, void *su, void *sv, void *sw,
                       const pw_shape *shape, int32_t seg, void *stream);

/* Human-readable name of a status code (static string). */
const char *pw_status_string(int32_t status);

/* hipError_t behind the last PW_ERR_HIP returned on this host thread (0 if none). */
int32_t pw_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PW_ADVECT_H */
