#!/usr/bin/env python3
"""Benchmark of the MI355X PW advection library.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload pw2048]

One step is one call of the whole stencil (su, sv and sw of every point of
one domain) on the 2048 x 2048 x 64 FP64 grid, inputs resident in HBM.  Rank
0 prints one JSON line: Gpoints/s, the HBM roofline of the kernel (algorithmic
bytes / measured kernel time against the 8 TB/s peak), the median and minimum
of single launches, the CPU oracle timed on the host cores (all usable cores up
to 16, and one thread), the storage-precision variants (FP32, BF16, FP16 and int16
with FP32 compensated compute; int32 fixed point with FP64 compute) with their
error against the FP64 oracle, the batched many-subdomain form, board power
and host-resident (PCIe-inclusive) runs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gpoints/s su/sv/sw + % HBM peak: FP64 vs FP32/BF16-storage at stated error"
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="pw2048", choices=["pw64", "pw512", "pw2048"])
    ap.add_argument("--tuning", default=None, help="JSON pw_tuning override, e.g. '{\"chunk\":512,\"seg\":64}'")
    ap.add_argument("--skip-cpu", action="store_true", help="do not time the CPU oracle (no error figures)")
    ap.add_argument("--skip-variants", action="store_true", help="FP64 only")
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-streaming", action="store_true", help="no host-resident (PCIe-inclusive) runs")
    ap.add_argument("--skip-power", action="store_true", help="no board-power sampling")
    ap.add_argument("--skip-probes", action="store_true", help="no HBM probe family (no copy ceilings)")
    ap.add_argument("--skip-pw512", action="store_true", help="no 512x512x64 record")
    ap.add_argument("--batched-tuning", default=None,
                    help="JSON pw_tuning for the batched leg instead of the autotuner's choice")
    ap.add_argument("--batched-replays", type=int, default=100, help="graph replays timed in the batched leg")
    ap.add_argument("--skip-per-domain", action="store_true",
                    help="batched leg without the one-launch-per-domain baseline")
    ap.add_argument("--streaming-536m", action="store_true",
                    help="also stream the 536M-point (2048x4096x64) domain, the paper's largest")
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads (0: all usable cores, max 16)")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="only time a plain device copy of this many GB per direction (HBM calibration)")
    return ap.parse_args()


def time_steps(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def per_launch(fn, n, stream):
    """Median and minimum of n launches, each bracketed by its own pair of
    events on the launch stream (run after the timed region, not part of it)."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) for a, b in evs)
    return {"median": round(t[n // 2], 5), "min": round(t[0], 5), "launches": n}


def settle(fn, stream, seconds=0.3):
    """Run fn back to back for about `seconds` (untimed) so the GPU leaves its
    idle clocks after host-side work such as input generation."""
    import torch
    t0 = time.time()
    while time.time() - t0 < seconds:
        for _ in range(10):
            fn()
        torch.cuda.synchronize()


def copy_ceiling(gbytes, steps, warmup, dev, stream, nstreams=1, grids=(16384, 32768, 65536)):
    """Read+write bandwidth of the library's streaming copy (pw_probe_copy:
    four words per lane, grid-stride) over `nstreams` buffers of `gbytes` GB
    each, best over several grid sizes; used with --copy-probe only."""
    import torch
    from paper_2107_13500_amd import binding as B
    n = int(gbytes * 1e9) // 16 * 16
    moved = 2 * n * nstreams
    bufs = [torch.empty(n // 8, dtype=torch.float64, device=dev) for _ in range(2 * nstreams)]
    src, dst = bufs[:nstreams], bufs[nstreams:]
    for a in src:
        a.fill_(1.0)
    per = {g: time_steps(lambda: B.probe_copy(src, dst, n, g, stream), steps, warmup, stream) for g in grids}
    best = min(per, key=per.get)
    return {"streams": nstreams, "bytes_per_copy": moved, "ms": round(per[best], 5),
            "gbs": round(moved / (per[best] * 1e-3) / 1e9, 1), "workgroups": best}


#: probe family (pw_probe_bandwidth): mode -> (sources, destinations, flag sets tried)
PROBE_MODES = {
    "read_only_3": (3, 0, (0, 1)),           # plain / non-temporal loads
    "write_only_3": (0, 3, (0, 2)),          # non-temporal / cached stores
    "copy_1x1": (1, 1, (0, 1, 2)),
    "copy_3x3": (3, 3, (0, 1, 2)),           # the stencil's stream count and read/write ratio
}


def probe_family(gbytes, dev, stream, steps=10, warmup=3):
    """Attainable HBM bandwidth: read-only, write-only, 1-in/1-out and
    3-in/3-out streaming over buffers of `gbytes` GB each, the best over the
    probe's variants (load and store cache policy; one word per lane with one
    block per workgroup, or four words per lane with one block per workgroup
    or a 65536-workgroup grid) and two layouts (separate allocations, and all
    six buffers packed in one allocation as the stencil's arrays are); each
    variant's rate is the median of three timings."""
    import torch
    from paper_2107_13500_amd import binding as B
    n = int(gbytes * 1e9) // 16 * 16
    shapes = [(0, 0), (B.PROBE_UNROLL4, 0), (B.PROBE_UNROLL4, 65536)]   # (unroll flag, grid; 0: one per block)
    best = {m: (0.0, None) for m in PROBE_MODES}
    sink = torch.empty(n // 256 + 16, dtype=torch.uint8, device=dev)   # 16 B per workgroup of the largest grid
    for layout in ("separate", "packed"):
        if layout == "packed":
            bufs = B.pooled_fields((n // 8,), torch.float64, dev, count=6)
        else:
            bufs = [torch.empty(n // 8, dtype=torch.float64, device=dev) for _ in range(6)]
        for a in bufs[:3]:
            a.fill_(1.0)
        for mode, (ni, no, flag_sets) in PROBE_MODES.items():
            src, dst = bufs[:ni], bufs[3:3 + no]
            for fl in flag_sets:
                for unroll, grid in shapes:
                    # median of three timings, so one short fast sample cannot set the ceiling
                    ms = sorted(time_steps(lambda: B.probe_bandwidth(src, dst, n, grid, fl | unroll, sink, stream),
                                           steps, warmup, stream) for _ in range(3))[1]
                    gbs = (ni + no) * n / (ms * 1e-3) / 1e9
                    if gbs > best[mode][0]:
                        best[mode] = (gbs, {"layout": layout, "flags": fl | unroll,
                                            "words_per_lane": 4 if unroll else 1,
                                            "workgroups": grid or "one per block"})
        del bufs, src, dst
        torch.cuda.empty_cache()
    del sink
    return {m: {"gbs": round(g, 1), "config": c} for m, (g, c) in best.items()}


def march_pattern(fields, nx, plan_seg, abytes, stream, steps=10):
    """The march kernel's own access pattern without LDS or arithmetic
    (pw_probe_march over the stencil's own six arrays; it overwrites su, sv,
    sw), the best of 16-plane and the plan's segments, each the median of
    three timings; rated in the stencil's algorithmic bytes.  Returns
    (GB/s, segment) or (0.0, None) if no segment applies."""
    from paper_2107_13500_amd import binding as B
    best = (0.0, None)
    for sg in sorted({16, plan_seg}):
        if sg % 2 or nx % sg:
            continue
        t = sorted(time_steps(lambda: B.probe_march(fields, sg, stream), steps, 3, stream) for _ in range(3))[1]
        best = max(best, (abytes / (t * 1e-3) / 1e9, sg), key=lambda r: r[0])
    return best


def measured_traffic(kernel_key, chunk, seg):
    """Calibrated HBM bytes per launch from the committed rocprofv3 counter summary,
    or None if the kernel sources or launch shape changed since it was taken."""
    from paper_2107_13500_amd import kernel_sources_sha256
    path = os.path.join(ROOT, "profiles", kernel_key + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != kernel_sources_sha256():
        return None
    if rec.get("chunk") != chunk or rec.get("seg") != seg:
        return None
    return rec.get("traffic_bytes")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(p, threads, slab=256):
    """The FP64 oracle on the same grid, timed on the host with `threads`
    OpenMP threads, and on one thread over an x-slab of the grid (the same
    per-point work, so the rate carries over); returns (record, reference
    outputs of the full grid)."""
    import numpy as np
    import oracle
    reps = 6   # about 1 s of wall time (10-20 s of CPU time) on 16 host threads
    t0 = time.perf_counter()
    ref = None
    for _ in range(reps):
        ref = oracle.advect_problem(p, threads=threads)
    dt = (time.perf_counter() - t0) / reps
    # one thread: the first `slab` interior x-planes with their halo planes
    c = p.coeffs
    sl = [np.ascontiguousarray(a[:slab + 2]) for a in (p.u, p.v, p.w)]
    reps1 = 3
    t0 = time.perf_counter()
    for _ in range(reps1):
        oracle.advect(*sl, c.tcx, c.tcy, *c.arrays(), threads=1)
    dt1 = (time.perf_counter() - t0) / reps1
    pts1 = slab * p.ny * p.nz
    rec = {"value": p.npoints / dt / 1e9, "unit": "Gpoints/s", "cores": threads, "kind": "oracle",
           "sample": "full %dx%dx%d grid, %d oracle calls (plain C FP64, no FMA), %d OpenMP threads, "
                     "%.2f s per call" % (p.nx, p.ny, p.nz, reps, threads, dt),
           "single_thread": {"value": pts1 / dt1 / 1e9, "unit": "Gpoints/s",
                             "sample": "x-slab of %d planes (%dx%dx%d), %d oracle calls on 1 thread, %.2f s per call"
                                       % (slab, slab, p.ny, p.nz, reps1, dt1)},
           "cpu_model": cpu_model(), "host_cpus_usable": len(os.sched_getaffinity(0))}
    return rec, ref


def errors_vs(ref, outs, out_scales, nx, ny):
    """max-norm and RMS relative error of device outputs against FP64 reference outputs."""
    import numpy as np
    import torch
    res = {}
    for name, r, o, s in zip(("su", "sv", "sw"), ref, outs, out_scales):
        g = o[1:-1, 1:-1].to(torch.float64).cpu().numpy()
        if s != 1.0:
            g /= s
        ri = r[1:-1, 1:-1]
        diff = g - ri
        res[name] = {"max_rel": float(np.max(np.abs(diff)) / np.max(np.abs(ri))),
                     "rms_rel": float(np.sqrt(np.mean(diff * diff)) / np.sqrt(np.mean(ri * ri)))}
        del g, diff
    res["max_rel"] = max(v["max_rel"] for v in res.values() if isinstance(v, dict))
    return res


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: measures one GPU only (the stencil kernel on one GPU's domain); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2107_13500_amd import binding as B
    from paper_2107_13500_amd import inputs, metrics

    B.lib()   # fails loudly if the HIP library is missing
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(3)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    tuning = json.loads(args.tuning) if args.tuning else None
    if args.copy_probe > 0:
        rec = copy_ceiling(args.copy_probe, args.steps, args.warmup, dev, stream)
        print(json.dumps({"copy_probe": rec}), flush=True)
        return

    t0 = time.perf_counter()
    p = inputs.workload(args.workload)
    log("inputs %s generated in %.1f s" % (args.workload, time.perf_counter() - t0))
    nx, ny, nz = p.nx, p.ny, p.nz
    c = p.coeffs
    tz = [torch.from_numpy(a).to(dev) for a in c.arrays()]

    # ---------------- FP64 headline ----------------
    # the six arrays packed into one allocation (the layout the library
    # recommends: pooled_fields)
    pool = B.pooled_fields(p.u.shape, torch.float64, dev)
    for k, a in enumerate((p.u, p.v, p.w)):
        pool[k].copy_(torch.from_numpy(a))
    u, v, w = pool[:3]
    d64 = B.DeviceDomain(u, v, w, c.tcx, c.tcy, *tz, outputs=pool[3:])
    plan = B.Plan(B.F64, [B.shape_of(u)], tuning)
    info = plan.info()
    log("plan", info)
    settle(lambda: d64.run(plan, stream), stream)   # untimed: leave idle clocks after input generation
    ms = time_steps(lambda: d64.run(plan, stream), args.steps, args.warmup, stream)
    gpts = p.npoints / (ms * 1e-3) / 1e9
    abytes = metrics.algorithmic_bytes(nx, ny, nz, 8)
    achieved = abytes / (ms * 1e-3) / 1e9
    log("FP64: %.4f ms/step, %.2f Gpts/s, %.1f GB/s algorithmic" % (ms, gpts, achieved))
    launches = per_launch(lambda: d64.run(plan, stream), max(args.steps, 5), stream)
    log("FP64 per launch", launches)

    result = {
        "metric": METRIC, "value": round(gpts, 3), "unit": "Gpoints/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded: u=5+N(0,1), v=2+N(0,1), w=0.3N(0,1), stretched z-grid, rho0 exp(-z/H))",
        "config": {"workload": "%s: one %dx%dx%d FP64 domain with a 1-point periodic x-y halo, "
                               "su+sv+sw per step" % (args.workload, nx, ny, nz),
                   "nx": nx, "ny": ny, "nz": nz, "points": p.npoints,
                   "kernel": "march" if info["variant"] == B.VARIANT_MARCH else "direct",
                   "chunk": info["chunk"], "seg": info["seg"], "workgroups": info["workgroups"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes_per_launch": abytes},
        "paper_equivalent_gflops": round(metrics.paper_equivalent_gflops(gpts * 1e9, nz), 1),
        "per_launch_ms": launches,
    }

    if info["variant"] == B.VARIANT_MARCH:
        t = measured_traffic("pw_march_f64_%s" % args.workload, info["chunk"], info["seg"])
        result["roofline"]["traffic"] = None if t is None else int(round(t))

    # attainable bandwidth on this card: buffers of one FP64 array of the
    # headline grid each (2.15 GB), read only, write only and mixed
    if not args.skip_probes:
        probes = probe_family(2.15, dev, stream)
        result["roofline"]["probes"] = probes
        mixed = max(probes["copy_1x1"]["gbs"], probes["copy_3x3"]["gbs"])
        result["roofline"]["frac_of_copy_3x3"] = round(achieved / probes["copy_3x3"]["gbs"], 4)
        result["roofline"]["frac_of_best_mixed_copy"] = round(achieved / mixed, 4)
        if info["variant"] == B.VARIANT_MARCH:
            # the march kernel's own access pattern without LDS or arithmetic,
            # over the stencil's own arrays (pw_probe_march overwrites su, sv,
            # sw, so the stencil runs once more afterwards)
            best = march_pattern(pool, nx, info["seg"], abytes, stream)
            d64.run(plan, stream)
            torch.cuda.synchronize()
            if best[1] is not None:
                probes["march_pattern"] = {"gbs": round(best[0], 1),
                                           "config": {"seg": best[1], "buffers": "the stencil's own arrays",
                                                      "bytes": "the stencil's algorithmic bytes per call"}}
                result["roofline"]["frac_of_march_pattern"] = round(achieved / best[0], 4)
        log("probe family", probes)

    # ---------------- the paper's Table I size (512 x 512 x 64), FP64 ----------------
    small = None
    if args.workload != "pw512" and not args.skip_pw512:
        small = small_workload_leg("pw512", tuning, dev, stream, args.steps, args.warmup, log,
                                   probes=not args.skip_probes)
        result["pw512"] = small["record"]

    # ---------------- storage-precision variants (outputs kept for the error check) ----------------
    kept = {}
    if not args.skip_variants:
        variants = {}
        for storage in (B.F32, B.BF16, B.F16, B.I16, B.I32):
            name = B.DTYPE_NAMES[storage]
            ins, outs_s = inputs.storage_scales(p, name)
            sc = B.make_scales(ins, outs_s)
            vpool = B.pooled_fields(p.u.shape, B.torch_dtype(storage), dev)
            for k, (a, s) in enumerate(zip((p.u, p.v, p.w), ins)):
                vpool[k].copy_(B.to_storage(a, storage, s, dev))
            fu, fv, fw = vpool[:3]
            dd = B.DeviceDomain(fu, fv, fw, c.tcx, c.tcy, *tz, scales=sc, outputs=vpool[3:])
            pl = B.Plan(storage, [B.shape_of(fu)], tuning)
            settle(lambda: dd.run(pl, stream), stream)
            vms = time_steps(lambda: dd.run(pl, stream), args.steps, args.warmup, stream)
            vb = metrics.algorithmic_bytes(nx, ny, nz, metrics.ELEM_BYTES[name])
            rec = {"gpoints_per_s": round(p.npoints / (vms * 1e-3) / 1e9, 3), "ms_per_step": round(vms, 5),
                   "speedup_vs_f64": round(ms / vms, 3),
                   "hbm_frac": round(vb / (vms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "in_scale": list(ins), "out_scale": list(outs_s)}
            variants[name] = rec
            kept[name] = (dd.outputs, outs_s)
            log(name, rec)
            del fu, fv, fw, vpool, pl
        result["precision"] = variants

    # ---------------- batched subdomains ----------------
    batches = {}
    if not args.skip_batched:
        bt = json.loads(args.batched_tuning) if args.batched_tuning else None
        result["batched"], batches = batched_leg(dev, stream, gpts, log, replays=args.batched_replays,
                                                 tuning=bt, per_domain=not args.skip_per_domain)

    # ---------------- board power during the FP64 kernel ----------------
    if not args.skip_power:
        result["power"] = power_leg(lambda: d64.run(plan, stream), ms, p.npoints, stream, log)

    # ---------------- host-resident domains, transfers included ----------------
    if not args.skip_streaming:
        sizes = [("pw512", p if args.workload == "pw512" else inputs.workload("pw512")),
                 ("pw1024", inputs.make_problem(1024, 1024, 64, inputs.SEED_BASE + 4)),
                 ("pw2048", p if args.workload == "pw2048" else inputs.workload("pw2048"))]
        if args.streaming_536m:
            sizes.append(("pw2048x4096", inputs.make_problem(2048, 4096, 64, inputs.SEED_BASE + 5)))
        result["streaming"] = streaming_leg(sizes, log)

    # ---------------- CPU oracle baseline (the only leg that runs the oracle) ----------------
    if not args.skip_cpu:
        usable = len(os.sched_getaffinity(0))
        threads = args.cpu_threads or min(usable, 16)
        rec, ref = cpu_baseline(p, threads)
        rec["gpu_over_oracle"] = round(gpts / rec["value"], 1)
        result["cpu_baseline"] = rec
        log("oracle: %.3f Gpts/s on %d threads" % (rec["value"], threads))
        torch.cuda.synchronize()
        result["parity_f64"] = errors_vs(ref, d64.outputs, (1.0, 1.0, 1.0), nx, ny)
        log("FP64 parity", result["parity_f64"]["max_rel"])
        if small is not None:
            import oracle
            sref = oracle.advect_problem(small["problem"], threads=threads)
            result["pw512"]["parity_f64"] = errors_vs(sref, small["domain"].outputs, (1.0, 1.0, 1.0),
                                                      small["problem"].nx, small["problem"].ny)
            log("pw512 FP64 parity", result["pw512"]["parity_f64"]["max_rel"])
            del sref
        for name, (outs, outs_s) in kept.items():
            result["precision"][name]["error_vs_f64_oracle"] = errors_vs(ref, outs, outs_s, nx, ny)
            log(name, "error", result["precision"][name]["error_vs_f64_oracle"]["max_rel"])
        del ref
        for name, batch in batches.items():
            result["batched"][name]["max_rel_err_sampled"] = batched_errors(batch, threads)
            log("batched", name, "error", result["batched"][name]["max_rel_err_sampled"])

    failures = parity_gate(result)
    if failures:
        result["value"] = None
        result["parity_failures"] = failures
        log("parity gate FAILED:", failures)
    print(json.dumps(result), flush=True)
    if failures:
        sys.exit(4)


def parity_gate(result):
    """Every error figure of a benchmark record against its acceptance bound
    (the bounds the GPU tests use); returns the violations, empty if none.
    A figure that was not computed (e.g. --skip-cpu) is not checked."""
    from paper_2107_13500_amd import metrics
    fails = []

    def check(where, err, bound):
        if err is None:
            return
        if not (err <= bound):   # NaN fails too
            fails.append("%s: max-norm relative error %r > %g" % (where, err, bound))

    check("f64", (result.get("parity_f64") or {}).get("max_rel"), metrics.F64_PARITY_TOL)
    check("pw512 f64", ((result.get("pw512") or {}).get("parity_f64") or {}).get("max_rel"),
          metrics.F64_PARITY_TOL)
    for name, rec in (result.get("precision") or {}).items():
        check("storage %s" % name, (rec.get("error_vs_f64_oracle") or {}).get("max_rel"),
              metrics.STORAGE_ERROR_BOUND[name])
    for name, rec in (result.get("batched") or {}).items():
        check("batched %s" % name, rec.get("max_rel_err_sampled"), metrics.BATCHED_ERROR_BOUND[name])
    return fails


def small_workload_leg(name, tuning, dev, stream, steps, warmup, log, probes=True):
    """One more FP64 workload (inputs resident in HBM, six arrays packed in one
    allocation), timed like the headline with its own roofline; its outputs are
    kept for the parity check against the oracle."""
    import torch
    from paper_2107_13500_amd import binding as B
    from paper_2107_13500_amd import inputs, metrics
    p = inputs.workload(name)
    c = p.coeffs
    tz = [torch.from_numpy(a).to(dev) for a in c.arrays()]
    pool = B.pooled_fields(p.u.shape, torch.float64, dev)
    for k, a in enumerate((p.u, p.v, p.w)):
        pool[k].copy_(torch.from_numpy(a))
    d = B.DeviceDomain(*pool[:3], c.tcx, c.tcy, *tz, outputs=pool[3:])
    plan = B.Plan(B.F64, [B.shape_of(pool[0])], tuning)
    info = plan.info()
    settle(lambda: d.run(plan, stream), stream)
    ms = time_steps(lambda: d.run(plan, stream), max(steps, 50), warmup, stream)
    abytes = metrics.algorithmic_bytes(p.nx, p.ny, p.nz, 8)
    achieved = abytes / (ms * 1e-3) / 1e9
    rec = {"workload": "%s: one %dx%dx%d FP64 domain (the paper's Table I size), su+sv+sw per call"
                       % (name, p.nx, p.ny, p.nz),
           "points": p.npoints, "ms_per_call": round(ms, 5),
           "gpoints_per_s": round(p.npoints / (ms * 1e-3) / 1e9, 3),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                        "algorithmic_bytes_per_launch": abytes},
           "per_launch_ms": per_launch(lambda: d.run(plan, stream), 20, stream),
           "chunk": info["chunk"], "seg": info["seg"], "workgroups": info["workgroups"],
           "note": "0.81 GB of arrays against the 256 MB last-level cache: repeated calls may hit it"}
    if info["variant"] == B.VARIANT_MARCH:
        t = measured_traffic("pw_march_f64_%s" % name, info["chunk"], info["seg"])
        rec["roofline"]["traffic"] = None if t is None else int(round(t))
        if probes:
            # the same access pattern without LDS or arithmetic on these arrays
            # (overwrites su, sv, sw, so the stencil runs once more after it)
            gbs, sg = march_pattern(pool, p.nx, info["seg"], abytes, stream, steps=max(steps, 50))
            d.run(plan, stream)
            torch.cuda.synchronize()
            if sg is not None:
                rec["roofline"]["march_pattern"] = {"gbs": round(gbs, 1), "seg": sg}
                rec["roofline"]["frac_of_march_pattern"] = round(achieved / gbs, 4)
    log(name, rec)
    return {"record": rec, "problem": p, "domain": d, "plan": plan}


def read_power_w():
    """Current socket power of GPU 0 in W from amd-smi, or None.  amd-smi runs
    in a process group of its own, which is killed once the reading is in (or
    after 20 s), so no helper process it started outlives the reading."""
    import signal
    import subprocess
    try:
        proc = subprocess.Popen(["amd-smi", "metric", "-g", "0", "-p", "--json"], stdout=subprocess.PIPE,
                                stderr=subprocess.DEVNULL, text=True, start_new_session=True)
    except OSError:
        return None
    try:
        out, _ = proc.communicate(timeout=20)
    except subprocess.TimeoutExpired:
        out = ""
    finally:
        try:
            os.killpg(proc.pid, signal.SIGKILL)
        except (ProcessLookupError, PermissionError):
            pass
        proc.wait()
    try:
        data = json.loads(out)
        rec = data["gpu_data"][0] if isinstance(data, dict) else data[0]
        return float(rec["power"]["socket_power"]["value"])
    except Exception:
        return None


def power_leg(step, ms_per_step, npoints, stream, log, seconds=6.0):
    """Mean board power while the kernel runs back to back for `seconds`, and
    the idle power before it; energy efficiency in Gpoints per joule."""
    import threading
    import torch
    torch.cuda.synchronize()
    time.sleep(2.0)   # the reading averages over a window: let earlier legs' load fall off
    idle = []
    for _ in range(5):
        w = read_power_w()
        if w is not None:
            idle.append(w)
        time.sleep(0.2)
    if not idle:
        return {"available": False, "reason": "amd-smi socket power not readable"}
    samples, stop = [], threading.Event()

    def poll():
        while not stop.is_set():
            w = read_power_w()
            if w is not None:
                samples.append((time.perf_counter(), w))

    n = max(1, int(seconds * 1e3 / ms_per_step))
    torch.cuda.synchronize()
    th = threading.Thread(target=poll, daemon=True)
    t0 = time.perf_counter()
    th.start()
    done = 0
    while done < n:
        for _ in range(min(200, n - done)):
            step()
        done += min(200, n - done)
        torch.cuda.synchronize()
    t1 = time.perf_counter()
    stop.set()
    th.join(timeout=30)
    busy = [w for (t, w) in samples if t0 + 0.5 <= t <= t1]
    if not busy:
        return {"available": False, "reason": "no power sample during the run"}
    mean_w = sum(busy) / len(busy)
    gpts = n * npoints / (t1 - t0) / 1e9
    rec = {"available": True, "source": "amd-smi metric -p (socket_power)", "idle_w": round(sum(idle) / len(idle), 1),
           "busy_w": round(mean_w, 1), "samples": len(busy), "seconds": round(t1 - t0, 2),
           "gpoints_per_s": round(gpts, 2), "gpoints_per_joule": round(gpts / mean_w, 4)}
    log("power", rec)
    return rec


def streaming_leg(sizes, log, chunks=(32, 64, 128), reps=3):
    """Host-resident domains in pinned memory: one bulk round trip (copy in,
    compute, copy out) against x-slabs whose transfers overlap the kernel
    (paper Sec. IV).  End-to-end Gpoints/s including the transfers."""
    import torch
    from paper_2107_13500_amd import binding as B
    out = {}
    for name, p in sizes:
        t0 = time.perf_counter()
        ins = [torch.from_numpy(a).pin_memory() for a in (p.u, p.v, p.w)]
        outs = [torch.zeros(p.u.shape, dtype=torch.float64, pin_memory=True) for _ in range(3)]
        tz = [torch.from_numpy(x).clone() for x in p.coeffs.arrays()]
        log("streaming %s: pinned host buffers in %.1f s" % (name, time.perf_counter() - t0))
        shape = B.shape_of(ins[0])
        moved = 8 * (3 * (p.nx + 2) * (p.ny + 2) * p.nz + 3 * p.npoints)

        def run_mode(**kw):
            sp = B.StreamPlan(B.F64, shape, **kw)
            sp.run(*ins, *outs, p.coeffs.tcx, p.coeffs.tcy, *tz)   # warm-up
            ts = []
            for _ in range(reps):
                a = time.perf_counter()
                sp.run(*ins, *outs, p.coeffs.tcx, p.coeffs.tcy, *tz)
                ts.append(time.perf_counter() - a)
            sp.close()
            t = sorted(ts)[len(ts) // 2]
            return {"s": round(t, 5), "gpoints_per_s": round(p.npoints / t / 1e9, 3),
                    "host_device_gbs": round(moved / t / 1e9, 2)}

        rec = {"points": p.npoints, "host_device_bytes": moved, "bulk": run_mode(bulk=True), "overlapped": {}}
        for c in chunks:
            rec["overlapped"]["chunk%d" % c] = run_mode(chunk=c, nbuffers=3)
        best = min(rec["overlapped"].values(), key=lambda r: r["s"])
        rec["best_overlapped_gpoints_per_s"] = best["gpoints_per_s"]
        rec["overlap_speedup"] = round(rec["bulk"]["s"] / best["s"], 3)
        log("streaming", name, rec)
        out[name] = rec
        del ins, outs
        import gc
        gc.collect()
        if hasattr(torch._C, "_host_emptyCache"):
            torch._C._host_emptyCache()   # return the cached pinned blocks before the next size
    return out


def batched_leg(dev, stream, f64_gpts, log, replays=100, tuning=None, per_domain=True):
    """384 uneven subdomains, FP64 and FP32: autotuned launch, one
    graph-captured timestep (perturb u, v; refill halos; advect; recorded
    through the library's graph entry points) replayed
    `replays` times, compared with the same timestep as one pw_advect launch
    per domain."""
    import torch
    from paper_2107_13500_amd import batched as BT
    from paper_2107_13500_amd import binding as B
    from paper_2107_13500_amd import inputs, metrics, tune

    t0 = time.perf_counter()
    specs = inputs.batched_specs()
    probs = [inputs.make_domain(sp) for sp in specs]
    log("batched inputs: %d domains generated in %.1f s" % (len(probs), time.perf_counter() - t0))
    out, keep = {}, {}
    for storage in (B.F64, B.F32):
        name = B.DTYPE_NAMES[storage]
        batch = BT.DeviceBatch(probs, storage, dev)
        npts = batch.npoints
        if tuning is None:
            log("batched", name, "autotuning")
            tun, tms, hit = tune.tuning_for(batch, reps=5)
        else:
            tun, hit = dict(tuning), None
        plan = batch.plan(tun)
        log("batched", name, "plan", plan.info())
        eager_ms = time_steps(lambda: batch.advect(plan, stream), 20, 5, stream)
        g = batch.capture_timestep(plan, seed=inputs.SEED_BASE, amplitude=1e-3)
        graph_ms = time_steps(lambda: g.launch(stream), replays, 3, stream)
        log("batched", name, "graph timestep %.4f ms" % graph_ms)
        per_dom_ms, gp, plans = None, None, None
        if per_domain:
            # baseline: the same timestep with one pw_advect launch per domain,
            # also as a graph
            plans = batch.per_domain_plans()
            torch.cuda.synchronize()

            def per_domain_step(rs):
                batch.perturb(plan, inputs.SEED_BASE + 1, 1e-3, rs)
                batch.fill_halo(plan, rs)
                batch.advect_per_domain(plans, rs)

            gp = B.Graph.record(per_domain_step)
            per_dom_ms = time_steps(lambda: gp.launch(stream), 20, 3, stream)
            log("batched", name, "per-domain launches %.4f ms" % per_dom_ms)
        ebytes = metrics.ELEM_BYTES[name]
        abytes = sum(metrics.algorithmic_bytes(pp.nx, pp.ny, pp.nz, ebytes) for pp in probs)
        rec = {"domains": len(probs), "points": npts, "tuning": tun, "tuning_from_cache": hit,
               "advect_ms": round(eager_ms, 5),
               "gpoints_per_s": round(npts / (eager_ms * 1e-3) / 1e9, 3),
               "hbm_frac": round(abytes / (eager_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "graph_timestep_ms": round(graph_ms, 5), "graph_replays": replays,
               "per_domain_launch_timestep_ms": None if per_dom_ms is None else round(per_dom_ms, 5),
               "speedup_vs_per_domain_launches": None if per_dom_ms is None else round(per_dom_ms / graph_ms, 3),
               "speedup_vs_plain_f64_rate": round(npts / (eager_ms * 1e-3) / 1e9 / f64_gpts, 3),
               "plan": plan.info()}
        log("batched", name, rec)
        out[name] = rec
        keep[name] = batch
        torch.cuda.synchronize()
        g.close()
        if gp is not None:
            gp.close()
        del g, gp, plans
    return out, keep


def batched_errors(batch, threads, sample=(0, 1, 2, 57, 128, 191, 255, 300, 350, 383)):
    """Max-norm relative error of sampled domains' outputs against the oracle on
    the domains' final (perturbed) fields."""
    import numpy as np
    import oracle
    worst = 0.0
    for d in sample:
        if d >= len(batch.problems):
            continue
        u, v, w = batch.host_fields(d)
        p = batch.problems[d]
        ref = oracle.advect(u, v, w, p.coeffs.tcx, p.coeffs.tcy, *p.coeffs.arrays(), threads=threads)
        for g, r in zip(batch.host_outputs(d), ref):
            gi, ri = g[1:-1, 1:-1], r[1:-1, 1:-1]
            worst = max(worst, float(np.max(np.abs(gi - ri)) / np.max(np.abs(ri))))
    return worst


if __name__ == "__main__":
    main()
