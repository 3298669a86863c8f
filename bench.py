#!/usr/bin/env python3
"""Benchmark of the MI355X PW advection library.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload pw2048]

One step is one call of the whole stencil (su, sv and sw of every point of
one domain) on the 2048 x 2048 x 64 FP64 grid, inputs resident in HBM.  Rank
0 prints one JSON line: Gpoints/s, the HBM roofline of the kernel (algorithmic
bytes / measured kernel time against the 8 TB/s peak), the CPU oracle timed on
the host cores, the storage-precision variants (FP32, BF16, FP16 with FP32
compensated compute) with their error against the FP64 oracle, and the
batched many-subdomain form.
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


def copy_ceiling(gbytes, steps, warmup, dev, stream):
    """Read+write bandwidth of a plain device-to-device copy (torch's copy kernel)."""
    import torch
    n = int(gbytes * 1e9) // 8
    a = torch.empty(n, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    ms = time_steps(lambda: b.copy_(a), steps, warmup, stream)
    moved = 2 * n * 8
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_copy": moved, "ms": round(ms, 5), "gbs": round(moved / (ms * 1e-3) / 1e9, 1)}


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


def cpu_baseline(p, threads):
    """The FP64 oracle on the same grid, timed on the host; returns (record, reference outputs)."""
    import oracle
    reps = 2
    t0 = time.perf_counter()
    ref = None
    for _ in range(reps):
        ref = oracle.advect_problem(p, threads=threads)
    dt = (time.perf_counter() - t0) / reps
    rec = {"value": p.npoints / dt / 1e9, "unit": "Gpoints/s", "cores": threads, "kind": "oracle",
           "sample": "full %dx%dx%d grid, %d oracle calls (plain C FP64, no FMA), %d OpenMP threads, "
                     "%.2f s per call" % (p.nx, p.ny, p.nz, reps, threads, dt)}
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
        print("bench.py: this build measures one GPU only (the stencil kernel on one GPU's domain); "
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
    u, v, w = (torch.from_numpy(a).to(dev) for a in (p.u, p.v, p.w))
    d64 = B.DeviceDomain(u, v, w, c.tcx, c.tcy, *tz)
    plan = B.Plan(B.F64, [B.shape_of(u)], tuning)
    info = plan.info()
    log("plan", info)
    ms = time_steps(lambda: d64.run(plan, stream), args.steps, args.warmup, stream)
    gpts = p.npoints / (ms * 1e-3) / 1e9
    abytes = metrics.algorithmic_bytes(nx, ny, nz, 8)
    achieved = abytes / (ms * 1e-3) / 1e9
    log("FP64: %.4f ms/step, %.2f Gpts/s, %.1f GB/s algorithmic" % (ms, gpts, achieved))

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
    }

    if info["variant"] == B.VARIANT_MARCH:
        t = measured_traffic("pw_march_f64_%s" % args.workload, info["chunk"], info["seg"])
        result["roofline"]["traffic"] = None if t is None else int(round(t))

    ceiling = copy_ceiling(2.0, 10, 3, dev, stream)
    result["roofline"]["copy_ceiling_gbs"] = ceiling["gbs"]
    result["roofline"]["frac_of_copy_ceiling"] = round(achieved / ceiling["gbs"], 4)
    log("copy ceiling", ceiling)

    # ---------------- CPU oracle baseline ----------------
    ref = None
    if not args.skip_cpu:
        usable = len(os.sched_getaffinity(0))
        threads = args.cpu_threads or min(usable, 16)
        rec, ref = cpu_baseline(p, threads)
        result["cpu_baseline"] = rec
        log("oracle: %.3f Gpts/s on %d threads" % (rec["value"], threads))
        torch.cuda.synchronize()
        result["parity_f64"] = errors_vs(ref, d64.outputs, (1.0, 1.0, 1.0), nx, ny)
        log("FP64 parity", result["parity_f64"]["max_rel"])
    del d64, u, v, w
    torch.cuda.empty_cache()

    # ---------------- storage-precision variants ----------------
    if not args.skip_variants:
        variants = {}
        for storage in (B.F32, B.BF16, B.F16):
            name = B.DTYPE_NAMES[storage]
            dt = B.torch_dtype(storage)
            if storage == B.F16:
                ins = tuple(inputs.pow2_scale(float(np.max(np.abs(a)))) for a in (p.u, p.v, p.w))
                outs_s = inputs.fp16_output_scales(p)
            else:
                ins, outs_s = (1.0, 1.0, 1.0), (1.0, 1.0, 1.0)
            sc = B.make_scales(ins, outs_s)
            fu, fv, fw = (torch.from_numpy(a).to(dev).mul_(s).to(dt) for a, s in zip((p.u, p.v, p.w), ins))
            dd = B.DeviceDomain(fu, fv, fw, c.tcx, c.tcy, *tz, scales=sc)
            pl = B.Plan(storage, [B.shape_of(fu)], tuning)
            vms = time_steps(lambda: dd.run(pl, stream), args.steps, args.warmup, stream)
            eb = metrics.ELEM_BYTES[name]
            vb = metrics.algorithmic_bytes(nx, ny, nz, eb)
            rec = {"gpoints_per_s": round(p.npoints / (vms * 1e-3) / 1e9, 3), "ms_per_step": round(vms, 5),
                   "speedup_vs_f64": round(ms / vms, 3),
                   "hbm_frac": round(vb / (vms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "in_scale": list(ins), "out_scale": list(outs_s)}
            if ref is not None:
                rec["error_vs_f64_oracle"] = errors_vs(ref, dd.outputs, outs_s, nx, ny)
            variants[name] = rec
            log(name, rec)
            del dd, fu, fv, fw, pl
            torch.cuda.empty_cache()
        result["precision"] = variants

    # ---------------- batched subdomains ----------------
    if not args.skip_batched:
        try:
            from paper_2107_13500_amd import batched_bench
            result["batched"] = batched_bench.run(dev, stream, log)
        except ImportError:
            pass

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
