"""Build the HIP library ``libpwadvect.so`` for gfx950 with hipcc.

    python -m paper_2107_13500_amd.build

Compiles every source under ``csrc/`` into one shared library next to this
file.  Flags: ``-O3``; fused multiply-add formed only within a source
expression (``-ffp-contract=on``); packed FP32 instructions disabled
(hand-written code never uses them and the compiler must not form them
either); no fast-math.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBRARY = os.path.join(HERE, "libpwadvect.so")
SOURCES = ["pw_advect.hip", "pw_batched.hip", "pw_graph.hip", "pw_tune.hip", "pw_stream.hip", "pw_probe.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    # fuse a*b + c only within one source expression: the rounding then
    # depends on the source alone, not on the code around it, so every
    # kernel variant that shares the per-point code rounds identically
    "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-I", INCLUDE,
    "-I", CSRC,
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra=()) -> str:
    """Compile all sources and link ``libpwadvect.so`` (always rebuilds)."""
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="pwadv_build_") as tmp:
        jobs = []
        for src in SOURCES:
            path = os.path.join(CSRC, src)
            if not os.path.exists(path):
                continue
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            jobs.append(([cc, *HIPCC_FLAGS, *extra, "-c", path, "-o", obj], obj))
            if verbose:
                print(" ".join(jobs[-1][0]), flush=True)
        # one compiler process per source file, in parallel
        workers = max(1, min(len(jobs), os.cpu_count() or 1, 8))
        with ThreadPoolExecutor(max_workers=workers) as ex:
            for f in [ex.submit(subprocess.run, cmd, check=True) for cmd, _ in jobs]:
                f.result()
        objs = [obj for _, obj in jobs]
        out_tmp = LIBRARY + ".tmp%d" % os.getpid()
        cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", out_tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out_tmp, LIBRARY)
    return LIBRARY


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
