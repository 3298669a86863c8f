"""Autotuner front end: a persistent cache of the library's tuning decisions.

The search itself is ``pw_autotune`` in the HIP library (it times candidate
launch shapes on the caller's buffers).  This module keys its answers by GPU
architecture, HIP version, the built library, storage type and problem shape,
and keeps them in
a JSON file (``$PW_TUNE_CACHE``, else ``~/.cache/pwadvect/tune.json``) so a
later run reuses them without searching again.

    python -m paper_2107_13500_amd.tune --workload batched384 --storage f64
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
from typing import Optional

from . import binding as B


def cache_path() -> str:
    p = os.environ.get("PW_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "pwadvect", "tune.json")


def load_cache(path: Optional[str] = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_entry(key: str, entry: dict, path: Optional[str] = None) -> None:
    """Merge one entry into the cache file (atomic replace)."""
    path = path or cache_path()
    data = load_cache(path)
    data[key] = entry
    d = os.path.dirname(path) or "."
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".tune", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_key() -> str:
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "nogpu"
    return "%s|hip%s" % (arch, torch.version.hip)


def library_key() -> str:
    """Hash of the built HIP library: a rebuilt library (new kernels, a new
    candidate space) searches again instead of reusing an older choice."""
    with open(B.LIBRARY, "rb") as f:
        return "lib" + hashlib.sha256(f.read()).hexdigest()[:12]


def shape_key(storage: int, shapes) -> str:
    desc = ";".join("%d,%d,%d,%d,%d" % (s.nx, s.ny, s.nz, s.sy, s.sx) for s in shapes)
    if len(shapes) == 1:
        return "%s|%s" % (B.DTYPE_NAMES[storage], desc)
    return "%s|batch%d|%s" % (B.DTYPE_NAMES[storage], len(shapes), hashlib.sha1(desc.encode()).hexdigest()[:16])


def tuning_for(batch, reps: int = 5, candidates=None, path: Optional[str] = None, force: bool = False):
    """Cached tuning of a ``batched.DeviceBatch`` (one or many domains); searches on a miss."""
    from . import batched
    key = device_key() + "|" + library_key() + "|" + shape_key(batch.storage, batch.shapes)
    cache = load_cache(path)
    if not force and key in cache and isinstance(cache[key].get("tuning"), dict):
        return cache[key]["tuning"], cache[key].get("ms"), True
    best, ms, table = batched.autotune(batch, candidates, reps)
    save_entry(key, {"tuning": best, "ms": ms, "candidates": len(table)}, path)
    return best, ms, False


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", default="batched384", choices=["pw512", "pw2048", "batched384"])
    ap.add_argument("--storage", default="f64", choices=["f64", "f32", "bf16", "f16"])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--force", action="store_true", help="search even if the cache has an answer")
    args = ap.parse_args(argv)
    import torch

    from . import batched, inputs
    storage = {"f64": B.F64, "f32": B.F32, "bf16": B.BF16, "f16": B.F16}[args.storage]
    if args.workload == "batched384":
        problems = [inputs.make_domain(s) for s in inputs.batched_specs()]
    else:
        problems = [inputs.workload(args.workload)]
    batch = batched.DeviceBatch(problems, storage, "cuda:0")
    tuning, ms, hit = tuning_for(batch, reps=args.reps, force=args.force)
    print(json.dumps({"workload": args.workload, "storage": args.storage, "tuning": tuning, "ms": ms,
                      "cached": hit, "cache": cache_path()}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
