"""CPU oracle of the PW advection stencil (plain C, FP64) and its ctypes loader.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg are the only callers.  The product (the HIP
library under ``paper_2107_13500_amd``) never imports this package, and this
package imports nothing from the product; inputs come from the shared seeded
generator module ``paper_2107_13500_amd.inputs``, which holds no stencil
arithmetic.

The C source, ``pw_oracle.c``, states what is computed and which passage of
the paper (Sec. II-A, Listing 1; Sec. III op counts) each part follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "pw_oracle.c")
LIBRARY = os.path.join(_HERE, "libpw_oracle.so")

# No contraction into fused multiply-adds, no fast-math: the textual order of
# the source is the rounding order.  OpenMP only splits the outer x loop.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp"]

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libpw_oracle.so``."""
    global _lib
    if not force and os.path.exists(LIBRARY):
        return LIBRARY
    tmp = LIBRARY + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, SOURCE, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIBRARY)
    _lib = None
    return LIBRARY


def bind(path: str):
    """Load a compiled oracle library and declare its entry point."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.pw_oracle_f64.restype = ctypes.c_int32
    lib.pw_oracle_f64.argtypes = [
        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
        dp, dp, dp, dp, dp, dp,
        ctypes.c_double, ctypes.c_double,
        dp, dp, dp, dp,
        ctypes.c_int32,
    ]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY) or os.path.getmtime(LIBRARY) < os.path.getmtime(SOURCE):
            build()
        _lib = bind(LIBRARY)
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _strides(a: np.ndarray) -> Tuple[int, int]:
    """(sy, sx) element strides of a (nx+2, ny+2, nz) float64 view with unit k stride."""
    if a.dtype != np.float64 or a.ndim != 3 or a.strides[2] != 8:
        raise ValueError("oracle arrays must be float64 (nx+2, ny+2, nz) views with contiguous k")
    return a.strides[1] // 8, a.strides[0] // 8


def advect(u: np.ndarray, v: np.ndarray, w: np.ndarray,
           tcx: float, tcy: float,
           tzc1: np.ndarray, tzc2: np.ndarray, tzd1: np.ndarray, tzd2: np.ndarray,
           out: Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]] = None,
           threads: int = 1, lib=None):
    """su, sv, sw for halo'd float64 fields of shape (nx+2, ny+2, nz).

    Outputs have the inputs' shape; their halo columns are left as allocated
    (zeros unless ``out`` is given).  Sub-views are accepted (e.g. an x-slab
    ``u[i0-1:i1+2]``, which is contiguous, or a y-slab, which is copied first),
    so large grids can be checked in pieces.
    """
    lib = _load() if lib is None else lib
    if not (u.shape == v.shape == w.shape) or u.ndim != 3:
        raise ValueError("u, v, w must share one (nx+2, ny+2, nz) shape")
    nx, ny, nz = u.shape[0] - 2, u.shape[1] - 2, u.shape[2]
    if out is None and not (u.flags.c_contiguous and v.flags.c_contiguous and w.flags.c_contiguous):
        u, v, w = (np.ascontiguousarray(a) for a in (u, v, w))
    sy, sx = _strides(u)
    if _strides(v) != (sy, sx) or _strides(w) != (sy, sx):
        raise ValueError("u, v, w must share strides")
    coef = [np.ascontiguousarray(c, dtype=np.float64) for c in (tzc1, tzc2, tzd1, tzd2)]
    if any(c.shape != (nz,) for c in coef):
        raise ValueError("coefficient arrays must have nz entries")
    if out is None:
        out = tuple(np.zeros(u.shape) for _ in range(3))
    for o in out:
        if o.shape != u.shape or _strides(o) != (sy, sx):
            raise ValueError("outputs must match the inputs' shape and strides")
    rc = lib.pw_oracle_f64(nx, ny, nz, sy, sx, _ptr(u), _ptr(v), _ptr(w),
                           _ptr(out[0]), _ptr(out[1]), _ptr(out[2]),
                           float(tcx), float(tcy), *[_ptr(c) for c in coef], int(threads))
    if rc != 0:
        raise ValueError("pw_oracle_f64 rejected the shape (rc=%d)" % rc)
    return out


def advect_problem(p, threads: int = 1):
    """Convenience: run the oracle on a ``paper_2107_13500_amd.inputs.Problem``."""
    c = p.coeffs
    return advect(p.u, p.v, p.w, c.tcx, c.tcy, c.tzc1, c.tzc2, c.tzd1, c.tzd2, threads=threads)
