"""Helpers for the GPU tests: seeded problems on the device, comparison with the oracle."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from paper_2107_13500_amd import binding as B
from paper_2107_13500_amd import inputs

DEV = "cuda:0"
F64_TOL = 1e-12          # max-norm relative, per field

SENTINEL = {torch.float64: -7.25e300, torch.float32: -7.25e30, torch.bfloat16: -7.25e30, torch.float16: -6.0e4,
            torch.int16: -32000}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def device_domain(p: inputs.Problem, storage: int = B.F64, scales=None, sentinel=True):
    dt = B.torch_dtype(storage)
    ins = (1.0, 1.0, 1.0) if scales is None else tuple(scales.in_scale)
    u, v, w = (B.to_storage(a, storage, s, DEV) for a, s in zip((p.u, p.v, p.w), ins))
    c = p.coeffs
    tz = [torch.from_numpy(x).to(DEV) for x in c.arrays()]
    d = B.DeviceDomain(u, v, w, c.tcx, c.tcy, *tz, scales=scales)
    if sentinel:
        for o in d.outputs:
            o.fill_(SENTINEL[dt])
    return d


_BITS = {torch.float64: torch.int64, torch.float32: torch.int32, torch.bfloat16: torch.int16,
         torch.float16: torch.int16}


def same_bits(a: torch.Tensor, b: torch.Tensor) -> bool:
    """Bit-for-bit equality (torch.equal compares values, so +0 and -0 would pass)."""
    if a.dtype != b.dtype or a.shape != b.shape:
        return False
    if a.dtype in _BITS:
        a = a.contiguous().view(_BITS[a.dtype])
        b = b.contiguous().view(_BITS[b.dtype])
    return torch.equal(a, b)


def positive_zeros(x: np.ndarray) -> bool:
    """Every element is +0.0 (value zero, sign bit clear)."""
    return bool(np.all(x == 0.0) and not np.any(np.signbit(x)))


def max_rel(g: np.ndarray, o: np.ndarray) -> float:
    den = np.max(np.abs(o))
    return float(np.max(np.abs(g - o)) / den) if den > 0 else float(np.max(np.abs(g)))


def check_halo_untouched(d: B.DeviceDomain):
    dt = d.su.dtype
    for o in d.outputs:
        for face in (o[0], o[-1], o[:, 0], o[:, -1]):
            assert torch.all(face == SENTINEL[dt]).item(), "an output halo column was written"


def compare_f64(d: B.DeviceDomain, ref, tol: float = F64_TOL, where: str = ""):
    """Element-wise comparison of the device outputs with oracle outputs."""
    errs = []
    for name, g_t, o in zip(("su", "sv", "sw"), d.outputs, ref):
        g = g_t.cpu().numpy()
        gi, oi = g[1:-1, 1:-1], o[1:-1, 1:-1]
        assert positive_zeros(gi[:, :, 0]), "%s %s: k = 1 must be exactly +0" % (where, name)
        if name == "sw":
            assert positive_zeros(gi[:, :, -1]), "%s: sw(nz) must be exactly +0" % where
        e = max_rel(gi, oi)
        errs.append(e)
        assert e <= tol, "%s %s: max-norm relative error %.3e > %.1e" % (where, name, e, tol)
    return errs


def sampled_columns(nx, ny, n_random=160, seed=11, extra_i=()):
    """Interior columns (i, j) to check one by one: first and last columns,
    chunk boundaries (8 columns of 64 levels per 512-point chunk), segment
    boundaries (128 planes) and `extra_i` planes, plus random columns."""
    ii = {1, 2, 127, 128, 129, 130, nx // 2, nx - 1, nx} | set(extra_i)
    jj = {1, 2, 8, 9, 16, 17, ny // 2, ny - 8, ny - 7, ny - 1, ny}
    cols = {(i, j) for i in ii for j in jj if 1 <= i <= nx and 1 <= j <= ny}
    rng = np.random.default_rng(seed)
    cols |= set(zip(rng.integers(1, nx + 1, n_random).tolist(), rng.integers(1, ny + 1, n_random).tolist()))
    return sorted(cols)


def column_oracle(fields, scales, coeffs, cols):
    """FP64 oracle outputs (ncols, nz) per field at the sampled columns, from
    each column's 3 x 3-column neighbourhood of the given (stored) fields."""
    out = [[], [], []]
    for i, j in cols:
        nb = [t[i - 1:i + 2, j - 1:j + 2, :].to(torch.float64).cpu().numpy() / s for t, s in zip(fields, scales)]
        r = oracle.advect(*[np.ascontiguousarray(a) for a in nb], coeffs.tcx, coeffs.tcy, *coeffs.arrays())
        for f in range(3):
            out[f].append(r[f][1, 1, :])
    return [np.stack(o) for o in out]
