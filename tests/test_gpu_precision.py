"""Reduced-storage forms against the FP64 oracle (GPU): FP32, BF16, FP16 and
int16 storage computed in FP32; int32 fixed point computed in FP64.

Two errors per field, both max-norm relative:
  vs the oracle on the original FP64 fields (what a user sees), and
  vs the oracle on the dequantised inputs (the arithmetic alone): bounded by
  the output type's unit roundoff plus a few FP32 roundings.
"""
import numpy as np
import pytest
import torch

import oracle
import staggered_rule as rule
from gpu_helpers import DEV, max_rel, positive_zeros, say
from paper_2107_13500_amd import binding as B
from paper_2107_13500_amd import inputs, metrics

pytestmark = pytest.mark.gpu

UNIT_ROUNDOFF = {B.F32: 2.0 ** -24, B.BF16: 2.0 ** -8, B.F16: 2.0 ** -11}
ORIG_BOUND = {B.F32: metrics.STORAGE_ERROR_BOUND["f32"], B.BF16: metrics.STORAGE_ERROR_BOUND["bf16"],
              B.F16: metrics.STORAGE_ERROR_BOUND["f16"], B.I16: metrics.STORAGE_ERROR_BOUND["i16"],
              B.I32: metrics.STORAGE_ERROR_BOUND["i32"]}
FIXED = (B.I16, B.I32)
# Arithmetic error of the FP32-compute path against the oracle on the same
# (dequantised) inputs, relative to the largest output: a few FP32 roundings
# of terms no larger than a few times the output (the seeded fields are
# smooth, so the flux differences cancel at most about tenfold): 8 units of
# 2^-24.  The FP64-compute path (int32 storage) gets 8 units of 2^-53 times
# the same cancellation allowance.
FP32_ARITH = 8 * 2.0 ** -24
FP64_ARITH = 80 * 2.0 ** -53


def arith_bound(storage, out_scale, max_abs):
    """Max-norm bound against the oracle on dequantised inputs: the output
    type's rounding plus the compute type's arithmetic."""
    if storage in FIXED:
        return 0.5 / (out_scale * max_abs) + (FP64_ARITH if storage == B.I32 else FP32_ARITH)
    return UNIT_ROUNDOFF[storage] + FP32_ARITH


def run_storage(p, storage, tuning=None):
    ins, outs = inputs.storage_scales(p, B.DTYPE_NAMES[storage])
    sc = B.make_scales(ins, outs)
    fields = [B.to_storage(a, storage, s, DEV) for a, s in zip((p.u, p.v, p.w), ins)]
    tz = [torch.from_numpy(x).to(DEV) for x in p.coeffs.arrays()]
    d = B.DeviceDomain(*fields, p.coeffs.tcx, p.coeffs.tcy, *tz, scales=sc)
    plan = B.Plan(storage, [B.shape_of(fields[0])], tuning)
    d.run(plan)
    torch.cuda.synchronize()
    got = [B.from_storage(o, storage, s) for o, s in zip(d.outputs, outs)]
    deq = [B.from_storage(f, storage, s) for f, s in zip(fields, ins)]
    return got, deq, outs


@pytest.mark.parametrize("storage", [B.F32, B.BF16, B.F16, B.I16, B.I32], ids=["f32", "bf16", "f16", "i16", "i32"])
@pytest.mark.parametrize("shape", [(64, 64, 64), (37, 29, 96), (9, 5, 128)], ids=lambda s: "x".join(map(str, s)))
def test_reduced_storage_error_bounds(storage, shape):
    p = inputs.make_problem(*shape, seed=1234 + shape[0])
    got, deq, out_scales = run_storage(p, storage)
    ref_orig = oracle.advect_problem(p)
    c = p.coeffs
    ref_deq = oracle.advect(*deq, c.tcx, c.tcy, *c.arrays())
    for name, g, ro, rd, os_ in zip(("su", "sv", "sw"), got, ref_orig, ref_deq, out_scales):
        gi = g[1:-1, 1:-1]
        assert positive_zeros(gi[:, :, 0]), "%s: k = 1 must be exactly +0" % name
        if name == "sw":
            assert positive_zeros(gi[:, :, -1]), "sw(nz) must be exactly +0"
        e_orig = max_rel(gi, ro[1:-1, 1:-1])
        e_deq = max_rel(gi, rd[1:-1, 1:-1])
        say(B.DTYPE_NAMES[storage], shape, name, "vs original %.3e, vs dequantised %.3e" % (e_orig, e_deq))
        # output quantum (fixed point: half of 1/out_scale; floating: the
        # type's unit roundoff) relative to the largest output, plus the
        # compute type's arithmetic
        bound = arith_bound(storage, os_, np.max(np.abs(rd[1:-1, 1:-1])))
        assert e_deq <= bound, "%s arithmetic error %.3e > %.3e" % (name, e_deq, bound)
        assert e_orig <= ORIG_BOUND[storage], "%s error vs FP64 oracle %.3e" % (name, e_orig)


TILINGS = [{"variant": B.VARIANT_MARCH, "chunk": 256, "seg": 1}, {"variant": B.VARIANT_MARCH, "chunk": 512, "seg": 3},
           {"variant": B.VARIANT_MARCH, "chunk": 1024, "seg": 2}, {"variant": B.VARIANT_MARCH, "chunk": 1024, "seg": 64},
           {"variant": B.VARIANT_DIRECT}]


@pytest.mark.parametrize("storage", [B.F32, B.BF16, B.F16, B.I16, B.I32], ids=["f32", "bf16", "f16", "i16", "i32"])
@pytest.mark.parametrize("shape", [(37, 29, 64), (20, 9, 96), (13, 6, 128), (7, 13, 72), (5, 3, 30), (6, 75, 64)],
                         ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("tuning", TILINGS, ids=["m256s1", "m512s3", "m1024s2", "m1024s64", "direct"])
def test_reduced_storage_tilings(storage, shape, tuning):
    """Every tiling (one or two pairs of levels per thread, single points,
    one-plane segments, ragged last chunks, run-time heights) within the
    arithmetic bound against the oracle on the dequantised inputs."""
    p = inputs.make_problem(*shape, seed=2300 + shape[0] + shape[2])
    got, deq, out_scales = run_storage(p, storage, tuning)
    c = p.coeffs
    ref_deq = oracle.advect(*deq, c.tcx, c.tcy, *c.arrays())
    for name, g, rd, os_ in zip(("su", "sv", "sw"), got, ref_deq, out_scales):
        gi = g[1:-1, 1:-1]
        assert positive_zeros(gi[:, :, 0]), "%s: k = 1 must be exactly +0" % name
        if name == "sw":
            assert positive_zeros(gi[:, :, -1]), "sw(nz) must be exactly +0"
        e = max_rel(gi, rd[1:-1, 1:-1])
        bound = arith_bound(storage, os_, np.max(np.abs(rd[1:-1, 1:-1])))
        assert e <= bound, "%s %s %s: %.3e > %.3e" % (B.DTYPE_NAMES[storage], tuning, name, e, bound)



@pytest.mark.parametrize("storage", [B.I16, B.I32], ids=["i16", "i32"])
@pytest.mark.parametrize("tuning", [{"variant": B.VARIANT_MARCH, "chunk": 512, "seg": 4}, {"variant": B.VARIANT_DIRECT}],
                         ids=["march", "direct"])
def test_fixed_point_outputs_round_and_saturate(storage, tuning):
    """Output scales 64 times too large for the type: results beyond the range
    store its limits, the others round to the nearest integer."""
    p = inputs.make_problem(21, 11, 64, seed=4321)
    ins, outs = inputs.storage_scales(p, B.DTYPE_NAMES[storage])
    outs = [s * 64.0 for s in outs]
    fields = [B.to_storage(a, storage, s, DEV) for a, s in zip((p.u, p.v, p.w), ins)]
    tz = [torch.from_numpy(x).to(DEV) for x in p.coeffs.arrays()]
    d = B.DeviceDomain(*fields, p.coeffs.tcx, p.coeffs.tcy, *tz, scales=B.make_scales(ins, outs))
    d.run(B.Plan(storage, [B.shape_of(fields[0])], tuning))
    torch.cuda.synchronize()
    c = p.coeffs
    deq = [B.from_storage(f, storage, s) for f, s in zip(fields, ins)]
    ref = oracle.advect(*deq, c.tcx, c.tcy, *c.arrays())
    lo, hi = B.FIXED_RANGE[storage]
    for name, o, r, s in zip(("su", "sv", "sw"), d.outputs, ref, outs):
        g = o.cpu().numpy()[1:-1, 1:-1].astype(np.int64)
        x = r[1:-1, 1:-1] * s
        # half a unit for the rounding, plus the compute type's error relative
        # to the largest result; results farther than that from a limit must
        # saturate or stay in range
        tol = 0.5 + (FP64_ARITH if storage == B.I32 else FP32_ARITH) * np.max(np.abs(x))
        over, under = x > hi + tol, x < lo - tol
        assert over.any() and under.any(), "%s: the scale must push results out of range" % name
        assert np.all(g[over] == hi) and np.all(g[under] == lo), "%s: saturation" % name
        inside = (x > lo + tol) & (x < hi - tol)
        assert inside.any()
        err = np.max(np.abs(g[inside] - x[inside]))
        say(B.DTYPE_NAMES[storage], tuning, name, "in-range error %.3f units (bound %.3f)" % (err, tol))
        assert err <= tol, "%s: %.3f > %.3f" % (name, err, tol)

def naive_fp32(u, v, w, co, nx, ny, nz):
    """The staggering rule evaluated term by term in np.float32 (products
    first, then their difference: no compensation), every computed point."""
    F = rule.Fields(u, v, w, co.tcx, co.tcy, *co.arrays(), conv=np.float32)
    shp = u.shape
    out = {n: np.zeros(shp) for n in "uvw"}
    for i in range(1, nx + 1):
        for j in range(1, ny + 1):
            for k in range(1, nz + 1):
                for n in "uvw":
                    out[n][i, j, k - 1] = float(rule.source(F, n, (k, j, i)))
    return [out[n] for n in "uvw"]


def pow2_coefficients(nz, tc=2.0 ** -10, tz=2.0 ** -8):
    """Uniform coefficients that are powers of two (tzc1 = tzc2, tzd1 = tzd2),
    so every coefficient product is exact and uniform fields give exactly
    zero: the flux differences then cancel as much as the fields do."""
    one = np.full(nz, tz)
    one[0] = 0.0
    d = one.copy()
    d[-1] = 0.0
    return inputs.Coefficients(tc, tc, one.copy(), one.copy(), d.copy(), d.copy())


def test_fp32_difference_first_beats_naive_fp32_on_cancelling_fields():
    """u = 50 + N(0, 0.01), v = 20 + N(0, 0.01), w = 30 + N(0, 0.01) with
    uniform power-of-two coefficients: every flux difference of su, sv and sw
    cancels about 10^3-fold.  Naive FP32 (the staggering rule in np.float32)
    loses about three digits; the library's difference-first FP32 stays within
    a few FP32 roundings of the result."""
    nx, ny, nz = 6, 5, 8
    rng = np.random.default_rng(77)
    shp = (nx + 2, ny + 2, nz)
    u = (50.0 + 0.01 * rng.standard_normal(shp)).astype(np.float32).astype(np.float64)
    v = (20.0 + 0.01 * rng.standard_normal(shp)).astype(np.float32).astype(np.float64)
    w = (30.0 + 0.01 * rng.standard_normal(shp)).astype(np.float32).astype(np.float64)
    co = pow2_coefficients(nz)
    p = inputs.Problem(nx, ny, nz, u, v, w, co, inputs.vertical_grid(nz))
    got, deq, _ = run_storage(p, B.F32)
    ref = oracle.advect(u, v, w, co.tcx, co.tcy, *co.arrays())
    naive = naive_fp32(u, v, w, co, nx, ny, nz)
    # levels 2 .. nz-1: at the column top su and sv keep only the lower
    # vertical flux, which does not cancel and would dominate the max norm
    inner = (slice(1, -1), slice(1, -1), slice(1, nz - 1))
    for name, g, r, nv in zip("uvw", got, ref, naive):
        e_gpu = max_rel(g[inner], r[inner])
        e_naive = max_rel(nv[inner], r[inner])
        say("cancelling s%s: library FP32 %.2e, naive FP32 %.2e" % (name, e_gpu, e_naive))
        assert e_gpu <= UNIT_ROUNDOFF[B.F32] + FP32_ARITH
        assert e_naive >= 20 * e_gpu, "s%s: compensation gains nothing (%.2e vs %.2e)" % (name, e_gpu, e_naive)


def checkerboard_fields(nx, ny, nz, big, small, quantum_big, quantum_small, seed, spread=1):
    """Stored values exactly representable in the 16-bit type: a 3-D
    checkerboard of `big` and `small` magnitudes (parity of i + j + k) with
    random offsets of up to `spread` quanta.  Neighbours along any axis differ in
    magnitude, so each sum of two neighbours carries the bits of both and
    the products of the flux terms need more than FP32's 24 bits; values two
    apart along an axis have the same parity, so each flux difference
    cancels about a thousandfold."""
    rng = np.random.default_rng(seed)
    shp = (nx + 2, ny + 2, nz)
    ii, jj, kk = np.meshgrid(np.arange(shp[0]), np.arange(shp[1]), np.arange(shp[2]), indexing="ij")
    even = (ii + jj + kk) % 2 == 0
    out = []
    for f in range(3):
        a = np.where(even, big[f] + quantum_big * rng.integers(-spread, spread + 1, shp),
                     small[f] + quantum_small * rng.integers(-3 * spread, 3 * spread + 1, shp))
        out.append(a.astype(np.float64))
    return out


def correctly_rounded(x, storage, out_scale):
    """Exact values x (FP64 oracle) rounded to the stored output as the
    library's contract says: scaled, then round to nearest even (fixed point
    also saturated)."""
    t = torch.from_numpy(x * out_scale)
    if storage in FIXED:
        return torch.round(t).clamp_(*B.FIXED_RANGE[storage]).to(B.torch_dtype(storage))
    return t.to(B.torch_dtype(storage))


@pytest.mark.parametrize("storage", [B.F16, B.I16], ids=["f16", "i16"])
def test_kahan_product_differences_round_correctly_where_naive_fp32_does_not(storage):
    """16-bit storage computes each product difference E F - G H by Kahan's
    algorithm.  On fields whose flux differences cancel a thousandfold while
    the products need more than 24 bits, the stored su, sv and sw must be the
    correctly rounded exact results (FP64 oracle on the stored inputs,
    scaled and rounded to the output type) at almost every point, while the
    naive FP32 evaluation of the same rule, rounded the same way, is wrong at
    a large share of them."""
    nx, ny, nz = 6, 5, 64
    if storage == B.F16:
        # FP16: 1024 + integers (quantum 1) next to 4 + multiples of 2^-8
        fields = checkerboard_fields(nx, ny, nz, (1024.0, 1536.0, 1280.0), (4.0, 6.0, 5.0), 1.0, 2.0 ** -8, 91)
    else:
        # int16: 24000 + integers next to 100 + integers
        fields = checkerboard_fields(nx, ny, nz, (24000.0, 20000.0, 16000.0), (100.0, 80.0, 60.0), 1.0, 1.0, 92)
    co = pow2_coefficients(nz)
    exact = oracle.advect(*fields, co.tcx, co.tcy, *co.arrays())
    # inputs stored as they are (scale 1, every value representable); output
    # scales put the largest result of levels 2 .. nz-1 near 2^14 (the column
    # top keeps only the lower vertical flux, which does not cancel: it is
    # left out of the scales and the statistics, and may saturate)
    inner = (slice(1, -1), slice(1, -1), slice(1, nz - 1))
    out_scales = tuple(inputs.pow2_scale(float(np.max(np.abs(r[inner])))) for r in exact)
    sc = B.make_scales((1.0, 1.0, 1.0), out_scales)
    stored = [B.to_storage(a, storage, 1.0, DEV) for a in fields]
    for a, st in zip(fields, stored):
        assert np.array_equal(st.double().cpu().numpy(), a), "inputs must be exactly representable"
    tz = [torch.from_numpy(x).to(DEV) for x in co.arrays()]
    d = B.DeviceDomain(*stored, co.tcx, co.tcy, *tz, scales=sc)
    d.run(B.Plan(storage, [B.shape_of(stored[0])]))
    torch.cuda.synchronize()
    naive = naive_fp32(*fields, co, nx, ny, nz)
    for name, g, r, nv, os_ in zip("uvw", d.outputs, exact, naive, out_scales):
        want = correctly_rounded(r, storage, os_)[inner]
        got = g.cpu()[inner]
        naive_s = correctly_rounded(nv, storage, os_)[inner]
        lib_wrong = float((got != want).double().mean())
        naive_wrong = float((naive_s != want).double().mean())
        say("%s s%s: not correctly rounded: library %.4f, naive FP32 %.4f of %d points"
            % (B.DTYPE_NAMES[storage], name, lib_wrong, naive_wrong, want.numel()))
        assert lib_wrong <= 0.01, "s%s: %.3f of the library's outputs are not correctly rounded" % (name, lib_wrong)
        assert naive_wrong >= 0.05 and naive_wrong >= 5 * lib_wrong, \
            "s%s: the fields do not separate compensated from naive FP32 (%.3f vs %.3f)" % (name, lib_wrong, naive_wrong)


@pytest.mark.parametrize("tuning", [None, {"variant": B.VARIANT_DIRECT}], ids=["march", "direct"])
def test_fp32_storage_keeps_denormal_results(tuning):
    """Fields scaled by 2^-64 (exactly; still normal FP32 values) put every FP32
    output below 2^-126, in the denormal range, and the products of the flux
    terms with them.  With no flush to zero anywhere, the results follow the
    oracle on the same stored inputs to within a few denormal spacings
    (2^-149) plus the usual relative error; a flush would return zeros."""
    p = inputs.make_problem(24, 20, 64, seed=4242)
    s = 2.0 ** -64
    fields = [B.to_storage(a * s, B.F32, 1.0, DEV) for a in (p.u, p.v, p.w)]
    c = p.coeffs
    tz = [torch.from_numpy(x).to(DEV) for x in c.arrays()]
    d = B.DeviceDomain(*fields, c.tcx, c.tcy, *tz)
    d.run(B.Plan(B.F32, [B.shape_of(fields[0])], tuning))
    torch.cuda.synchronize()
    deq = [f.double().cpu().numpy() for f in fields]
    ref = oracle.advect(*deq, c.tcx, c.tcy, *c.arrays())
    for name, o, r in zip(("su", "sv", "sw"), d.outputs, ref):
        g = o.double().cpu().numpy()[1:-1, 1:-1]
        ri = r[1:-1, 1:-1]
        m = np.max(np.abs(ri))
        assert 2.0 ** -140 < m < 2.0 ** -126, "%s: outputs must lie in the denormal range (max %.3e)" % (name, m)
        live = ri != 0
        assert np.count_nonzero(g[live]) >= 0.99 * np.count_nonzero(live), "%s: denormal results flushed" % name
        err = np.max(np.abs(g - ri))
        bound = 8 * 2.0 ** -149 + (UNIT_ROUNDOFF[B.F32] + FP32_ARITH) * m
        say("f32 denormal", name, tuning, "max %.3e err %.3e bound %.3e" % (m, err, bound))
        assert err <= bound, "%s: %.3e > %.3e" % (name, err, bound)
