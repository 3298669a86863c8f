"""FP64 parity of the HIP kernels with the CPU oracle, through the C ABI (GPU).

Criterion (per field): max |gpu - oracle| / max |oracle| over the computed
points <= 1e-12; level k = 1 and sw(nz) exactly 0; output halo columns never
written (they keep a sentinel).
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import DEV, F64_TOL, check_halo_untouched, compare_f64, device_domain, same_bits, say
from paper_2107_13500_amd import binding as B
from paper_2107_13500_amd import inputs

pytestmark = pytest.mark.gpu

SHAPES = [
    (1, 1, 2), (2, 3, 3), (3, 5, 4), (7, 13, 63), (33, 17, 65), (20, 9, 96),
    (11, 7, 127), (9, 5, 128), (5, 3, 256), (64, 64, 64), (37, 29, 64),
    # 8 or more chunks per plane (compact tile order), counts not a multiple of 8, ragged last chunks
    (6, 75, 64), (5, 41, 96), (4, 160, 65),
]
TUNINGS = [
    {"variant": B.VARIANT_DIRECT},
    {"variant": B.VARIANT_MARCH, "chunk": 256, "seg": 1},
    {"variant": B.VARIANT_MARCH, "chunk": 512, "seg": 3},
    {"variant": B.VARIANT_MARCH, "chunk": 1024, "seg": 64},
    {},
]


def _run(p, tuning, storage=B.F64):
    d = device_domain(p, storage)
    plan = B.Plan(storage, [B.shape_of(d.u)], tuning)
    d.run(plan)
    torch.cuda.synchronize()
    return d, plan


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("tuning", TUNINGS, ids=["direct", "m256s1", "m512s3", "m1024s64", "auto"])
def test_f64_parity_shapes(shape, tuning):
    nx, ny, nz = shape
    say("parity", shape, tuning)
    p = inputs.make_problem(nx, ny, nz, seed=1000 + nx * 7 + ny * 3 + nz)
    ref = oracle.advect_problem(p)
    d, plan = _run(p, tuning)
    compare_f64(d, ref, where="%s %s" % (shape, tuning))
    check_halo_untouched(d)


def test_f64_parity_pw64_all_points():
    p = inputs.workload("pw64")
    ref = oracle.advect_problem(p)
    d, plan = _run(p, {})
    info = plan.info()
    say("pw64 plan", info)
    assert info["variant"] == B.VARIANT_MARCH
    compare_f64(d, ref, where="pw64")
    check_halo_untouched(d)


def test_f64_parity_pw512_all_points():
    p = inputs.workload("pw512")
    ref = oracle.advect_problem(p, threads=8)
    d, plan = _run(p, {})
    errs = compare_f64(d, ref, where="pw512")
    say("pw512 errors", errs, plan.info())


def test_f64_padded_strides_direct():
    """Non-default strides (padded columns and planes) run the direct variant."""
    nx, ny, nz = 6, 5, 10
    p = inputs.make_problem(nx, ny, nz, seed=77)
    sy, sx = nz + 6, (ny + 2) * (nz + 6) + 10
    buf = [torch.full(((nx + 2) * sx,), 3.0e300, dtype=torch.float64) for _ in range(6)]

    def view(t):
        return t.as_strided((nx + 2, ny + 2, nz), (sx, sy, 1))

    for t, a in zip(buf[:3], (p.u, p.v, p.w)):
        view(t).copy_(torch.from_numpy(a))
    dbuf = [t.to(DEV) for t in buf]
    ins = [view(t) for t in dbuf[:3]]
    outs = [view(t) for t in dbuf[3:]]
    c = p.coeffs
    tz = [torch.from_numpy(x).to(DEV) for x in c.arrays()]
    plan = B.Plan(B.F64, [B.shape_of(ins[0])], {})
    assert plan.info()["variant"] == B.VARIANT_DIRECT
    B.advect(plan, *ins, *outs, c.tcx, c.tcy, *tz)
    torch.cuda.synchronize()
    ref = oracle.advect_problem(p)
    for o, r in zip(outs, ref):
        g = o.cpu().numpy()
        assert np.max(np.abs(g[1:-1, 1:-1] - r[1:-1, 1:-1])) <= 1e-12 * np.max(np.abs(r))
    # padding between columns and planes is never written
    for t in dbuf[3:]:
        h = t.cpu().numpy()
        mask = np.ones_like(h, dtype=bool)
        idx = np.arange(nz)[None, None, :] + np.arange(1, ny + 1)[None, :, None] * sy + \
            np.arange(1, nx + 1)[:, None, None] * sx
        mask[idx.ravel()] = False
        assert np.all(h[mask] == 3.0e300)


def test_variants_agree_to_rounding():
    p = inputs.make_problem(40, 33, 64, seed=5)
    outs = []
    for tuning in TUNINGS:
        d, _ = _run(p, tuning)
        outs.append([o.cpu().numpy() for o in d.outputs])
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(a))


def test_repeat_is_deterministic():
    p = inputs.make_problem(30, 20, 64, seed=6)
    d, plan = _run(p, {})
    first = [o.clone() for o in d.outputs]
    for _ in range(3):
        d.run(plan)
    torch.cuda.synchronize()
    for a, b in zip(first, d.outputs):
        assert same_bits(a, b)


@pytest.mark.parametrize("tuning", [{}, {"variant": B.VARIANT_DIRECT}, {"variant": B.VARIANT_MARCH, "chunk": 256, "seg": 4}],
                         ids=["auto", "direct", "m256s4"])
def test_f64_column_top_ignores_values_above_the_top(tuning):
    """FP64 storage takes the truncated column-top form (Listing 1 drops the
    upper vertical flux at k = nz) by a select: NaN in u and v at level 1 of
    the next column (which sits just above the top in a staged window) and
    Inf in w at level nz must not reach su(nz) or sv(nz).  Everywhere the
    oracle (which never reads those values there) is finite the GPU must
    match it to 1e-12; where it is not, the GPU must not be finite either."""
    nx, ny, nz = 9, 12, 64
    p = inputs.make_problem(nx, ny, nz, seed=4242)
    for i, j in ((2, 3), (5, 7), (9, 12), (1, 1)):
        p.u[i, j, 0] = np.nan         # level 1: above the top of column j - 1 in the window
        p.v[i, j, 0] = np.nan
        p.w[i, j, nz - 1] = np.inf    # level nz
    say("non-finite inputs", tuning)
    ref = oracle.advect_problem(p)
    d, plan = _run(p, tuning)
    for name, g_t, o in zip(("su", "sv", "sw"), d.outputs, ref):
        g = g_t.cpu().numpy()[1:-1, 1:-1]
        oi = o[1:-1, 1:-1]
        fin = np.isfinite(oi)
        assert np.array_equal(np.isfinite(g), fin), "%s: the non-finite points differ from the oracle's" % name
        top_ok = np.isfinite(oi[:, :, nz - 1]).all() if name != "sw" else True
        assert top_ok, "%s(nz) must not read the planted values" % name
        den = np.max(np.abs(oi[fin]))
        assert np.max(np.abs(g[fin] - oi[fin])) <= F64_TOL * den


def padded_domain(p, storage, pad, sentinel):
    """u, v, w, su, sv, sw of `p` with packed columns (sy = nz) and a plane
    stride padded by `pad` elements; every element starts at `sentinel`, the
    inputs' views then hold the fields.  Returns (buffers, views)."""
    dt = B.torch_dtype(storage)
    nx, ny, nz = p.nx, p.ny, p.nz
    sx = (ny + 2) * nz + pad
    bufs = [torch.full(((nx + 1) * sx + (ny + 2) * nz,), sentinel, dtype=dt, device=DEV) for _ in range(6)]
    views = [b.as_strided((nx + 2, ny + 2, nz), (sx, nz, 1)) for b in bufs]
    for v, a in zip(views[:3], (p.u, p.v, p.w)):
        v.copy_(B.to_storage(a, storage, 1.0, DEV))
    return bufs, views


def padding_untouched(buf, p, pad, sentinel):
    """The `pad` elements after each plane's (ny + 2) nz still hold the sentinel."""
    if pad == 0:
        return True
    plane = (p.ny + 2) * p.nz
    h = buf.float().cpu().numpy()
    gaps = np.concatenate([h[i * (plane + pad) + plane:(i + 1) * (plane + pad)] for i in range(p.nx + 1)])
    return bool(np.all(gaps == sentinel))


@pytest.mark.parametrize("storage", [B.F64, B.BF16], ids=["f64", "bf16"])
@pytest.mark.parametrize("pad", [16, 3], ids=["pad16-vector", "pad3-scalar"])
def test_march_padded_plane_stride_matches_packed(storage, pad):
    """Packed columns with a padded plane stride run the march kernel (vector
    loads when the stride keeps 16-byte alignment, element loads otherwise);
    the interior equals the packed layout's bit for bit, and the padding
    between planes is never written."""
    p = inputs.make_problem(9, 70, 64, seed=91)          # 9 chunks of 512 per plane: the compact tile order
    tuning = {"variant": B.VARIANT_MARCH, "chunk": 512, "seg": 4}
    ref = device_domain(p, storage)
    ref.run(B.Plan(storage, [B.shape_of(ref.u)], tuning))
    bufs, views = padded_domain(p, storage, pad, -5.0)
    c = p.coeffs
    tz = [torch.from_numpy(x).to(DEV) for x in c.arrays()]
    d = B.DeviceDomain(*views[:3], c.tcx, c.tcy, *tz, outputs=views[3:])
    plan = B.Plan(storage, [B.shape_of(views[0])], tuning)
    assert plan.info()["variant"] == B.VARIANT_MARCH
    d.run(plan)
    torch.cuda.synchronize()
    for o, r in zip(d.outputs, ref.outputs):
        assert same_bits(o[1:-1, 1:-1], r[1:-1, 1:-1])
    for b in bufs[3:]:
        assert padding_untouched(b, p, pad, -5.0)


def test_batched_padded_plane_strides_match_single_calls():
    """A batch mixing a vector-aligned padded plane stride, an odd one and a
    packed domain (the plan then takes element loads for all): every domain's
    interior equals its single-domain call on packed arrays bit for bit, and
    no padding is written."""
    specs = [((7, 40, 64), 16), ((9, 33, 96), 3), ((5, 24, 128), 0)]
    probs, bufs, recs = [], [], []
    for d, ((nx, ny, nz), pad) in enumerate(specs):
        p = inputs.make_problem(nx, ny, nz, seed=930 + d)
        b, v = padded_domain(p, B.F64, pad, -5.0)
        tz = [torch.from_numpy(x).to(DEV) for x in p.coeffs.arrays()]
        for o in v[3:]:
            o.zero_()
        recs.append(B.domain_record(*v, p.coeffs.tcx, p.coeffs.tcy, *tz))
        probs.append((p, pad, v, tz))
        bufs.append(b)
    plan = B.Plan(B.F64, [r.shape for r in recs], {"chunk": 512, "seg": 16})
    B.advect_batched(plan, B.domain_args_tensor(recs, DEV))
    torch.cuda.synchronize()
    assert plan.error_count() == 0
    for (p, pad, v, tz), b in zip(probs, bufs):
        ref = device_domain(p, B.F64)
        ref.run(B.Plan(B.F64, [B.shape_of(ref.u)], {"variant": B.VARIANT_MARCH, "chunk": 512, "seg": 5}))
        torch.cuda.synchronize()
        for o, r in zip(v[3:], ref.outputs):
            assert same_bits(o[1:-1, 1:-1], r[1:-1, 1:-1])
        for o in b[3:]:
            assert padding_untouched(o, p, pad, -5.0)


@pytest.mark.parametrize("shape", [(3, 4, 257), (5, 3, 300), (2, 2, 513)], ids=lambda s: "x".join(map(str, s)))
def test_tall_columns_take_the_direct_kernel(shape):
    """Columns taller than the march kernel's LDS window allows (nz > 256):
    the automatic plan takes the direct kernel, which matches the oracle to
    1e-12; an explicit march plan and a batched plan are refused."""
    nx, ny, nz = shape
    p = inputs.make_problem(nx, ny, nz, seed=2000 + nz)
    ref = oracle.advect_problem(p)
    d, plan = _run(p, {})
    assert plan.info()["variant"] == B.VARIANT_DIRECT
    compare_f64(d, ref, where="%s" % (shape,))
    check_halo_untouched(d)
    with pytest.raises(RuntimeError):
        B.Plan(B.F64, [B.shape_of(d.u)], {"variant": B.VARIANT_MARCH})
    bplan = B.Plan(B.F64, [B.shape_of(d.u)] * 2, None)
    assert bplan.info()["batched_workgroups"] == 0
