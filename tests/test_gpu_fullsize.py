"""The 2048 x 2048 x 64 workload at full size, in the launch configuration the
benchmark times (the automatic plan), against the oracle on sampled columns
(GPU).

The oracle cannot run the whole grid inside a test, so each sampled interior
column (i, j) is evaluated on its own 3 x 3-column neighbourhood: a 1 x 1
domain whose halo holds the neighbouring columns, which is exactly the data
the stencil reads for that column.  The samples cover the first and last
columns, chunk boundaries (8 columns of 64 levels per 512-point chunk) and
segment boundaries (128 planes), plus random columns.  Properties checked over
the whole grid: level k = 1 and sw(nz) are +0, output halos keep a sentinel.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import DEV, F64_TOL, SENTINEL, check_halo_untouched, column_oracle, sampled_columns, say
from paper_2107_13500_amd import binding as B
from paper_2107_13500_amd import inputs

pytestmark = pytest.mark.gpu

UNIT_ROUNDOFF = {B.F32: 2.0 ** -24, B.BF16: 2.0 ** -8, B.F16: 2.0 ** -11}


@pytest.fixture(scope="module")
def pw2048():
    say("generating pw2048 inputs")
    return inputs.workload("pw2048")


def device_columns(outputs, scales, cols):
    I = torch.tensor([c[0] for c in cols], device=DEV)
    J = torch.tensor([c[1] for c in cols], device=DEV)
    return [o[I, J, :].to(torch.float64).cpu().numpy() / s for o, s in zip(outputs, scales)]


def check_ends(outputs):
    """k = 1 of every output and sw(nz) are +0 over the whole grid."""
    for f, o in enumerate(outputs):
        planes = [o[1:-1, 1:-1, 0]] + ([o[1:-1, 1:-1, -1]] if f == 2 else [])
        for x in planes:
            x = x.to(torch.float32) if x.dtype in (torch.int16, torch.int32) else x
            assert bool((x == 0).all()) and not bool(torch.signbit(x).any()), "column ends must be +0"


def test_f64_pw2048_sampled_columns(pw2048):
    """FP64 with the six arrays packed into one allocation, as the benchmark
    allocates them (the other GPU tests use separate allocations)."""
    p = pw2048
    say("pw2048 FP64: device copy into one pooled allocation")
    pool = B.pooled_fields(p.u.shape, torch.float64, DEV)
    for k, a in enumerate((p.u, p.v, p.w)):
        pool[k].copy_(torch.from_numpy(a))
    tz = [torch.from_numpy(x).to(DEV) for x in p.coeffs.arrays()]
    d = B.DeviceDomain(*pool[:3], p.coeffs.tcx, p.coeffs.tcy, *tz, outputs=pool[3:])
    for o in d.outputs:
        o.fill_(SENTINEL[torch.float64])
    plan = B.Plan(B.F64, [B.shape_of(d.u)])
    info = plan.info()
    say("pw2048 FP64 plan", info)
    assert info["variant"] == B.VARIANT_MARCH
    d.run(plan)
    torch.cuda.synchronize()
    check_ends(d.outputs)
    check_halo_untouched(d)
    cols = sampled_columns(p.nx, p.ny)
    ref = column_oracle((d.u, d.v, d.w), (1.0, 1.0, 1.0), p.coeffs, cols)
    got = device_columns(d.outputs, (1.0, 1.0, 1.0), cols)
    for name, g, r in zip(("su", "sv", "sw"), got, ref):
        e = float(np.max(np.abs(g - r)) / np.max(np.abs(r)))
        say("pw2048 FP64", name, "%d columns, max-norm relative error %.3e" % (len(cols), e))
        assert e <= F64_TOL
    del d, pool
    torch.cuda.empty_cache()


@pytest.mark.parametrize("storage", [B.F32, B.BF16, B.F16, B.I16, B.I32], ids=["f32", "bf16", "f16", "i16", "i32"])
def test_reduced_storage_pw2048_sampled_columns(pw2048, storage):
    """Each storage type at full size, scales as the benchmark picks them,
    against the oracle on the dequantised stored inputs."""
    p = pw2048
    name = B.DTYPE_NAMES[storage]
    ins, outs = inputs.storage_scales(p, name)
    say("pw2048", name, "scales", ins, outs)
    fields = [B.to_storage(a, storage, s, DEV) for a, s in zip((p.u, p.v, p.w), ins)]
    tz = [torch.from_numpy(x).to(DEV) for x in p.coeffs.arrays()]
    d = B.DeviceDomain(*fields, p.coeffs.tcx, p.coeffs.tcy, *tz,
                       scales=B.make_scales(ins, outs) if storage in B.SCALED else None)
    plan = B.Plan(storage, [B.shape_of(fields[0])])
    d.run(plan)
    torch.cuda.synchronize()
    check_ends(d.outputs)
    cols = sampled_columns(p.nx, p.ny, seed=12)
    ref = column_oracle(fields, ins, p.coeffs, cols)
    got = device_columns(d.outputs, outs, cols)
    for f, (g, r, os_) in enumerate(zip(got, ref, outs)):
        m = np.max(np.abs(r))
        e = float(np.max(np.abs(g - r)) / m)
        if storage in (B.I16, B.I32):
            bound = 0.5 / (os_ * m) + (1e-12 if storage == B.I32 else 2e-6)
        else:
            bound = UNIT_ROUNDOFF[storage] + 2e-6
        say("pw2048", name, ("su", "sv", "sw")[f], "error %.3e (bound %.3e)" % (e, bound))
        assert e <= bound
    del d, fields
    torch.cuda.empty_cache()
