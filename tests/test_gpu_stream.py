"""Host-resident domains through pw_advect_host (GPU).

The slab pipeline and the bulk round trip must give exactly what pw_advect
gives on the same data already in device memory (the same kernel arithmetic
per point), match the oracle to 1e-12, and leave the host outputs' halo
columns untouched.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import DEV, F64_TOL, column_oracle, max_rel, positive_zeros, same_bits, sampled_columns, say
from paper_2107_13500_amd import binding as B
from paper_2107_13500_amd import inputs

pytestmark = pytest.mark.gpu

HOST_SENTINEL = -5.5e300


def host_arrays(p, pinned=True, storage=B.F64):
    dt = B.torch_dtype(storage)
    ins = [torch.from_numpy(a).to(dt) for a in (p.u, p.v, p.w)]
    if pinned:
        ins = [t.pin_memory() for t in ins]
    outs = [torch.full(p.u.shape, HOST_SENTINEL if storage == B.F64 else -7.0e30, dtype=dt, pin_memory=pinned)
            for _ in range(3)]
    tz = [torch.from_numpy(x).clone() for x in p.coeffs.arrays()]
    return ins, outs, tz


def device_reference(p, storage=B.F64):
    dt = B.torch_dtype(storage)
    u, v, w = (torch.from_numpy(a).to(dt).to(DEV) for a in (p.u, p.v, p.w))
    tz = [torch.from_numpy(x).to(DEV) for x in p.coeffs.arrays()]
    d = B.DeviceDomain(u, v, w, p.coeffs.tcx, p.coeffs.tcy, *tz)
    d.run(B.Plan(storage, [B.shape_of(u)]))
    torch.cuda.synchronize()
    return [o.cpu() for o in d.outputs]


@pytest.mark.parametrize("shape", [(37, 29, 64), (20, 9, 96), (13, 6, 128), (5, 4, 30)],
                         ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("mode", [dict(chunk=1, nbuffers=2), dict(chunk=5, nbuffers=3), dict(chunk=16, nbuffers=2),
                                  dict(bulk=True)], ids=["c1b2", "c5b3", "c16b2", "bulk"])
def test_host_domain_matches_device_call_and_oracle(shape, mode):
    p = inputs.make_problem(*shape, seed=4321 + shape[0])
    ins, outs, tz = host_arrays(p)
    sp = B.StreamPlan(B.F64, B.shape_of(ins[0]), **mode)
    sp.run(*ins, *outs, p.coeffs.tcx, p.coeffs.tcy, *tz)
    dev = device_reference(p)
    ref = oracle.advect_problem(p)
    for o, dref, r in zip(outs, dev, ref):
        a = o.numpy()
        for face in (a[0], a[-1], a[:, 0], a[:, -1]):
            assert np.all(face == HOST_SENTINEL), "host output halo written"
        assert same_bits(o[1:-1, 1:-1], dref[1:-1, 1:-1]), "differs from the device-resident call"
        assert max_rel(a[1:-1, 1:-1], r[1:-1, 1:-1]) <= F64_TOL
    sp.close()


def test_pageable_host_memory_and_fp32_storage():
    p = inputs.make_problem(24, 17, 64, seed=99)
    ins, outs, tz = host_arrays(p, pinned=False, storage=B.F32)
    sp = B.StreamPlan(B.F32, B.shape_of(ins[0]), chunk=7, nbuffers=3)
    sp.run(*ins, *outs, p.coeffs.tcx, p.coeffs.tcy, *tz)
    dev = device_reference(p, B.F32)
    for o, dref in zip(outs, dev):
        assert same_bits(o[1:-1, 1:-1], dref[1:-1, 1:-1])


@pytest.mark.parametrize("storage", [B.BF16, B.I16, B.I32], ids=["bf16", "i16", "i32"])
def test_scaled_storage_host_domain_matches_device_call(storage):
    p = inputs.make_problem(30, 11, 64, seed=123)
    ins_s, outs_s = inputs.storage_scales(p, B.DTYPE_NAMES[storage])
    sc = B.make_scales(ins_s, outs_s)
    ins = [B.to_storage(a, storage, s_).pin_memory() for a, s_ in zip((p.u, p.v, p.w), ins_s)]
    outs = [torch.zeros(p.u.shape, dtype=B.torch_dtype(storage), pin_memory=True) for _ in range(3)]
    tz = [torch.from_numpy(x).clone() for x in p.coeffs.arrays()]
    sp = B.StreamPlan(storage, B.shape_of(ins[0]), chunk=8, nbuffers=2)
    sp.run(*ins, *outs, p.coeffs.tcx, p.coeffs.tcy, *tz, scales=sc)
    sp.close()
    dev_in = [t.to(DEV) for t in ins]
    d = B.DeviceDomain(*dev_in, p.coeffs.tcx, p.coeffs.tcy, *[t.to(DEV) for t in tz], scales=sc)
    d.run(B.Plan(storage, [B.shape_of(dev_in[0])]))
    torch.cuda.synchronize()
    for o, dref in zip(outs, d.outputs):
        assert same_bits(o[1:-1, 1:-1], dref.cpu()[1:-1, 1:-1])


def test_repeated_calls_reuse_the_plan():
    p = inputs.make_problem(40, 12, 64, seed=7)
    ins, outs, tz = host_arrays(p)
    sp = B.StreamPlan(B.F64, B.shape_of(ins[0]), chunk=8, nbuffers=2)
    sp.run(*ins, *outs, p.coeffs.tcx, p.coeffs.tcy, *tz)
    first = [o.clone() for o in outs]
    for _ in range(3):
        sp.run(*ins, *outs, p.coeffs.tcx, p.coeffs.tcy, *tz)
    for a, b in zip(first, outs):
        assert same_bits(a, b)


def test_stream_plan_argument_checks():
    l = B.lib()
    h = ctypes.c_void_p()
    padded = B.PwShape(8, 6, 16, 0, 20, 0)
    assert l.pw_stream_plan_create(ctypes.byref(h), B.F64, ctypes.byref(padded), 4, 2, 0, None) == -2
    ok = B.PwShape(8, 6, 16, 0, 0, 0)
    assert l.pw_stream_plan_create(ctypes.byref(h), B.F64, ctypes.byref(ok), 0, 2, 0, None) == -1
    assert l.pw_stream_plan_create(ctypes.byref(h), B.F64, ctypes.byref(ok), 4, 1, 0, None) == -1
    assert l.pw_stream_plan_create(ctypes.byref(h), 9, ctypes.byref(ok), 4, 2, 0, None) == -2
    p = inputs.make_problem(8, 6, 16, seed=3)
    ins, outs, tz = host_arrays(p)
    sp = B.StreamPlan(B.F64, B.shape_of(ins[0]), chunk=4, nbuffers=2)
    st = l.pw_advect_host(sp.handle, ins[0].data_ptr(), ins[1].data_ptr(), ins[2].data_ptr(), ins[0].data_ptr(),
                          outs[1].data_ptr(), outs[2].data_ptr(), 0.01, 0.01, *[t.data_ptr() for t in tz], None)
    assert st == -3
    st = l.pw_advect_host(sp.handle, None, ins[1].data_ptr(), ins[2].data_ptr(), outs[0].data_ptr(),
                          outs[1].data_ptr(), outs[2].data_ptr(), 0.01, 0.01, *[t.data_ptr() for t in tz], None)
    assert st == -1


def test_host_resident_537m_points_sampled_columns():
    """The paper's largest grid (2048 x 4096 x 64, 537M points) host-resident
    in pinned memory, overlapped x-slabs of 64 planes as the benchmark runs
    it: sampled columns (including slab boundaries) against the oracle, k = 1
    and sw(nz) +0, host output halos untouched."""
    import gc
    p = inputs.make_problem(2048, 4096, 64, inputs.SEED_BASE + 5)
    say("537M points: pinned host arrays")
    ins, outs, tz = host_arrays(p)
    sp = B.StreamPlan(B.F64, B.shape_of(ins[0]), chunk=64, nbuffers=3)
    sp.run(*ins, *outs, p.coeffs.tcx, p.coeffs.tcy, *tz)
    sp.close()
    say("537M points: checking sampled columns")
    cols = sampled_columns(p.nx, p.ny, seed=13, extra_i=(64, 65, 1984, 1985))
    ref = column_oracle(ins, (1.0, 1.0, 1.0), p.coeffs, cols)
    I = torch.tensor([c[0] for c in cols])
    J = torch.tensor([c[1] for c in cols])
    for name, o, r in zip(("su", "sv", "sw"), outs, ref):
        g = o[I, J, :].numpy()
        e = float(np.max(np.abs(g - r)) / np.max(np.abs(r)))
        say("537M", name, "%d columns, max-norm relative error %.3e" % (len(cols), e))
        assert e <= F64_TOL
        assert positive_zeros(g[:, 0])
        if name == "sw":
            assert positive_zeros(g[:, -1])
        for face in (o[0], o[-1], o[:, 0], o[:, -1]):
            assert bool((face == HOST_SENTINEL).all()), "a host output halo column was written"
    del ins, outs, p
    gc.collect()
    if hasattr(torch._C, "_host_emptyCache"):
        torch._C._host_emptyCache()   # return the pinned blocks
