"""C-ABI argument checking (needs a GPU; every call here is rejected on the host
before anything is launched, so no kernel runs with a bad argument)."""
import ctypes

import pytest
import torch

from gpu_helpers import DEV, device_domain
from paper_2107_13500_amd import binding as B
from paper_2107_13500_amd import inputs

pytestmark = pytest.mark.gpu

L = None


def lib():
    global L
    if L is None:
        L = B.lib()
    return L


def plan_status(storage, shapes, tuning=None):
    h = ctypes.c_void_p()
    arr = (B.PwShape * len(shapes))(*shapes)
    t = B.make_tuning(tuning)
    st = lib().pw_advect_plan(ctypes.byref(h), storage, arr, len(shapes), ctypes.byref(t) if t else None)
    if st == 0:
        lib().pw_plan_destroy(h)
    return st


def test_plan_rejects_bad_shapes_and_tunings():
    ok = B.PwShape(4, 4, 8, 0, 0, 0)
    assert plan_status(B.F64, [ok]) == 0
    assert plan_status(B.F64, [B.PwShape(0, 4, 8, 0, 0, 0)]) == -1
    assert plan_status(B.F64, [B.PwShape(4, 4, 1, 0, 0, 0)]) == -1
    assert plan_status(B.F64, [B.PwShape(4, 4, 8, 0, 7, 0)]) == -1          # sy < nz
    assert plan_status(B.F64, [B.PwShape(4, 4, 8, 0, 8, 40)]) == -1         # sx < (ny+2) sy
    assert plan_status(B.F64, [B.PwShape(4, 4, 8, 1, 0, 0)]) == -1          # reserved != 0
    assert plan_status(7, [ok]) == -2                                        # unknown storage
    assert plan_status(B.F64, [ok], {"chunk": 300}) == -1
    assert plan_status(B.F64, [ok], {"variant": 9}) == -2
    assert plan_status(B.F64, [ok], {"wg_per_cu": -2}) == -1
    assert plan_status(B.F64, [ok], {"wg_per_cu": 9}) == -1
    assert plan_status(B.F64, [ok], {"wg_per_cu": B.WG_ONE_PER_TILE}) == 0
    assert plan_status(B.F64, [B.PwShape(4, 4, 8, 0, 10, 0)], {"variant": B.VARIANT_MARCH}) == -2
    assert plan_status(B.F64, [B.PwShape(4, 4, 300, 0, 0, 0)], {"variant": B.VARIANT_MARCH}) == -2
    assert plan_status(B.F64, [ok], {"variant": B.VARIANT_DIRECT, "block": 100}) == -1
    h = ctypes.c_void_p()
    assert lib().pw_advect_plan(None, B.F64, (B.PwShape * 1)(ok), 1, None) == -1
    assert lib().pw_advect_plan(ctypes.byref(h), B.F64, None, 1, None) == -1
    assert lib().pw_advect_plan(ctypes.byref(h), B.F64, (B.PwShape * 1)(ok), 0, None) == -1


def _call(plan, ptrs, tz, tcx=0.01, tcy=0.01, scales=None):
    return lib().pw_advect(plan.handle, *ptrs, tcx, tcy, *tz, scales, None)


def test_advect_rejects_bad_arguments_before_launch():
    p = inputs.make_problem(8, 6, 16, seed=3)
    d = device_domain(p)
    plan = B.Plan(B.F64, [B.shape_of(d.u)])
    ptrs = [t.data_ptr() for t in (d.u, d.v, d.w, d.su, d.sv, d.sw)]
    tz = [t.data_ptr() for t in d.tz]
    assert _call(plan, ptrs, tz) == 0
    torch.cuda.synchronize()
    for i in range(6):                                   # null field pointer
        bad = list(ptrs)
        bad[i] = None
        assert _call(plan, bad, tz) == -1
    bad_tz = list(tz)
    bad_tz[2] = None
    assert _call(plan, ptrs, bad_tz) == -1
    assert _call(plan, ptrs, tz, tcx=float("nan")) == -1
    # an output aliasing an input, or two outputs overlapping
    assert _call(plan, ptrs[:3] + [ptrs[0]] + ptrs[4:], tz) == -3
    assert _call(plan, ptrs[:3] + [ptrs[3], ptrs[3] + 64, ptrs[5]], tz) == -3
    # misaligned (not a multiple of 8 bytes for FP64)
    assert _call(plan, [ptrs[0] + 4] + ptrs[1:], tz) == -4
    assert _call(plan, ptrs, [tz[0] + 2] + tz[1:]) == -4
    # a batched plan handed to pw_advect
    two = B.Plan(B.F64, [B.shape_of(d.u), B.shape_of(d.u)])
    assert lib().pw_advect(two.handle, *ptrs, 0.01, 0.01, *tz, None, None) == -8
    assert lib().pw_advect(None, *ptrs, 0.01, 0.01, *tz, None, None) == -1


def test_scales_must_be_positive_powers_of_two():
    p = inputs.make_problem(8, 6, 16, seed=4)
    d = device_domain(p, B.F16)
    plan = B.Plan(B.F16, [B.shape_of(d.u)])
    ptrs = [t.data_ptr() for t in (d.u, d.v, d.w, d.su, d.sv, d.sw)]
    tz = [t.data_ptr() for t in d.tz]
    good = B.make_scales((1024.0, 2048.0, 4096.0), (8.0, 8.0, 8.0))
    assert _call(plan, ptrs, tz, scales=ctypes.byref(good)) == 0
    torch.cuda.synchronize()
    for bad in (B.make_scales((3.0, 1, 1)), B.make_scales((0.0, 1, 1)), B.make_scales((1, 1, 1), (1, -2, 1)),
                B.make_scales((float("inf"), 1, 1))):
        assert _call(plan, ptrs, tz, scales=ctypes.byref(bad)) == -1


def test_batched_checks():
    p = inputs.make_problem(8, 6, 16, seed=5)
    d = device_domain(p)
    plan = B.Plan(B.F64, [B.shape_of(d.u)] * 3)
    args = B.domain_args_tensor([d.record()] * 3, DEV)
    assert lib().pw_advect_batched(plan.handle, 2, args.data_ptr(), None) == -8
    assert lib().pw_advect_batched(plan.handle, 3, None, None) == -1
    assert lib().pw_advect_batched(None, 3, args.data_ptr(), None) == -1
    assert lib().pw_fill_halo_batched(plan.handle, 4, args.data_ptr(), None) == -8
    call = torch.zeros(1, dtype=torch.int64, device=DEV)
    assert lib().pw_perturb_batched(plan.handle, 3, args.data_ptr(), 1, None, 1e-3, None) == -1
    assert lib().pw_perturb_batched(plan.handle, 3, args.data_ptr(), 1, call.data_ptr(), float("nan"), None) == -1
    # a plan whose shapes the batched kernel cannot use
    padded = B.Plan(B.F64, [B.PwShape(8, 6, 16, 0, 20, 0)])
    assert lib().pw_advect_batched(padded.handle, 1, args.data_ptr(), None) == -2


def test_status_strings_and_probe_checks():
    for code in list(B.STATUS_NAMES) + [-99]:
        assert lib().pw_status_string(code)
    a = torch.zeros(64, dtype=torch.float64, device=DEV)
    src = (ctypes.c_void_p * 1)(a.data_ptr())
    assert lib().pw_probe_copy(src, src, 0, 512, 0, None) == -1
    assert lib().pw_probe_copy(src, src, 1, 500, 0, None) == -1
    odd = (ctypes.c_void_p * 1)(a.data_ptr() + 8)
    assert lib().pw_probe_copy(src, odd, 1, 256, 0, None) == -4
