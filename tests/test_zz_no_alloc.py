"""The allocation-free batched entry point (GPU), through the C ABI.

pw_advect_batched_noalloc keeps its tile table and error word in a fixed
per-GPU array instead of a plan's device memory.  Its outputs must be bit for
bit those of pw_advect_batched with the same tuning, on consecutive calls
whose second batch is smaller than the first (the array keeps the previous
call's table), and records whose shapes differ from the host shapes must be
refused on the device and counted.
"""
import ctypes

import pytest
import torch

from gpu_helpers import DEV, say, same_bits
from paper_2107_13500_amd import batched as BT
from paper_2107_13500_amd import binding as B
from paper_2107_13500_amd import inputs

pytestmark = pytest.mark.gpu

FIRST = [(16, 16, 64), (17, 23, 96), (40, 9, 128), (5, 3, 64), (96, 31, 96), (33, 50, 64), (1, 1, 64),
         (20, 20, 128), (61, 17, 96), (70, 44, 64), (12, 90, 128)]
SECOND = [(9, 7, 64), (30, 11, 96), (3, 40, 128)]


def problems(shapes, seed):
    return [inputs.make_problem(nx, ny, nz, seed + d, dx=30.0 + 5 * d) for d, (nx, ny, nz) in enumerate(shapes)]


def sentinel(batch, value):
    for f in batch.fields:
        for o in f[3:]:
            o.fill_(value)


def outputs(batch):
    return [[o.clone() for o in f[3:]] for f in batch.fields]


@pytest.mark.parametrize("storage", [B.F64, B.F32, B.BF16], ids=["f64", "f32", "bf16"])
@pytest.mark.parametrize("tuning", [None, {"chunk": 256, "seg": 8, "wg_per_cu": B.WG_ONE_PER_TILE},
                                    {"chunk": 1024, "seg": 32, "wg_per_cu": 2}],
                         ids=["default", "c256s8-one-per-tile", "c1024s32w2"])
def test_noalloc_matches_the_plan_path_on_two_calls(storage, tuning):
    skipped = torch.zeros(1, dtype=torch.int64, device=DEV)
    for call, (shapes, seed) in enumerate(((FIRST, 700), (SECOND, 800))):
        say("no-alloc call", call, B.DTYPE_NAMES[storage], tuning, "domains", len(shapes))
        batch = BT.DeviceBatch(problems(shapes, seed), storage, DEV)
        plan = batch.plan(tuning)
        sentinel(batch, 0)
        batch.advect(plan)
        torch.cuda.synchronize()
        assert plan.error_count() == 0
        want = outputs(batch)
        sentinel(batch, 0)
        B.advect_batched_noalloc(storage, batch.shapes, batch.d_args, tuning, skipped)
        torch.cuda.synchronize()
        got = outputs(batch)
        assert int(skipped.item()) == 0, "records skipped"
        for d in range(len(shapes)):
            for f in range(3):
                assert same_bits(got[d][f], want[d][f]), "call %d domain %d field %d differs" % (call, d, f)


def test_noalloc_refuses_records_whose_shapes_differ_from_the_host_shapes():
    batch = BT.DeviceBatch(problems(SECOND, 900), B.F64, DEV)
    sentinel(batch, -3.0)
    host = list(batch.shapes)
    s = host[1]
    host[1] = B.PwShape(s.nx, s.ny, s.nz, 0, s.sy, s.sx + 64)   # wider x stride than the record's
    skipped = torch.zeros(1, dtype=torch.int64, device=DEV)
    B.advect_batched_noalloc(B.F64, host, batch.d_args, None, skipped)
    torch.cuda.synchronize()
    assert int(skipped.item()) == len(SECOND)
    for f in batch.fields:
        for o in f[3:]:
            assert torch.all(o == -3.0).item(), "a refused batch wrote an output"
    # the next matching call runs normally on the same scratch array
    skipped.zero_()
    B.advect_batched_noalloc(B.F64, batch.shapes, batch.d_args, None, skipped)
    torch.cuda.synchronize()
    assert int(skipped.item()) == 0
    assert not torch.all(batch.fields[0][3] == -3.0).item()


def test_noalloc_rejects_batches_beyond_its_fixed_table():
    l = B.lib()
    shapes = (B.PwShape * 4097)(*[B.PwShape(4, 4, 64, 0, 0, 0)] * 4097)
    dummy = torch.zeros(8, dtype=torch.uint8, device=DEV)
    assert l.pw_advect_batched_noalloc(B.F64, shapes, 4097, dummy.data_ptr(), None, None, None) == -1
    assert l.pw_advect_batched_noalloc(B.F64, shapes, 0, dummy.data_ptr(), None, None, None) == -1
    assert l.pw_advect_batched_noalloc(9, shapes, 1, dummy.data_ptr(), None, None, None) == -2
