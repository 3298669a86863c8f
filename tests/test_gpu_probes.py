"""The bandwidth probes' own contracts (GPU): pw_probe_march stores exactly
the documented values in the interior columns and touches nothing else, and
rejects every shape its indexing does not cover before launching."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_helpers import DEV
from paper_2107_13500_amd import binding as B

pytestmark = pytest.mark.gpu

SENTINEL = -7.25
TAIL = 4096   # doubles after each array's extent that must keep the sentinel


def arrays(nx, ny, nz, sx, seed):
    extent = (nx + 1) * sx + (ny + 2) * nz
    g = torch.Generator().manual_seed(seed)
    ins = [torch.randn(extent + TAIL, dtype=torch.float64, generator=g).to(DEV) for _ in range(3)]
    outs = [torch.full((extent + TAIL,), SENTINEL, dtype=torch.float64, device=DEV) for _ in range(3)]
    return ins, outs, extent


def expected(inp, nx, ny, nz, sx):
    """out(plane i, element nz + c*512 + 2t + e) = in(i, c*512 + 2t + e) + in(i, c*512 + 2*min(256 + t, 255 + nz) + e)."""
    e = np.full_like(inp, SENTINEL)
    nc = ny * nz // 512
    t = np.arange(256)
    v1 = np.minimum(256 + t, 255 + nz)
    for i in range(1, nx + 1):
        for c in range(nc):
            base = i * sx + c * 512
            for comp in (0, 1):
                e[base + nz + 2 * t + comp] = inp[base + 2 * t + comp] + inp[base + 2 * v1 + comp]
    return e


@pytest.mark.parametrize("nx,ny,nz,pad,seg", [(8, 16, 64, 0, 2), (12, 48, 32, 0, 4), (6, 12, 128, 64, 6),
                                              (16, 8, 256, 2, 16), (4, 32, 16, 0, 4)])
def test_probe_march_stores_the_documented_values_and_nothing_else(nx, ny, nz, pad, seg):
    sx = (ny + 2) * nz + pad
    ins, outs, extent = arrays(nx, ny, nz, sx, seed=nx * 1000 + nz)
    shape = B.PwShape(nx, ny, nz, 0, nz, sx)
    torch.cuda.synchronize()
    B.check(B.lib().pw_probe_march(*[a.data_ptr() for a in ins + outs], ctypes.byref(shape), seg, None),
            "pw_probe_march")
    torch.cuda.synchronize()
    for a, o in zip(ins, outs):
        want = expected(a.cpu().numpy(), nx, ny, nz, sx)
        np.testing.assert_array_equal(o.cpu().numpy(), want)


def test_probe_march_rejects_shapes_it_does_not_cover():
    nx, ny, nz = 8, 16, 64
    sx = (ny + 2) * nz
    ins, outs, _ = arrays(nx, ny, nz, sx, seed=3)
    ptrs = [a.data_ptr() for a in ins + outs]
    call = lambda shape, seg, p=ptrs: B.lib().pw_probe_march(*p, ctypes.byref(shape), seg, None)
    ok = B.PwShape(nx, ny, nz, 0, nz, sx)
    assert call(ok, 2) == 0
    torch.cuda.synchronize()
    assert call(B.PwShape(nx, ny, 63, 0, 63, (ny + 2) * 63), 2) == -1       # odd nz
    assert call(B.PwShape(nx, 2, 512, 0, 512, 4 * 512), 2) == -1            # nz > 256
    assert call(B.PwShape(nx, ny, nz, 0, nz + 2, sx), 2) == -1              # sy != nz
    assert call(B.PwShape(nx, ny, nz, 0, nz, sx - 2), 2) == -1              # sx too small
    assert call(B.PwShape(nx, 15, nz, 0, nz, 17 * nz), 2) == -1             # ny nz not a multiple of 512
    assert call(B.PwShape(nx, ny, nz, 1, nz, sx), 2) == -1                  # reserved field
    assert call(ok, 3) == -1 and call(ok, 0) == -1 and call(ok, 6) == -1   # odd, zero, not dividing nx
    assert B.lib().pw_probe_march(*ptrs[:5], None, ctypes.byref(ok), 2, None) == -1
    assert B.lib().pw_probe_march(*ptrs[:3], ptrs[3] + 8, *ptrs[4:], ctypes.byref(ok), 2, None) == -4
    assert B.lib().pw_probe_march(*ptrs, None, 2, None) == -1
