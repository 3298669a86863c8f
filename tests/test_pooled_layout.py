"""The pooled layout helper (CPU only): six arrays in one allocation, back to
back, each start aligned, no overlap; DeviceDomain takes them as outputs."""
import pytest
import torch

from paper_2107_13500_amd import binding as B


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16, torch.int16, torch.int32])
def test_pooled_fields_are_disjoint_aligned_views(dtype):
    shape = (7, 5, 13)
    a = B.pooled_fields(shape, dtype, "cpu")
    assert len(a) == 6
    esize = a[0].element_size()
    n = 7 * 5 * 13
    starts = [t.data_ptr() for t in a]
    for t in a:
        assert t.shape == shape and t.dtype == dtype and t.is_contiguous()
        assert (t.data_ptr() - starts[0]) % 256 == 0
    for s0, s1 in zip(starts, starts[1:]):
        assert s1 - s0 >= n * esize            # no overlap
        assert s1 - s0 < n * esize + 256       # packed: at most the alignment gap
    for k, t in enumerate(a):
        t.fill_(k)
    assert [int(t.double().mean()) for t in a] == list(range(6))


def test_device_domain_takes_and_clears_given_outputs():
    a = B.pooled_fields((4, 4, 8), torch.float64, "cpu")
    for t in a:
        t.fill_(3.0)
    tz = [torch.zeros(8, dtype=torch.float64) for _ in range(4)]
    d = B.DeviceDomain(a[0], a[1], a[2], 0.1, 0.1, *tz, outputs=a[3:])
    assert all(o.data_ptr() == t.data_ptr() for o, t in zip(d.outputs, a[3:]))
    assert all(bool((o == 0).all()) for o in d.outputs)
    assert bool((a[0] == 3.0).all())
    with pytest.raises(ValueError):
        B.DeviceDomain(a[0], a[1], a[2], 0.1, 0.1, *tz, outputs=[torch.zeros(4, 4, 7, dtype=torch.float64)] * 3)
