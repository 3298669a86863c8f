"""Host-side argument checks of the binding (CPU only): tensors that do not
match a plan's storage type or shape, or coefficient arrays that are too
short, are refused before any pointer reaches the library."""
import pytest
import torch

from paper_2107_13500_amd import binding as B


def fields(nx=6, ny=5, nz=8, dtype=torch.float64):
    return [torch.zeros(nx + 2, ny + 2, nz, dtype=dtype) for _ in range(6)]


def coefs(nz=8, dtype=torch.float64):
    return [torch.zeros(nz, dtype=dtype) for _ in range(4)]


SHAPE = B.PwShape(6, 5, 8, 0, 0, 0)


def test_wrong_storage_dtype_is_refused():
    with pytest.raises(ValueError, match="dtype"):
        B.check_fields(B.F64, SHAPE, fields(dtype=torch.float32), coefs())
    f = fields()
    f[4] = f[4].float()
    with pytest.raises(ValueError, match="sv has dtype"):
        B.check_fields(B.F64, SHAPE, f, coefs())


def test_smaller_or_differently_strided_fields_are_refused():
    f = fields()
    f[3] = torch.zeros(7, 7, 8, dtype=torch.float64)   # one x plane short
    with pytest.raises(ValueError, match="su has shape"):
        B.check_fields(B.F64, SHAPE, f, coefs())
    f = fields()
    f[0] = torch.zeros(8, 7, 10, dtype=torch.float64)[:, :, :8]   # padded columns: sy = 10, not nz
    with pytest.raises(ValueError, match="u has shape"):
        B.check_fields(B.F64, SHAPE, f, coefs())


def test_short_or_non_double_coefficients_are_refused():
    with pytest.raises(ValueError, match="at least nz"):
        B.check_fields(B.F64, SHAPE, fields(), coefs(nz=7))
    with pytest.raises(ValueError, match="float64"):
        B.check_fields(B.F64, SHAPE, fields(), coefs(dtype=torch.float32))


def test_host_tensors_are_refused_for_device_calls():
    with pytest.raises(ValueError, match="CUDA tensor"):
        B.check_fields(B.F64, SHAPE, fields(), coefs())
