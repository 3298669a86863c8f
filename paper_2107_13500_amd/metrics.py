"""Counting conventions for PW advection throughput (no stencil arithmetic).

Flop model (paper Sec. III): each of the three advection stages costs 21
floating-point operations per cell, 63 per cell in total, reduced to 55 at
the column top; level k = 1 is not computed.  The paper's "theoretical"
figure is clock x average operations per computed cell (one cell per cycle).

Byte model (paper Sec. IV): three FP64 input arrays in, three out, 48 B per
grid point, which reproduces the quoted transfer volumes.  The algorithmic
bytes of one device call add the one-point x-y halo that each input is read
with and the per-level coefficients.
"""
from __future__ import annotations

FLOPS_PER_CELL = 63        # 21 per field, Sec. III
FLOPS_COLUMN_TOP = 55      # 17 + 17 + 21, Sec. III
BYTES_PER_POINT_F64 = 48   # 3 arrays in + 3 out, Sec. IV data volumes

ELEM_BYTES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2, "i16": 2, "i32": 4}


def flops_per_column(nz: int) -> int:
    """Paper flop count of one column of nz levels (k = 2 .. nz computed)."""
    if nz < 2:
        raise ValueError("nz >= 2")
    return (nz - 2) * FLOPS_PER_CELL + FLOPS_COLUMN_TOP


def theoretical_gflops(clock_hz: float, nz: int = 64) -> float:
    """Clock x average flops per computed cell (one cell per cycle), in GFLOP/s."""
    return clock_hz * flops_per_column(nz) / (nz - 1) / 1e9


def paper_equivalent_gflops(points_per_s: float, nz: int = 64) -> float:
    """GFLOP/s under the paper's flop model for a measured point rate."""
    return points_per_s * flops_per_column(nz) / nz / 1e9


def transfer_bytes_f64(npoints: int) -> int:
    """Host<->device bytes for one run (3 FP64 arrays each way), Sec. IV."""
    return BYTES_PER_POINT_F64 * npoints


def algorithmic_bytes(nx: int, ny: int, nz: int, elem: int = 8, coef_elem: int = 8) -> int:
    """Bytes one call must move: each input read once with its x-y halo, each
    output written once over the interior, plus the four per-level coefficients."""
    halo = (nx + 2) * (ny + 2) * nz
    inner = nx * ny * nz
    return elem * (3 * halo + 3 * inner) + 4 * nz * coef_elem


# Acceptance bounds, max-norm relative error per field (max |g - o| / max |o|
# over the computed points), shared by the GPU tests and the benchmark's
# parity gate.
F64_PARITY_TOL = 1e-12
#: reduced storage against the FP64 oracle on the original FP64 fields, for
#: the seeded synthetic inputs (u = 5 + N(0,1), v = 2 + N(0,1), w = 0.3 N(0,1))
#: and the per-field scales of ``inputs.storage_scales``
STORAGE_ERROR_BOUND = {"f32": 2e-6, "bf16": 2e-2, "f16": 3e-3, "i16": 3e-3, "i32": 2e-8}
#: batched domains after perturbation, against the oracle on the domains'
#: final stored fields: FP64 parity, or FP32 output roundoff plus the
#: compensated FP32 arithmetic
BATCHED_ERROR_BOUND = {"f64": F64_PARITY_TOL, "f32": 2.0 ** -24 + 2e-6}
