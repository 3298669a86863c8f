"""Seeded synthetic inputs for the Piacsek-Williams (PW) advection stencil.

This module builds what the stencil is *given*: the stretched vertical grid,
the density profile, the coefficients tcx, tcy, tzc1, tzc2, tzd1, tzd2 and the
wind fields u, v, w with their one-point periodic x-y halo.  It holds none of
the stencil's own arithmetic, so both the CPU oracle (test infrastructure) and
the HIP path take their inputs from here and from nowhere else.

Array convention (paper, Sec. II-A, Listing 1): Fortran ``u(k, j, i)`` with k
(vertical) fastest and i (x) slowest.  In numpy this is a C-ordered array of
shape ``(nx + 2, ny + 2, nz)`` indexed ``a[i, j, k - 1]``: i and j run over the
halo'd range ``0 .. n + 1`` and k over ``1 .. nz`` with no vertical halo.  The
element strides are therefore ``sy = nz`` and ``sx = (ny + 2) * nz``.

The paper never prints its test fields or coefficient construction, so the
recipe here is a stated reading:

* u = 5 + N(0, 1), v = 2 + N(0, 1), w = 0.3 * N(0, 1) on the interior,
  w = 0 at k = 1 and k = nz (rigid bottom and lid);
* stretched z-grid, dz(k) linear in k from 10 m (k = 2) to 100 m (k = nz);
* density rho(z) = rho0 * exp(-z / H) with rho0 = 1.2 kg m^-3, H = 8000 m;
* tcx = 0.25 / dx, tcy = 0.25 / dy with dx = dy = 50 m;
* tzc1(k) = 0.25 rho_w(k-1) / (rho(k) dz(k)),  tzc2(k) = 0.25 rho_w(k) / (rho(k) dz(k)),
  tzd1(k) = 0.25 rho(k) / (rho_w(k) dzn(k+1)), tzd2(k) = 0.25 rho(k+1) / (rho_w(k) dzn(k+1)),
  where rho is taken at cell centres and rho_w at w-levels.  Entries the
  stencil never reads (k = 1, and tzd at k = nz) are 0.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

SEED_BASE = 2107135

#: Workloads of the measured configurations: (nx, ny, nz).
WORKLOADS = {
    "pw64": (64, 64, 64),          # small: the oracle finishes in well under a second
    "pw512": (512, 512, 64),       # 16.8 M points, the paper's Table I problem size
    "pw2048": (2048, 2048, 64),    # 268 M points, the largest grid of Sec. IV that fits HBM
}


# ----------------------------------------------------------------------------
# vertical grid, density and coefficients
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class VerticalGrid:
    """Stretched vertical grid; every array has length nz and is indexed k - 1.

    dz[k-1]  thickness of level k (k >= 2; dz[0] = 0)
    zw[k-1]  height of the w-level (top face) of level k, zw(1) = 0
    zc[k-1]  height of the centre of level k, zc(1) = -zc(2)
    dzn[k-1] centre spacing zc(k) - zc(k-1) (k >= 2; dzn[0] = 0)
    rho      density at centres, rho_w density at w-levels
    """

    nz: int
    dz: np.ndarray
    zw: np.ndarray
    zc: np.ndarray
    dzn: np.ndarray
    rho: np.ndarray
    rho_w: np.ndarray


def vertical_grid(nz: int, dz_min: float = 10.0, dz_max: float = 100.0,
                  rho0: float = 1.2, scale_height: float = 8000.0) -> VerticalGrid:
    if nz < 2:
        raise ValueError("nz must be >= 2")
    k = np.arange(1, nz + 1, dtype=np.float64)
    dz = np.zeros(nz)
    if nz == 2:
        dz[1] = dz_min
    else:
        dz[1:] = dz_min + (dz_max - dz_min) * (k[1:] - 2.0) / (nz - 2.0)
    zw = np.zeros(nz)
    zw[1:] = np.cumsum(dz[1:])
    zc = np.zeros(nz)
    zc[1:] = 0.5 * (zw[:-1] + zw[1:])
    zc[0] = -zc[1]
    dzn = np.zeros(nz)
    dzn[1:] = zc[1:] - zc[:-1]
    rho = rho0 * np.exp(-zc / scale_height)
    rho_w = rho0 * np.exp(-zw / scale_height)
    return VerticalGrid(nz, dz, zw, zc, dzn, rho, rho_w)


@dataclasses.dataclass
class Coefficients:
    """The stencil's coefficients: two scalars and four per-level arrays (k - 1)."""

    tcx: float
    tcy: float
    tzc1: np.ndarray
    tzc2: np.ndarray
    tzd1: np.ndarray
    tzd2: np.ndarray

    def arrays(self):
        return self.tzc1, self.tzc2, self.tzd1, self.tzd2


def coefficients(grid: VerticalGrid, dx: float = 50.0, dy: float = 50.0) -> Coefficients:
    nz = grid.nz
    tzc1 = np.zeros(nz)
    tzc2 = np.zeros(nz)
    tzd1 = np.zeros(nz)
    tzd2 = np.zeros(nz)
    for k in range(2, nz + 1):
        kk = k - 1
        tzc1[kk] = 0.25 * grid.rho_w[kk - 1] / (grid.rho[kk] * grid.dz[kk])
        tzc2[kk] = 0.25 * grid.rho_w[kk] / (grid.rho[kk] * grid.dz[kk])
    for k in range(2, nz):
        kk = k - 1
        tzd1[kk] = 0.25 * grid.rho[kk] / (grid.rho_w[kk] * grid.dzn[kk + 1])
        tzd2[kk] = 0.25 * grid.rho[kk + 1] / (grid.rho_w[kk] * grid.dzn[kk + 1])
    return Coefficients(0.25 / dx, 0.25 / dy, tzc1, tzc2, tzd1, tzd2)


# ----------------------------------------------------------------------------
# fields
# ----------------------------------------------------------------------------
def empty_field(nx: int, ny: int, nz: int, dtype=np.float64) -> np.ndarray:
    return np.zeros((nx + 2, ny + 2, nz), dtype=dtype)


def fill_periodic_halo(a: np.ndarray) -> np.ndarray:
    """Fill the one-point x-y halo of ``a`` (shape (nx+2, ny+2, nz)) periodically.

    x faces are copied first (interior j only), then y faces over the whole
    halo'd x range, so the four corner columns come out periodic as well.
    """
    nx = a.shape[0] - 2
    ny = a.shape[1] - 2
    a[0, 1:ny + 1] = a[nx, 1:ny + 1]
    a[nx + 1, 1:ny + 1] = a[1, 1:ny + 1]
    a[:, 0] = a[:, ny]
    a[:, ny + 1] = a[:, 1]
    return a


def wind_fields(nx: int, ny: int, nz: int, seed: int,
                u_mean: float = 5.0, v_mean: float = 2.0, w_std: float = 0.3):
    """Seeded u, v, w of shape (nx+2, ny+2, nz), float64, halos filled periodically.

    Draw order (fixes the values for a seed): all of u's interior in C order
    (i, then j, then k), then v's, then w's, from one PCG64 stream.  w is then
    set to 0 at k = 1 and k = nz.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for mean, std in ((u_mean, 1.0), (v_mean, 1.0), (0.0, w_std)):
        a = empty_field(nx, ny, nz)
        for i in range(1, nx + 1):           # plane by plane: same stream as one (nx,ny,nz) draw
            a[i, 1:ny + 1, :] = rng.standard_normal((ny, nz))
        if std != 1.0:
            a[1:nx + 1, 1:ny + 1, :] *= std
        if mean != 0.0:
            a[1:nx + 1, 1:ny + 1, :] += mean
        out.append(a)
    u, v, w = out
    w[:, :, 0] = 0.0
    w[:, :, nz - 1] = 0.0
    for a in out:
        fill_periodic_halo(a)
    return u, v, w


@dataclasses.dataclass
class Problem:
    """One domain: fields, coefficients and the shape."""

    nx: int
    ny: int
    nz: int
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    coeffs: Coefficients
    grid: VerticalGrid

    @property
    def npoints(self) -> int:
        return self.nx * self.ny * self.nz


def make_problem(nx: int, ny: int, nz: int, seed: int, dx: float = 50.0, dy: Optional[float] = None,
                 rho0: float = 1.2, scale_height: float = 8000.0) -> Problem:
    grid = vertical_grid(nz, rho0=rho0, scale_height=scale_height)
    co = coefficients(grid, dx, dx if dy is None else dy)
    u, v, w = wind_fields(nx, ny, nz, seed)
    return Problem(nx, ny, nz, u, v, w, co, grid)


def workload(name: str, seed_offset: int = 0) -> Problem:
    """The named single-domain workload ("pw64", "pw512", "pw2048")."""
    nx, ny, nz = WORKLOADS[name]
    index = list(WORKLOADS).index(name)
    return make_problem(nx, ny, nz, SEED_BASE + index + seed_offset)


# ----------------------------------------------------------------------------
# batched: many uneven subdomains
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class DomainSpec:
    nx: int
    ny: int
    nz: int
    dx: float
    rho0: float
    scale_height: float
    seed: int


def batched_specs(ndomains: int = 384, seed: int = SEED_BASE + 4,
                  nxy_range=(16, 96), nz_choices: Sequence[int] = (64, 96, 128),
                  dx_range=(25.0, 100.0), rho0_range=(1.1, 1.3),
                  h_range=(6000.0, 10000.0)) -> List[DomainSpec]:
    """Shapes and physical parameters of ``ndomains`` uneven subdomains.

    nx, ny ~ U{16..96}; nz ~ U{64, 96, 128}; dx = dy ~ U(25, 100) m; each domain
    has its own density profile rho0 ~ U(1.1, 1.3), H ~ U(6000, 10000) m.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for d in range(ndomains):
        nx = int(rng.integers(nxy_range[0], nxy_range[1] + 1))
        ny = int(rng.integers(nxy_range[0], nxy_range[1] + 1))
        nz = int(nz_choices[int(rng.integers(0, len(nz_choices)))])
        dx = float(rng.uniform(*dx_range))
        rho0 = float(rng.uniform(*rho0_range))
        hh = float(rng.uniform(*h_range))
        specs.append(DomainSpec(nx, ny, nz, dx, rho0, hh, seed * 1000 + d))
    return specs


def make_domain(spec: DomainSpec) -> Problem:
    return make_problem(spec.nx, spec.ny, spec.nz, spec.seed, dx=spec.dx,
                        rho0=spec.rho0, scale_height=spec.scale_height)


# ----------------------------------------------------------------------------
# reduced-precision storage: per-field power-of-two scales
# ----------------------------------------------------------------------------
def pow2_scale(max_abs: float, target: float = 2.0 ** 14) -> float:
    """Largest power of two s with s * max_abs <= target (1 if max_abs is 0)."""
    if max_abs <= 0.0 or not np.isfinite(max_abs):
        return 1.0
    return float(2.0 ** np.floor(np.log2(target / max_abs)))


def interior(a: np.ndarray) -> np.ndarray:
    """View of the computed points (i, j in 1..n) of a halo'd array."""
    return a[1:-1, 1:-1, :]


def output_bounds(p: Problem):
    """A-priori bounds on max |su|, |sv|, |sw| from the input maxima.

    Each flux is (one velocity) x (a sum of two velocities) times its
    coefficient, so |x-term| <= 4 tcx M M', |vertical| <= 2 (tz1 + tz2) M M'.
    Used only to choose FP16 output scales; no output value is computed.
    """
    mu, mv, mw = (float(np.max(np.abs(a))) for a in (p.u, p.v, p.w))
    c = p.coeffs
    zc = float(np.max(c.tzc1 + c.tzc2))
    zd = float(np.max(c.tzd1 + c.tzd2))
    bu = 4 * c.tcx * mu * mu + 4 * c.tcy * mu * mv + 2 * zc * mu * mw
    bv = 4 * c.tcy * mv * mv + 4 * c.tcx * mv * mu + 2 * zc * mv * mw
    bw = 4 * c.tcx * mw * mu + 4 * c.tcy * mw * mv + 2 * zd * mw * mw
    return bu, bv, bw


def fp16_input_scales(p: Problem, target: float = 2.0 ** 14):
    return tuple(pow2_scale(float(np.max(np.abs(a))), target) for a in (p.u, p.v, p.w))


def fp16_output_scales(p: Problem, target: float = 2.0 ** 14):
    return tuple(pow2_scale(b, target) for b in output_bounds(p))


# Largest scaled magnitude per scaled storage type: FP16 and int16 keep values
# below 2^14 (FP16 max 65504, int16 max 32767); int32 below 2^30.
SCALE_TARGET = {"f16": 2.0 ** 14, "i16": 2.0 ** 14, "i32": 2.0 ** 30}


def storage_scales(p: Problem, dtype: str):
    """(input scales, output scales) for storage `dtype` ("f64", "f32",
    "bf16", "f16", "i16", "i32"): powers of two from the input maxima and the
    a-priori output bounds; all 1 where the type needs none (BF16 keeps the
    FP32 exponent range)."""
    if dtype not in SCALE_TARGET:
        return (1.0, 1.0, 1.0), (1.0, 1.0, 1.0)
    t = SCALE_TARGET[dtype]
    return fp16_input_scales(p, t), fp16_output_scales(p, t)
