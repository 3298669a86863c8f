"""The seeded input generator (CPU only): determinism, halos, coefficients."""
import numpy as np

from paper_2107_13500_amd import inputs


def test_fields_are_seeded_and_deterministic():
    a = inputs.wind_fields(6, 5, 8, seed=1)
    b = inputs.wind_fields(6, 5, 8, seed=1)
    c = inputs.wind_fields(6, 5, 8, seed=2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert not np.array_equal(a[0], c[0])


def test_plane_by_plane_draw_equals_one_block_draw():
    nx, ny, nz = 4, 3, 5
    u, v, w = inputs.wind_fields(nx, ny, nz, seed=9)
    rng = np.random.Generator(np.random.PCG64(9))
    assert np.array_equal(u[1:-1, 1:-1], 5.0 + rng.standard_normal((nx, ny, nz)))
    assert np.array_equal(v[1:-1, 1:-1], 2.0 + rng.standard_normal((nx, ny, nz)))


def test_w_vanishes_at_bottom_and_lid_and_halos_are_periodic():
    u, v, w = inputs.wind_fields(7, 6, 9, seed=3)
    assert np.all(w[:, :, 0] == 0) and np.all(w[:, :, -1] == 0)
    for a in (u, v, w):
        assert np.array_equal(a[0, 1:-1], a[-2, 1:-1])
        assert np.array_equal(a[-1, 1:-1], a[1, 1:-1])
        assert np.array_equal(a[:, 0], a[:, -2])
        assert np.array_equal(a[:, -1], a[:, 1])
        assert a[0, 0, 3] == a[-2, -2, 3] and a[-1, -1, 3] == a[1, 1, 3]


def test_vertical_grid_is_stretched_10_to_100_m():
    g = inputs.vertical_grid(64)
    assert g.dz[1] == 10.0 and abs(g.dz[-1] - 100.0) < 1e-12
    assert np.all(np.diff(g.dz[1:]) > 0)
    assert g.zw[0] == 0.0 and np.allclose(np.diff(g.zw[1:]), g.dz[2:])
    assert np.allclose(g.rho, 1.2 * np.exp(-g.zc / 8000.0))


def test_coefficient_weights_telescope():
    """rho(k) dz(k) tzc1(k) = rho_w(k-1)/4 and rho(k) dz(k) tzc2(k) = rho_w(k)/4;
    rho_w(k) dzn(k+1) tzd1(k) = rho(k)/4 and ... tzd2(k) = rho(k+1)/4."""
    g = inputs.vertical_grid(20)
    c = inputs.coefficients(g, 50.0, 40.0)
    assert c.tcx == 0.25 / 50.0 and c.tcy == 0.25 / 40.0
    k = np.arange(1, 20)          # 0-based index of levels 2..nz
    assert np.allclose(g.rho[k] * g.dz[k] * c.tzc1[k], 0.25 * g.rho_w[k - 1])
    assert np.allclose(g.rho[k] * g.dz[k] * c.tzc2[k], 0.25 * g.rho_w[k])
    k = np.arange(1, 19)          # levels 2..nz-1
    assert np.allclose(g.rho_w[k] * g.dzn[k + 1] * c.tzd1[k], 0.25 * g.rho[k])
    assert np.allclose(g.rho_w[k] * g.dzn[k + 1] * c.tzd2[k], 0.25 * g.rho[k + 1])
    assert c.tzc1[0] == c.tzc2[0] == c.tzd1[0] == c.tzd1[-1] == c.tzd2[-1] == 0.0


def test_batched_specs_ranges():
    specs = inputs.batched_specs()
    assert len(specs) == 384
    assert all(16 <= s.nx <= 96 and 16 <= s.ny <= 96 for s in specs)
    assert {s.nz for s in specs} == {64, 96, 128}
    assert all(25.0 <= s.dx <= 100.0 and 1.1 <= s.rho0 <= 1.3 for s in specs)
    assert inputs.batched_specs() == specs


def test_pow2_scale():
    assert inputs.pow2_scale(10.0) == 1024.0
    assert inputs.pow2_scale(0.0) == 1.0
    s = inputs.pow2_scale(3e-3)
    assert s * 3e-3 <= 2 ** 14 < 2 * s * 3e-3
