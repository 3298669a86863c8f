"""The FP64 oracle against the paper and against mathematics (CPU only)."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import oracle_pins
import staggered_rule as rule
from paper_2107_13500_amd import inputs


@pytest.mark.parametrize("name", sorted(oracle_pins.ALL_PINS))
def test_oracle_pin(name):
    oracle_pins.ALL_PINS[name](oracle.advect)


def test_rule_u_case_is_listing1():
    """The staggering rule's u-case is Listing 1 (Sec. II-A), exactly, with
    non-dyadic rationals so no floating point is involved at all."""
    rng = np.random.default_rng(5)
    nx, ny, nz = 3, 3, 4
    shp = (nx + 2, ny + 2, nz)
    fr = lambda: [[[Fraction(int(rng.integers(-30, 31)), 7) for _ in range(nz)]
                   for _ in range(ny + 2)] for _ in range(nx + 2)]
    u, v, w = fr(), fr(), fr()
    cz = lambda: [Fraction(int(rng.integers(1, 20)), 13) for _ in range(nz)]
    F = rule.Fields(u, v, w, Fraction(3, 11), Fraction(5, 17), cz(), cz(), cz(), cz())
    for i in range(1, nx + 1):
        for j in range(1, ny + 1):
            for k in range(2, nz + 1):
                assert rule.source(F, "u", (k, j, i)) == rule.listing1_su(F, (k, j, i))


def test_rule_op_counts_match_paper():
    """Sec. III: 21 operations per field per cell, 63 in all, 55 at the column top."""
    nx, ny, nz = 1, 1, 4
    shp = (nx + 2, ny + 2, nz)
    ones = np.ones(shp)
    F = rule.Fields(ones, ones, ones, 1, 1, [1] * nz, [1] * nz, [1] * nz, [1] * nz, conv=rule.Counted)
    for k in range(2, nz):
        counts = [rule.op_count(F, phi, (k, 1, 1)) for phi in "uvw"]
        assert counts == [21, 21, 21]
    top = [rule.op_count(F, phi, (nz, 1, 1)) for phi in "uv"]
    assert top == [17, 17]
    # the paper's 55 at the top counts a full 21-op w stage there
    assert sum(top) + 21 == 55


def test_oracle_strided_slab_matches_full_grid():
    """An x-slab or a y-slab view evaluates exactly as the full grid does."""
    p = inputs.make_problem(9, 7, 6, 21)
    c = p.coeffs
    full = oracle.advect_problem(p)
    i0, i1 = 3, 6                      # interior planes i0..i1
    sl = slice(i0 - 1, i1 + 2)
    part = oracle.advect(p.u[sl], p.v[sl], p.w[sl], c.tcx, c.tcy, *c.arrays())
    for a, b in zip(full, part):
        assert np.array_equal(a[i0:i1 + 1, 1:-1], b[1:-1, 1:-1])
    j0, j1 = 2, 5
    sl = (slice(None), slice(j0 - 1, j1 + 2))
    part = oracle.advect(p.u[sl], p.v[sl], p.w[sl], c.tcx, c.tcy, *c.arrays())
    for a, b in zip(full, part):
        assert np.array_equal(a[1:-1, j0:j1 + 1], b[1:-1, 1:-1])


def test_oracle_thread_count_does_not_change_results():
    p = inputs.make_problem(16, 9, 10, 22)
    one = oracle.advect_problem(p, threads=1)
    many = oracle.advect_problem(p, threads=4)
    for a, b in zip(one, many):
        assert np.array_equal(a, b)


def test_oracle_rejects_bad_shapes():
    z = np.zeros((3, 3, 1))
    with pytest.raises(ValueError):
        oracle.advect(z, z, z, 1.0, 1.0, *[np.zeros(1)] * 4)
    z = np.zeros((3, 3, 4))
    with pytest.raises(ValueError):
        oracle.advect(z, z, z, 1.0, 1.0, *[np.zeros(3)] * 4)


def test_oracle_nz2_is_top_only():
    """nz = 2: only the top level is computed; su, sv keep only the lower
    vertical flux and sw is 0 (rigid lid)."""
    p = inputs.make_problem(4, 3, 2, 23)
    su, sv, sw = oracle.advect_problem(p)
    assert np.all(sw[1:-1, 1:-1] == 0.0)
    assert np.all(su[1:-1, 1:-1, 0] == 0.0)
    F = rule.Fields(p.u, p.v, p.w, p.coeffs.tcx, p.coeffs.tcy, *p.coeffs.arrays(), conv=float)
    for i in range(1, 5):
        for j in range(1, 4):
            assert su[i, j, 1] == pytest.approx(rule.source(F, "u", (2, j, i)), rel=1e-14)
