"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each pin is a function of an ``adv`` callable with the oracle's signature
``adv(u, v, w, tcx, tcy, tzc1, tzc2, tzd1, tzd2, out=None) -> (su, sv, sw)``
and raises AssertionError when the fact does not hold.  The suite runs every
pin on the real oracle, and also on copies of the oracle with planted
mistakes, to show that each plausible mistake is caught.

What each pin rests on:

exact_rule      exact-rational evaluation, at every point of tiny grids, of
                the staggering rule that Listing 1 (Sec. II-A) instantiates;
                dyadic inputs make every FP64 operation exact, so equality is
                bit for bit.  The rule's u-case is itself checked against a
                literal writing-out of Listing 1.
uniform         uniform winds with tzc1 = tzc2 and tzd1 = tzd2: every flux
                difference cancels (zero tendency); the truncated top level
                keeps only the lower vertical flux, su(nz) = 2 c U W.
linear          a wind linear along one axis gives the closed form
                -6 * coef * phi * slope for the self-advection term.
textbook        uniform advecting velocity reduces each cross term to the
                centred difference -U dphi/dx (numpy.gradient), sign and axis
                included.
energy          density-weighted sum of u*su, v*sv, w*sw vanishes under
                periodic x-y and w = 0 at bottom and lid (telescoping fluxes).
divfree         domain sums of su, sv vanish for a discretely divergence-free
                horizontal wind (stream function) and w = 0.
scaling         outputs are quadratic in the winds: x2 and x1/2 scale them by
                exactly 4 and 1/4.
translation     periodic shift of the fields shifts the outputs, bit for bit.
mirror          sv is su with the x and y roles (fields, axes, coefficients)
                exchanged, bit for bit.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

import staggered_rule as rule
from paper_2107_13500_amd import inputs

SENTINEL = np.nan


def _outs(shape):
    return tuple(np.full(shape, SENTINEL) for _ in range(3))


def _run(adv, u, v, w, tcx, tcy, c1, c2, d1, d2):
    return adv(u, v, w, tcx, tcy, np.asarray(c1, float), np.asarray(c2, float),
               np.asarray(d1, float), np.asarray(d2, float), out=_outs(u.shape))


def _check_unwritten_halo(outs):
    for o in outs:
        for face in (o[0], o[-1], o[:, 0], o[:, -1]):
            assert np.all(np.isnan(face)), "halo column of an output was written"


def _dyadic(rng, shape, lo=-8, hi=8, den=4):
    return rng.integers(lo, hi + 1, size=shape).astype(np.float64) / den


# ----------------------------------------------------------------------------
def pin_exact_rule(adv):
    rng = np.random.default_rng(7)
    for (nx, ny, nz) in [(1, 1, 2), (2, 3, 3), (3, 4, 5), (5, 4, 6)]:
        shp = (nx + 2, ny + 2, nz)
        # halos are random and unrelated to the interior: the stencil must read
        # exactly the halo cells the rule names, nothing periodic is assumed
        u, v, w = (_dyadic(rng, shp) for _ in range(3))
        tcx, tcy = 0.375, 0.3125
        c1, c2, d1, d2 = (_dyadic(rng, nz, 1, 8, 8) for _ in range(4))
        su, sv, sw = _run(adv, u, v, w, tcx, tcy, c1, c2, d1, d2)
        _check_unwritten_halo((su, sv, sw))
        F = rule.Fields(u, v, w, tcx, tcy, c1, c2, d1, d2)
        exact = rule.all_sources(F, nx, ny)
        for name, got in (("u", su), ("v", sv), ("w", sw)):
            for (k, j, i), val in exact[name].items():
                g = got[i, j, k - 1]
                assert np.isfinite(g), "s%s(%d,%d,%d) not written" % (name, k, j, i)
                assert Fraction(g) == val, "s%s(%d,%d,%d) = %r, rule gives %s (shape %s)" % (
                    name, k, j, i, g, val, (nx, ny, nz))


def pin_uniform(adv):
    nx, ny, nz = 4, 3, 7
    shp = (nx + 2, ny + 2, nz)
    U, V, W = 1.5, -0.75, 0.625
    c, d = 0.125, 0.375
    u, v, w = np.full(shp, U), np.full(shp, V), np.full(shp, W)
    su, sv, sw = _run(adv, u, v, w, 0.25, 0.5, [c] * nz, [c] * nz, [d] * nz, [d] * nz)
    _check_unwritten_halo((su, sv, sw))
    I = (slice(1, nx + 1), slice(1, ny + 1))
    for o in (su, sv, sw):
        assert np.all(o[I][:, :, 0] == 0.0), "k = 1 must be 0"
        assert np.all(o[I][:, :, 1:nz - 1] == 0.0), "uniform winds must give zero tendency"
    assert np.all(su[I][:, :, nz - 1] == 2 * c * U * W), "su(nz) = 2 c U W"
    assert np.all(sv[I][:, :, nz - 1] == 2 * c * V * W), "sv(nz) = 2 c V W"
    assert np.all(sw[I][:, :, nz - 1] == 0.0), "sw(nz) = 0"


def pin_linear(adv):
    nx, ny, nz = 5, 4, 6
    shp = (nx + 2, ny + 2, nz)
    i = np.arange(nx + 2)[:, None, None]
    j = np.arange(ny + 2)[None, :, None]
    k = np.arange(1, nz + 1)[None, None, :]
    a, b = 3.0, 0.5
    tcx, tcy, c = 0.25, 0.125, 0.0625
    zero = np.zeros(shp)
    I = (slice(1, nx + 1), slice(1, ny + 1), slice(1, nz))
    # u linear in x, v = w = 0: su = tcx * (-6 u b); halo continues the line
    u = np.broadcast_to(a + b * i, shp).copy()
    su, sv, sw = _run(adv, u, zero, zero, tcx, tcy, [c] * nz, [c] * nz, [c] * nz, [c] * nz)
    assert np.array_equal(su[I], (tcx * (-6.0 * u * b))[I]), "su of a linear u(x)"
    assert np.all(sv[I] == 0.0) and np.all(sw[I] == 0.0)
    # v linear in y: sv = tcy * (-6 v b)
    v = np.broadcast_to(a + b * j, shp).copy()
    su, sv, sw = _run(adv, zero, v, zero, tcx, tcy, [c] * nz, [c] * nz, [c] * nz, [c] * nz)
    assert np.array_equal(sv[I], (tcy * (-6.0 * v * b))[I]), "sv of a linear v(y)"
    # w linear in z, constant tzd: sw = c * (-6 w b) for k = 2..nz-1
    w = np.broadcast_to(a + b * k, shp).copy()
    su, sv, sw = _run(adv, zero, zero, w, tcx, tcy, [0.0] * nz, [0.0] * nz, [c] * nz, [c] * nz)
    K = (slice(1, nx + 1), slice(1, ny + 1), slice(1, nz - 1))
    assert np.array_equal(sw[K], (c * (-6.0 * w * b))[K]), "sw of a linear w(z)"


def _smooth(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape)


def pin_textbook(adv):
    nx, ny, nz = 6, 5, 7
    shp = (nx + 2, ny + 2, nz)
    dx, dy, dzz = 40.0, 25.0, 10.0
    tcx, tcy, cz = 0.25 / dx, 0.25 / dy, 0.25 / dzz
    U, V, W = 3.0, -2.0, 0.7
    zeros = [0.0] * nz
    I = (slice(1, nx + 1), slice(1, ny + 1), slice(1, nz - 1))   # k = 2..nz-1

    def close(a, b, what):
        scale = max(np.max(np.abs(b)), 1e-300)
        assert np.max(np.abs(a - b)) <= 1e-13 * scale, what

    phi = _smooth(shp, 1)
    ones = np.ones(shp)
    # su: y term with uniform v, others off  ->  -V du/dy
    su, _, _ = _run(adv, phi, V * ones, np.zeros(shp), 0.0, tcy, zeros, zeros, zeros, zeros)
    close(su[I], -V * np.gradient(phi, dy, axis=1)[I], "su y-term = -V du/dy")
    # su: vertical term with uniform w and tzc1 = tzc2 -> -W du/dz
    su, _, _ = _run(adv, phi, np.zeros(shp), W * ones, 0.0, 0.0, [cz] * nz, [cz] * nz, zeros, zeros)
    close(su[I], -W * np.gradient(phi, dzz, axis=2)[I], "su z-term = -W du/dz")
    # sv: x term with uniform u -> -U dv/dx
    _, sv, _ = _run(adv, U * ones, phi, np.zeros(shp), tcx, 0.0, zeros, zeros, zeros, zeros)
    close(sv[I], -U * np.gradient(phi, dx, axis=0)[I], "sv x-term = -U dv/dx")
    # sv: vertical term with uniform w -> -W dv/dz
    _, sv, _ = _run(adv, np.zeros(shp), phi, W * ones, 0.0, 0.0, [cz] * nz, [cz] * nz, zeros, zeros)
    close(sv[I], -W * np.gradient(phi, dzz, axis=2)[I], "sv z-term = -W dv/dz")
    # sw: horizontal terms with uniform u, v -> -U dw/dx - V dw/dy
    _, _, sw = _run(adv, U * ones, V * ones, phi, tcx, tcy, zeros, zeros, zeros, zeros)
    ref = -U * np.gradient(phi, dx, axis=0) - V * np.gradient(phi, dy, axis=1)
    close(sw[I], ref[I], "sw horizontal = -U dw/dx - V dw/dy")


def _periodic_problem(nx, ny, nz, seed, dx=50.0, dy=50.0):
    p = inputs.make_problem(nx, ny, nz, seed, dx=dx, dy=dy)
    return p


def pin_energy(adv):
    p = _periodic_problem(12, 10, 9, 11, dx=40.0, dy=55.0)
    c, g = p.coeffs, p.grid
    su, sv, sw = adv(p.u, p.v, p.w, c.tcx, c.tcy, c.tzc1, c.tzc2, c.tzd1, c.tzd2, out=_outs(p.u.shape))
    I = (slice(1, -1), slice(1, -1))
    wu = (g.rho * g.dz)[None, None, 1:]                      # k = 2..nz
    wwk = (g.rho_w[1:-1] * g.dzn[2:])[None, None, :]         # k = 2..nz-1
    for a, s, wt, K, name in ((p.u, su, wu, slice(1, None), "u"), (p.v, sv, wu, slice(1, None), "v"),
                              (p.w, sw, wwk, slice(1, -1), "w")):
        terms = (wt * a[I][:, :, K] * s[I][:, :, K])
        tot, mag = terms.sum(), np.abs(terms).sum()
        assert abs(tot) <= 1e-12 * mag, "weighted sum of %s*s%s = %g (|.| %g)" % (name, name, tot, mag)


def pin_divfree(adv):
    nx, ny, nz = 10, 8, 5
    dx, dy = 30.0, 45.0
    rng = np.random.default_rng(3)
    # stream function at corners (i+1/2, j+1/2), periodic in x and y
    psi = rng.standard_normal((nx, ny, nz))
    shp = (nx + 2, ny + 2, nz)
    u = np.zeros(shp)
    v = np.zeros(shp)
    for i in range(1, nx + 1):
        for j in range(1, ny + 1):
            ii, jj = i % nx, j % ny
            u[i, j] = 4.0 - (psi[ii, jj] - psi[ii, (jj - 1) % ny]) / dy
            v[i, j] = -1.5 + (psi[ii, jj] - psi[(ii - 1) % nx, jj]) / dx
    inputs.fill_periodic_halo(u)
    inputs.fill_periodic_halo(v)
    w = np.zeros(shp)
    cz = [0.01] * nz
    su, sv, _ = adv(u, v, w, 0.25 / dx, 0.25 / dy, np.array(cz), np.array(cz), np.array(cz),
                    np.array(cz), out=_outs(shp))
    I = (slice(1, -1), slice(1, -1), slice(1, None))
    for s, name in ((su, "su"), (sv, "sv")):
        tot, mag = s[I].sum(), np.abs(s[I]).sum()
        assert abs(tot) <= 1e-13 * mag, "sum of %s = %g (|.| %g)" % (name, tot, mag)


def pin_scaling(adv):
    p = _periodic_problem(7, 6, 8, 5)
    c = p.coeffs
    base = adv(p.u, p.v, p.w, c.tcx, c.tcy, c.tzc1, c.tzc2, c.tzd1, c.tzd2, out=_outs(p.u.shape))
    I = (slice(1, -1), slice(1, -1))
    for f in (2.0, 0.5):
        sc = adv(f * p.u, f * p.v, f * p.w, c.tcx, c.tcy, c.tzc1, c.tzc2, c.tzd1, c.tzd2,
                 out=_outs(p.u.shape))
        for a, b in zip(base, sc):
            assert np.array_equal(b[I], (f * f) * a[I]), "outputs must scale by exactly %g" % (f * f)


def pin_translation(adv):
    p = _periodic_problem(8, 6, 6, 9)
    c = p.coeffs
    base = adv(p.u, p.v, p.w, c.tcx, c.tcy, c.tzc1, c.tzc2, c.tzd1, c.tzd2, out=_outs(p.u.shape))
    si, sj = 3, 2
    rolled = []
    for a in (p.u, p.v, p.w):
        r = np.zeros_like(a)
        r[1:-1, 1:-1] = np.roll(a[1:-1, 1:-1], (si, sj), axis=(0, 1))
        rolled.append(inputs.fill_periodic_halo(r))
    sh = adv(*rolled, c.tcx, c.tcy, c.tzc1, c.tzc2, c.tzd1, c.tzd2, out=_outs(p.u.shape))
    for a, b in zip(base, sh):
        assert np.array_equal(np.roll(a[1:-1, 1:-1], (si, sj), axis=(0, 1)), b[1:-1, 1:-1]), \
            "outputs must shift with the fields"


def pin_mirror(adv):
    p = _periodic_problem(7, 5, 6, 13, dx=35.0, dy=60.0)
    c = p.coeffs
    su, sv, sw = adv(p.u, p.v, p.w, c.tcx, c.tcy, c.tzc1, c.tzc2, c.tzd1, c.tzd2, out=_outs(p.u.shape))
    T = lambda a: np.ascontiguousarray(np.swapaxes(a, 0, 1))
    su_m, _, _ = adv(T(p.v), T(p.u), T(p.w), c.tcy, c.tcx, c.tzc1, c.tzc2, c.tzd1, c.tzd2,
                     out=_outs(T(p.u).shape))
    assert np.array_equal(T(su_m)[1:-1, 1:-1], sv[1:-1, 1:-1]), "sv must be the x<->y mirror of su"


ALL_PINS = {
    "exact_rule": pin_exact_rule,
    "uniform": pin_uniform,
    "linear": pin_linear,
    "textbook": pin_textbook,
    "energy": pin_energy,
    "divfree": pin_divfree,
    "scaling": pin_scaling,
    "translation": pin_translation,
    "mirror": pin_mirror,
}
