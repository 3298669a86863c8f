"""Exact-rational brute force of the PW source terms from one staggering rule.

This evaluator is deliberately *not* a transcription of the oracle's three
formulas.  It encodes the single rule that Listing 1 (paper Sec. II-A)
instantiates for u, and applies that same rule to v and w:

* u lives on x faces, v on y faces, w on z faces (Arakawa C grid), so the
  control volume of a quantity phi at index c is centred at c + e_phi / 2;
* along each axis d, the source term is (flux in through the lower face) minus
  (flux out through the upper face), each flux being
  coefficient x phi(c -/+ e_d) x (sum of the two values of the d-velocity
  that straddle that face);
* horizontal coefficients (tcx, tcy) are common to both faces and multiply the
  difference; vertical ones are per level: tzc1/tzc2 for u and v, tzd1/tzd2
  for w;
* u and v are computed for k = 2..nz with the upper vertical flux dropped at
  k = nz (Listing 1); w for k = 2..nz-1; every other level is 0.

Arithmetic is done in ``fractions.Fraction`` (exact) or any number type that
supports + - * -- the op-counting type below checks the per-field operation
count of paper Sec. III.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Dict, Tuple

AXES = {"x": (0, 0, 1), "y": (0, 1, 0), "z": (1, 0, 0)}   # offsets in (k, j, i)
STAGGER = {"u": "x", "v": "y", "w": "z"}                  # face each quantity sits on
VELOCITY = {"x": "u", "y": "v", "z": "w"}                 # velocity along each axis
# Order of the three directional terms in each output (Listing 1 for u; the
# mirror for v; x, y, z for w).  Only matters for op-count bookkeeping.
TERM_ORDER = {"u": ("x", "y", "z"), "v": ("y", "x", "z"), "w": ("x", "y", "z")}


def _add(c, e, s=1):
    return (c[0] + s * e[0], c[1] + s * e[1], c[2] + s * e[2])


class Fields:
    """Accessor for halo'd fields given as nested python lists/arrays a[i][j][k-1]."""

    def __init__(self, u, v, w, tcx, tcy, tzc1, tzc2, tzd1, tzd2, conv=Fraction):
        self.f = {"u": u, "v": v, "w": w}
        self.tcx, self.tcy = conv(tcx), conv(tcy)
        self.tz = {"c1": tzc1, "c2": tzc2, "d1": tzd1, "d2": tzd2}
        self.conv = conv
        self.nz = len(tzc1)

    def at(self, name, c):
        k, j, i = c
        return self.conv(self.f[name][i][j][k - 1])

    def tzk(self, which, k):
        return self.conv(self.tz[which][k - 1])


def term(F: Fields, phi: str, d: str, c: Tuple[int, int, int], drop_upper: bool):
    """Directional source term of quantity ``phi`` along axis ``d`` at cell c."""
    e_d = AXES[d]
    e_phi = AXES[STAGGER[phi]]
    adv = VELOCITY[d]
    own = STAGGER[phi] == d

    def face_velocity(upper: bool):
        if own:
            # phi's control-volume faces along its own axis are cell centres:
            # the advecting velocity there is phi itself, summed across the centre
            return F.at(phi, c) + F.at(phi, _add(c, e_d, 1 if upper else -1))
        # the d-velocity summed across phi's offset, on the lower or upper face
        base = c if upper else _add(c, e_d, -1)
        return F.at(adv, base) + F.at(adv, _add(base, e_phi))

    def flux(upper: bool):
        phi_n = F.at(phi, _add(c, e_d, 1 if upper else -1))
        return phi_n, face_velocity(upper)

    k = c[0]
    if d in ("x", "y"):
        tc = F.tcx if d == "x" else F.tcy
        p_lo, a_lo = flux(False)
        p_hi, a_hi = flux(True)
        return tc * (p_lo * a_lo - p_hi * a_hi)
    c_lo, c_hi = ("c1", "c2") if phi in ("u", "v") else ("d1", "d2")
    p_lo, a_lo = flux(False)
    lower = F.tzk(c_lo, k) * p_lo * a_lo
    if drop_upper:
        return lower
    p_hi, a_hi = flux(True)
    return lower - F.tzk(c_hi, k) * p_hi * a_hi


def source(F: Fields, phi: str, c: Tuple[int, int, int]):
    """su, sv or sw at cell c = (k, j, i) by the staggering rule."""
    k = c[0]
    nz = F.nz
    if k < 2 or k > nz or (phi == "w" and k == nz):
        return F.conv(0)
    drop = (phi in ("u", "v")) and k == nz
    total = None
    for d in TERM_ORDER[phi]:
        t = term(F, phi, d, c, drop_upper=(drop and d == "z"))
        total = t if total is None else total + t
    return total


def listing1_su(F: Fields, c):
    """Listing 1 of the paper, written out literally (the u field only)."""
    k, j, i = c
    u = lambda kk, jj, ii: F.at("u", (kk, jj, ii))
    v = lambda kk, jj, ii: F.at("v", (kk, jj, ii))
    w = lambda kk, jj, ii: F.at("w", (kk, jj, ii))
    s = F.tcx * (u(k, j, i - 1) * (u(k, j, i) + u(k, j, i - 1)) - u(k, j, i + 1) * (u(k, j, i) + u(k, j, i + 1)))
    s = s + F.tcy * (u(k, j - 1, i) * (v(k, j - 1, i) + v(k, j - 1, i + 1)) - u(k, j + 1, i) * (v(k, j, i) + v(k, j, i + 1)))
    if k < F.nz:
        s = s + F.tzk("c1", k) * u(k - 1, j, i) * (w(k - 1, j, i) + w(k - 1, j, i + 1)) - F.tzk("c2", k) * u(k + 1, j, i) * (w(k, j, i) + w(k, j, i + 1))
    else:
        s = s + F.tzk("c1", k) * u(k - 1, j, i) * (w(k - 1, j, i) + w(k - 1, j, i + 1))
    return s


class Counted:
    """A number that counts the + - * operations applied to it (shared counter)."""

    ops = 0

    def __init__(self, x):
        self.x = x.x if isinstance(x, Counted) else Fraction(x)

    @staticmethod
    def _v(o):
        return o.x if isinstance(o, Counted) else Fraction(o)

    def __add__(self, o):
        Counted.ops += 1
        return Counted(self.x + self._v(o))

    __radd__ = __add__

    def __sub__(self, o):
        Counted.ops += 1
        return Counted(self.x - self._v(o))

    def __rsub__(self, o):
        Counted.ops += 1
        return Counted(self._v(o) - self.x)

    def __mul__(self, o):
        Counted.ops += 1
        return Counted(self.x * self._v(o))

    __rmul__ = __mul__


def op_count(F: Fields, phi: str, c) -> int:
    Counted.ops = 0
    source(F, phi, c)
    return Counted.ops


def all_sources(F: Fields, nx: int, ny: int) -> Dict[str, dict]:
    """Exact su, sv, sw at every computed point: {name: {(k, j, i): value}}."""
    out = {"u": {}, "v": {}, "w": {}}
    for i in range(1, nx + 1):
        for j in range(1, ny + 1):
            for k in range(1, F.nz + 1):
                for phi in ("u", "v", "w"):
                    out[phi][(k, j, i)] = source(F, phi, (k, j, i))
    return out
