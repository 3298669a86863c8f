"""Planted mistakes in copies of the oracle must each fail some pin (CPU only).

Each mutant is one plausible slip -- a wrong neighbour index, a dropped term, a
flipped sign, a transposed operand, swapped coefficients, a wrong loop bound --
written into a temporary copy of the oracle's C source and compiled with the
oracle's own flags.  The pins of ``oracle_pins`` must reject every one of them,
and (apart from the exact brute force) the pins that rest on closed forms and
invariants must reject each one too, so the oracle is not pinned only by a
second evaluation of the same formulas.
"""
import os
import subprocess

import pytest

import oracle
import oracle_pins

# (name, text in pw_oracle.c, replacement, occurrence index)
MUTANTS = [
    ("su_x_wrong_neighbour", "AT(u, k, j, i - 1) * (AT(u, k, j, i) + AT(u, k, j, i - 1))",
     "AT(u, k, j, i + 1) * (AT(u, k, j, i) + AT(u, k, j, i - 1))", 0),
    ("su_y_wrong_stagger", "(AT(v, k, j - 1, i) + AT(v, k, j - 1, i + 1))",
     "(AT(v, k, j - 1, i) + AT(v, k, j - 1, i - 1))", 0),
    ("su_y_transposed", "AT(u, k, j - 1, i) * (AT(v, k, j - 1, i)",
     "AT(v, k, j - 1, i) * (AT(u, k, j - 1, i)", 0),
    ("su_z_coeffs_swapped", "tzc1[k - 1] * AT(u, k - 1, j, i)", "tzc2[k - 1] * AT(u, k - 1, j, i)", 0),
    ("su_top_bound", "if (k < nz)\n                    s = s + tzc1[k - 1] * AT(u,",
     "if (k < nz - 1)\n                    s = s + tzc1[k - 1] * AT(u,", 0),
    ("sv_x_dropped", "s = s + tcx * (AT(v, k, j, i - 1)", "s = s + 0.0 * (AT(v, k, j, i - 1)", 0),
    ("sv_x_coeff", "s = s + tcx * (AT(v, k, j, i - 1)", "s = s + tcy * (AT(v, k, j, i - 1)", 0),
    ("sv_z_wrong_stagger", "(AT(w, k - 1, j, i) + AT(w, k - 1, j + 1, i))",
     "(AT(w, k - 1, j, i) + AT(w, k - 1, j, i + 1))", 0),
    ("sv_own_sign", "s = tcy * (AT(v, k, j - 1, i) * (AT(v, k, j, i) + AT(v, k, j - 1, i))\n"
     "                           - AT(v, k, j + 1, i)",
     "s = tcy * (AT(v, k, j - 1, i) * (AT(v, k, j, i) + AT(v, k, j - 1, i))\n"
     "                           + AT(v, k, j + 1, i)", 0),
    ("sw_z_sign", "- tzd2[k - 1]", "+ tzd2[k - 1]", 0),
    ("sw_x_wrong_level", "AT(u, k + 1, j, i - 1)", "AT(u, k - 1, j, i - 1)", 0),
    ("sw_y_coeff", "s = s + tcy * (AT(w, k, j - 1, i)", "s = s + tcx * (AT(w, k, j - 1, i)", 0),
    ("sw_z_coeff_level", "tzd1[k - 1] * AT(w, k - 1, j, i)", "tzd1[k - 2] * AT(w, k - 1, j, i)", 0),
    ("sw_bottom_not_cleared", "AT(sw, 1, j, i) = 0.0;", "", 0),
    ("su_x_dropped", "s = tcx * (AT(u, k, j, i - 1)", "s = 0.0 * (AT(u, k, j, i - 1)", 0),
]


def _mutate(src, old, new, occ):
    idx = -1
    for _ in range(occ + 1):
        idx = src.find(old, idx + 1)
        assert idx >= 0, "mutation anchor not found: %r" % old
    return src[:idx] + new + src[idx + len(old):]


@pytest.fixture(scope="module")
def source():
    with open(oracle.SOURCE) as f:
        return f.read()


@pytest.mark.parametrize("name,old,new,occ", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(source, name, old, new, occ, tmp_path):
    mutated = _mutate(source, old, new, occ)
    assert mutated != source
    c = tmp_path / "mutant.c"
    so = tmp_path / "libmutant.so"
    c.write_text(mutated)
    subprocess.run(["gcc", *oracle.CFLAGS, str(c), "-o", str(so)], check=True)
    lib = oracle.bind(str(so))

    def adv(*a, **kw):
        return oracle.advect(*a, lib=lib, **kw)

    caught = []
    for pin_name, pin in oracle_pins.ALL_PINS.items():
        try:
            pin(adv)
        except AssertionError:
            caught.append(pin_name)
    assert "exact_rule" in caught, "%s not caught by the exact brute force" % name
    others = [p for p in caught if p != "exact_rule"]
    assert others, "%s caught only by the brute force" % name
