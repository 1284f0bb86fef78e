"""The erfcx tables of the near-field kernels (paper_2507_00156_amd/csrc/sr_erfcx_table.h, written by
gen_erfcx.py): evaluated in float64 in the kernels' order of operations, exp(-t^2) L inv P(x) must
match erfc(t) from mpmath (an independent 40-digit reference) on [0, 6.25] within each table's
stated bound: 1e-15 for the double-precision path's degree-16 table, 2e-11 for the mixed path's
degree-11 table.  A wrong coefficient, degree or variable map fails by many orders of magnitude."""
import math
import os
import re
from fractions import Fraction

import mpmath
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_2507_00156_amd", "csrc", "sr_erfcx_table.h")


def tables():
    text = open(HEADER).read()
    out = {}
    for m in re.finditer(r"struct (\w+) \{(.*?)\n\};", text, re.S):
        body = m.group(2)

        def get(key):
            return float(re.search(rf"{key} = ([-+0-9.e]+);", body).group(1))

        out[m.group(1)] = dict(
            deg=int(re.search(r"kDegree = (\d+);", body).group(1)),
            L=get("kL"), A=get("kA"), B=get("kB"), err=get("kMaxErr"),
            c=[float(x) for x in re.findall(r"^\s+([-+0-9.e]+),$", body, re.M)])
    return out


def _fma(a, b, c):
    """a * b + c with one rounding (exact rational arithmetic, then one conversion to float)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def erfc_from_table(T, t):
    # the kernels' steps: inv = 1/(t + L), x = (A + B) - 2 A L inv, Horner on the coefficients times L,
    # erfcx = inv P_L(x) (_fma keeps the kernels' single roundings)
    inv = 1.0 / (t + T["L"])
    x = _fma(-2.0 * T["A"] * T["L"], inv, T["A"] + T["B"])
    cl = [T["L"] * c for c in T["c"]]
    p = cl[-1]
    for c in reversed(cl[:-1]):
        p = _fma(p, x, c)
    return math.exp(-t * t) * (inv * p)


@pytest.mark.parametrize("name,degree,bound", [("Fp64", 16, 1e-15), ("Mixed", 11, 2e-11)])
def test_table_matches_erfc(name, degree, bound):
    T = tables()[name]
    assert T["deg"] == degree and len(T["c"]) == degree + 1
    mpmath.mp.dps = 40
    worst = 0.0
    for i in range(1201):
        t = 6.25 * (i + 0.37) / 1201  # off the generator's own check grid
        worst = max(worst, abs(erfc_from_table(T, t) - float(mpmath.erfc(mpmath.mpf(t)))))
    assert worst <= bound, worst
    assert worst <= 2.0 * T["err"] + 2e-16  # consistent with the bound the generator recorded


def test_tables_share_the_variable_map():
    t = tables()
    assert set(t) == {"Fp64", "Mixed"}
    for k in ("L", "A", "B"):
        assert t["Fp64"][k] == t["Mixed"][k]
