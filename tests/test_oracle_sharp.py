"""Pins of the oracle's on-surface evaluation with the modified smoothing functions s1#, s2#, s3#
(paper section 2.1), one delta = 3h, no extrapolation.

- Taylor limits: s1# ~ (16/(3 sqrt pi)) t, s2# ~ (32/(3 sqrt pi)) t^3, s3# ~ (64/(45 sqrt pi)) t^5
  (from the series of erf and exp), and continuity where the oracle switches to its series;
- s# -> 1 beyond the cut-off;
- single layer of the translating and rotating unit sphere on the surface: (2/3) g and
  (1/3) Omega x y (Stokes), to an error that falls like h^5 (ratio > 16 per halving);
- double layer of a rigid motion on the surface: exactly (1/2)(U + Omega x y);
- the on-surface values converge to the extrapolated method's (difference falling > 10x per halving).
"""
import math

import numpy as np
import pytest

import oracle
from workload import harmonic_coeffs, harmonic_field, sphere_quadrature

SQPI = math.sqrt(math.pi)
DELTA_RHO = 3.0


def test_sharp_taylor_limits_and_switch():
    t = 1e-16
    s = oracle.smoothing_sharp(t)
    assert abs(s[0] / t / (16 / (3 * SQPI)) - 1) < 1e-15
    assert abs(s[1] / t ** 3 / (32 / (3 * SQPI)) - 1) < 1e-15
    assert abs(s[2] / t ** 5 / (64 / (45 * SQPI)) - 1) < 1e-15
    lo, hi = oracle.smoothing_sharp(0.2 - 1e-12), oracle.smoothing_sharp(0.2 + 1e-12)
    np.testing.assert_allclose(lo, hi, rtol=1e-9)
    # a few steps into the series region: second-order Taylor terms, read off erf and exp
    t = 1e-3
    s = oracle.smoothing_sharp(t)
    assert abs(s[0] / (2 / SQPI) - (8 / 3 * t - 8 / 3 * t ** 3)) < 1e-14  # the t^5 term is ~1.6e-15


def test_sharp_cutoff():
    assert np.all(oracle.smoothing_sharp(6.0 + 1e-12) == 1.0)
    # at the cut-off the polynomial factors (up to 4 t^5) leave e^{-36} 4 * 6^5 ~ 7e-12
    s = oracle.smoothing_sharp(6.0)
    assert np.all(np.abs(s - 1) < 1e-11)


def _on_surface(h):
    s = sphere_quadrature(h)
    return s


@pytest.mark.parametrize("kind", ["translate", "rotate"])
def test_sl_sharp_sphere_order(kind):
    errs = []
    g = np.array([0.3, -0.7, 0.5])
    Om = np.array([0.2, 0.9, -0.4])
    for inv_h in (8, 16):
        h = 1 / inv_h
        s = _on_surface(h)
        f = np.tile(g, (s.n, 1)) if kind == "translate" else np.cross(Om, s.x)
        u = oracle.sl_sharp(s.x, s.normal, s.w, f, s.x, s.normal, f, DELTA_RHO * h)
        ex = np.tile(2 / 3 * g, (s.n, 1)) if kind == "translate" else np.cross(Om, s.x) / 3
        errs.append(np.abs(u - ex).max())
    print(kind, errs)
    assert errs[1] < 2e-4 and errs[0] / errs[1] > 16


def test_dl_sharp_rigid_motion_exact():
    # with the unsplit stresslet, d . (q(x) - q(y)) = 0 for a rigid motion, so v = q(y)/2 exactly
    h = 1 / 16
    s = _on_surface(h)
    U = np.array([0.4, -0.2, 0.9])
    Om = np.array([-0.3, 0.5, 0.7])
    q = U + np.cross(Om, s.x)
    v = oracle.dl_sharp(s.x, s.normal, s.w, q, s.x, s.normal, q, DELTA_RHO * h)
    assert np.abs(v - 0.5 * q).max() < 1e-14


@pytest.mark.parametrize("layer", ["sl", "dl"])
def test_sharp_converges_to_the_extrapolated_value(layer):
    # both methods approximate the same on-surface integral to high order: their difference falls by
    # more than 10x per halving of h (a single delta with the original factors stays O(delta) apart)
    co = harmonic_coeffs(2, np.random.default_rng(4))
    base = sphere_quadrature(1 / 8)
    y, nn = base.x[::5], base.normal[::5]
    diffs = []
    for inv_h in (16, 32):
        h = 1 / inv_h
        s = sphere_quadrature(h)
        f, f0 = harmonic_field(co, s.x), harmonic_field(co, y)
        zero = np.zeros(len(y))
        if layer == "sl":
            a = oracle.sl_sharp(s.x, s.normal, s.w, f, y, nn, f0, DELTA_RHO * h)
            b = oracle.sl(s.x, s.normal, s.w, f, y, y, nn, zero, f0, h, (2, 3, 4))
        else:
            a = oracle.dl_sharp(s.x, s.normal, s.w, f, y, nn, f0, DELTA_RHO * h)
            b = oracle.dl(s.x, s.normal, s.w, f, y, y, nn, zero, f0, h, (2, 3, 4))
        diffs.append(np.abs(a - b).max() / np.abs(b).max())
    print(layer, diffs)
    assert diffs[1] < 3e-4 and diffs[0] / diffs[1] > 10
