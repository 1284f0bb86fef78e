"""Pins of the FP64 CPU oracle against facts fixed by the paper and by Stokes-flow mathematics.

Nothing here re-types the oracle's formulas: each check is a value the paper prints, a closed form,
an exact rational, a derivative identity, or a limit.  A dropped term, a wrong sign, a wrong index
or a transposed operand in the oracle fails at least one of them:
  - smoothing factors: small-t limits (regularity of s_k / t^(2k-1)), derivative identities, t > 6 cut-off;
  - I0, I2: values at 0 and derivative identities I0' = -erfc, I2' = -2 lambda I0;
  - extrapolation: exact on-surface weights (14/3, -16/3, 5/3) and (15/2, -10, 7/2), sum of weights 1;
  - single layer: translating and rotating unit sphere (Stokes' solution), at and near the surface;
  - double layer: rigid-body densities give chi (U + Omega x y), constant densities give chi q exactly;
  - far targets: brute force with the plain quadrature at h/4;
  - order: self-convergence ratio of about 2^5 under refinement.
"""
import math

import numpy as np
import pytest

import oracle
from workload import (closest_point_ellipsoid, concat_targets, ellipsoid_normal, ellipsoid_quadrature,
                      harmonic_coeffs, harmonic_field, near_targets, on_surface_targets, sphere_quadrature)

SQPI = math.sqrt(math.pi)


# ---------------------------------------------------------------- smoothing factors, eqs. (s1)-(s3)

def test_smoothing_small_t_limits():
    # s1 ~ (2/sqrt pi) t, s2 ~ (4/(3 sqrt pi)) t^3, s3 ~ (8/(15 sqrt pi)) t^5: the regularized kernels
    # s1/r, s2/r^3, s3/r^5 stay bounded at r = 0 (first Taylor terms of erf t - polynomial * e^{-t^2})
    t = 1e-2
    s = oracle.smoothing(t)
    assert abs(s[0] / t / (2 / SQPI) - 1) < 1e-4
    assert abs(s[1] / t ** 3 / (4 / (3 * SQPI)) - 1) < 1e-3
    assert abs(s[2] / t ** 5 / (8 / (15 * SQPI)) - 1) < 1e-3


@pytest.mark.parametrize("t", [0.2, 0.7, 1.3, 2.0, 3.1, 4.5])
def test_smoothing_derivatives(t):
    # d/dt s1 = (2/sqrt pi) e^{-t^2}; d/dt s2 = (4/sqrt pi) t^2 e^{-t^2}; d/dt s3 = (8/(3 sqrt pi)) t^4 e^{-t^2}
    eps = 1e-5
    ds = (oracle.smoothing(t + eps) - oracle.smoothing(t - eps)) / (2 * eps)
    e = math.exp(-t * t)
    expect = [2 / SQPI * e, 4 / SQPI * t * t * e, 8 / (3 * SQPI) * t ** 4 * e]
    np.testing.assert_allclose(ds, expect, rtol=1e-6, atol=2e-10)


def test_smoothing_cutoff():
    # section 3.2: s1 = s2 = s3 = 1 for t > 6; the tails (1 - s_k)/t^(2k-1) at t = 6 are below 1e-17
    assert np.all(oracle.smoothing(6.0 + 1e-9) == 1.0)
    assert np.all(oracle.smoothing(40.0) == 1.0)
    s6 = oracle.smoothing(6.0)
    tails = [(1 - s6[0]) / 6, (1 - s6[1]) / 6 ** 3, (1 - s6[2]) / 6 ** 5]
    assert max(abs(x) for x in tails) < 1e-17
    assert (1 - s6[2]) > 0  # s3(6) is still regularized (not exactly 1)


# ---------------------------------------------------------------- I0, I2, eqs. (I0), (I2)

def test_I0_I2_values_at_zero():
    assert abs(oracle.I0(0.0) - 1 / SQPI) < 1e-16
    assert abs(oracle.I2(0.0) - 1 / (3 * SQPI)) < 1e-16


@pytest.mark.parametrize("lam", [0.1, 0.5, 1.0, 1.7, 2.5])
def test_I0_I2_derivative_identities(lam):
    eps = 1e-6
    dI0 = (oracle.I0(lam + eps) - oracle.I0(lam - eps)) / (2 * eps)
    dI2 = (oracle.I2(lam + eps) - oracle.I2(lam - eps)) / (2 * eps)
    assert abs(dI0 + math.erfc(lam)) < 1e-9
    assert abs(dI2 + 2 * lam * oracle.I0(lam)) < 1e-9
    assert oracle.I0(-lam) == oracle.I0(lam) and oracle.I2(-lam) == oracle.I2(lam)


# ---------------------------------------------------------------- extrapolation, eq. (extrap_eqn)

def test_extrapolation_weights_on_surface():
    # b = 0: rows [1, rho/sqrt(pi), rho^3/(3 sqrt(pi))] give exact rational weights
    np.testing.assert_allclose(oracle.extrapolation_weights(0.0, 1 / 16, (2, 3, 4)), [14 / 3, -16 / 3, 5 / 3],
                               rtol=1e-13)
    np.testing.assert_allclose(oracle.extrapolation_weights(0.0, 1 / 64, (3, 4, 5)), [7.5, -10.0, 3.5], rtol=1e-13)


@pytest.mark.parametrize("b_over_h", [-3.0, -1.2, 0.4, 2.0, 5.5, 10.0])
def test_extrapolation_weights_sum_to_one(b_over_h):
    h = 1 / 32
    w = oracle.extrapolation_weights(b_over_h * h, h, (2, 3, 4))
    assert abs(w.sum() - 1) < 1e-12


def test_extrapolation_far_is_identity():
    h = 1 / 32
    np.testing.assert_array_equal(oracle.extrapolation_weights(24 * h, h, (2, 3, 4)), [1, 0, 0])


# ---------------------------------------------------------------- closed-form Stokes flows

def _sphere_targets(h, rng, n_on=250, n_near=250, far=True):
    s = sphere_quadrature(h)
    t_on = on_surface_targets(s).subset(np.arange(0, s.n, max(1, s.n // n_on)))
    t_near = near_targets((1, 1, 1), n_near, 3 * h, rng)
    parts = [t_on, t_near]
    if far:
        y = np.array([[1.6, 0.2, -0.3], [0.1, 0.2, -0.3], [-1.2, -1.1, 0.4], [0.0, 0.0, 2.5]])
        r = np.linalg.norm(y, axis=1)
        x0 = y / r[:, None]
        from workload.targets import Targets
        parts.append(Targets(y, x0, x0.copy(), r - 1.0, np.full(4, -1)))
    return s, concat_targets(*parts)


def _stokes_translate(g, y):
    r = np.linalg.norm(y, axis=1)[:, None]
    gy = (y @ g)[:, None]
    out = 0.5 * (g / r + gy * y / r ** 3) + (1 / 6) * (g / r ** 3 - 3 * gy * y / r ** 5)
    return np.where(r <= 1, 2 / 3 * g, out)


@pytest.mark.parametrize("inv_h,tol", [(16, 2e-5), (32, 1.5e-6)])
def test_sl_translating_sphere(inv_h, tol):
    # unit sphere, uniform force density g: u = (2/3) g on and inside; Stokes' flow outside
    rng = np.random.default_rng(100 + inv_h)
    h = 1 / inv_h
    s, t = _sphere_targets(h, rng)
    g = np.array([0.3, -0.7, 0.5])
    u = oracle.sl(s.x, s.normal, s.w, np.tile(g, (s.n, 1)), t.y, t.x0, t.n0, t.b, np.tile(g, (t.m, 1)), h,
                  (2, 3, 4))
    assert np.abs(u - _stokes_translate(g, t.y)).max() < tol


@pytest.mark.parametrize("inv_h,tol", [(16, 3e-5), (32, 2e-6)])
def test_sl_rotating_sphere(inv_h, tol):
    # f = Omega x x on the unit sphere: u = (1/3) Omega x y inside/on, (1/3) Omega x y / |y|^3 outside
    rng = np.random.default_rng(200 + inv_h)
    h = 1 / inv_h
    s, t = _sphere_targets(h, rng)
    Om = np.array([0.2, 0.9, -0.4])
    u = oracle.sl(s.x, s.normal, s.w, np.cross(Om, s.x), t.y, t.x0, t.n0, t.b, np.cross(Om, t.x0), h, (2, 3, 4))
    r = np.linalg.norm(t.y, axis=1)[:, None]
    ex = np.where(r <= 1, np.cross(Om, t.y) / 3, np.cross(Om, t.y) / (3 * r ** 3))
    assert np.abs(u - ex).max() < tol


@pytest.mark.parametrize("inv_h,tol", [(16, 4e-4), (32, 3e-5)])
def test_dl_rigid_motion(inv_h, tol):
    # q = U + Omega x x (rigid motion): v = chi(y) (U + Omega x y) (Lorentz reciprocal identity)
    rng = np.random.default_rng(300 + inv_h)
    h = 1 / inv_h
    s, t = _sphere_targets(h, rng)
    U = np.array([0.5, 0.1, -0.3])
    Om = np.array([0.2, 0.9, -0.4])
    q = U + np.cross(Om, s.x)
    q0 = U + np.cross(Om, t.x0)
    v = oracle.dl(s.x, s.normal, s.w, q, t.y, t.x0, t.n0, t.b, q0, h, (2, 3, 4))
    chi = np.where(t.b < 0, 1.0, np.where(t.b > 0, 0.0, 0.5))[:, None]
    assert np.abs(v - chi * (U + np.cross(Om, t.y))).max() < tol


def test_dl_rigid_motion_ellipsoid():
    # the identity holds on any closed surface; here on the ellipsoid at h = 1/32
    rng = np.random.default_rng(7)
    ax = (1.0, 0.8, 0.6)
    h = 1 / 32
    s = ellipsoid_quadrature(ax, h)
    t = concat_targets(on_surface_targets(s).subset(np.arange(0, s.n, 40)), near_targets(ax, 200, 3 * h, rng))
    U = np.array([-0.2, 0.4, 0.7])
    Om = np.array([0.6, -0.3, 0.2])
    chi = np.where(t.b < 0, 1.0, np.where(t.b > 0, 0.0, 0.5))[:, None]
    for rho, tol in (((2, 3, 4), 3e-4), ((3, 4, 5), 1e-3)):
        v = oracle.dl(s.x, s.normal, s.w, U + np.cross(Om, s.x), t.y, t.x0, t.n0, t.b, U + np.cross(Om, t.x0), h,
                      rho)
        assert np.abs(v - chi * (U + np.cross(Om, t.y))).max() < tol


def test_dl_constant_density_exact():
    # q constant: the subtracted integrand vanishes identically, so v = chi q exactly (eq. (Stokes_DL1))
    rng = np.random.default_rng(11)
    h = 1 / 16
    s, t = _sphere_targets(h, rng, far=False)
    qc = np.array([1.0, -2.0, 0.5])
    v = oracle.dl(s.x, s.normal, s.w, np.tile(qc, (s.n, 1)), t.y, t.x0, t.n0, t.b, np.tile(qc, (t.m, 1)), h,
                  (2, 3, 4))
    chi = np.where(t.b < 0, 1.0, np.where(t.b > 0, 0.0, 0.5))[:, None]
    np.testing.assert_array_equal(v, chi * qc)


def test_plain_dl_identity_far():
    # (1/8 pi) int T_ijk n_k dS = delta_ij inside, 0 outside (the identity behind the subtraction)
    s = sphere_quadrature(1 / 32)
    y = np.array([[0.1, -0.2, 0.15], [2.0, 0.5, -0.3]])
    for j in range(3):
        q = np.zeros((s.n, 3))
        q[:, j] = 1.0
        _, v = oracle.plain(s.x, s.normal, s.w, q, q, y)
        e = np.zeros(3)
        e[j] = 1.0
        assert np.abs(v[0] - e).max() < 1e-6
        assert np.abs(v[1]).max() < 1e-6


def test_far_targets_match_fine_plain_quadrature():
    # far from the surface no smoothing is active; the result equals the plain quadrature, which
    # converges rapidly: compare with the plain sum at h/4
    rng = np.random.default_rng(8)
    ax = (1.0, 0.8, 0.6)
    co = harmonic_coeffs(3, rng)
    y = np.array([[1.8, 0.3, -0.2], [0.1, -0.1, 0.05], [-0.2, 1.5, 0.9], [0.05, 0.02, -0.03]])
    x0, b = closest_point_ellipsoid(ax, y)
    n0 = ellipsoid_normal(ax, x0)
    h = 1 / 32
    s = ellipsoid_quadrature(ax, h)
    f = harmonic_field(co, s.x)
    f0 = harmonic_field(co, x0)
    u = oracle.sl(s.x, s.normal, s.w, f, y, x0, n0, b, f0, h, (2, 3, 4))
    v = oracle.dl(s.x, s.normal, s.w, f, y, x0, n0, b, f0, h, (2, 3, 4))
    sf = ellipsoid_quadrature(ax, h / 4)
    ff = harmonic_field(co, sf.x)
    us, vs = oracle.plain(sf.x, sf.normal, sf.w, ff, ff, y)
    assert np.abs(u - us).max() < 1e-6
    assert np.abs(v - vs).max() < 1e-5


@pytest.mark.slow
def test_self_convergence_order():
    # e_h = u_h - u_{h/2} (paper eq. (error_h)); about fifth order: the ratio should exceed 2^4
    rng = np.random.default_rng(9)
    ax = (1.0, 0.8, 0.6)
    co = harmonic_coeffs(3, rng)
    t = near_targets(ax, 150, 0.1, rng)
    f0 = harmonic_field(co, t.x0)
    us = []
    for inv_h in (16, 32, 64):
        s = ellipsoid_quadrature(ax, 1 / inv_h)
        us.append(oracle.sl(s.x, s.normal, s.w, harmonic_field(co, s.x), t.y, t.x0, t.n0, t.b, f0, 1 / inv_h,
                            (2, 3, 4)))
    e1 = np.abs(us[0] - us[1]).max()
    e2 = np.abs(us[1] - us[2]).max()
    assert e1 / e2 > 16


def test_smoothing_small_t_series_continuity():
    # below t = 0.2 the oracle evaluates s_k by their Maclaurin series; the two evaluations of the same
    # functions must agree across the switch, and s2/t^3, s3/t^5 must keep full relative accuracy at
    # tiny t (two quadrature points of different families can coincide up to rounding)
    lo, hi = oracle.smoothing(0.2 - 1e-12), oracle.smoothing(0.2 + 1e-12)
    np.testing.assert_allclose(lo, hi, rtol=1e-9)
    t = 1e-16
    s = oracle.smoothing(t)
    assert abs(s[0] / t / (2 / SQPI) - 1) < 1e-15
    assert abs(s[1] / t ** 3 / (4 / (3 * SQPI)) - 1) < 1e-15
    assert abs(s[2] / t ** 5 / (8 / (15 * SQPI)) - 1) < 1e-15
