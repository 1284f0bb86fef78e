"""Input generators pinned to the paper: Table 1 point counts, weight moments, target geometry."""
import os

import numpy as np
import pytest

import workload
from workload import (closest_point_ellipsoid, ellipsoid_normal, ellipsoid_quadrature, grid_targets_outside,
                      near_targets, sphere_quadrature)

SPHEROID = (1.0, 0.5, 0.5)  # x1^2 + 4 x2^2 + 4 x3^2 = 1, paper section 4.1
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_counts.txt")
TABLE1 = np.loadtxt(GOLDEN, dtype=np.int64, comments="#")


@pytest.mark.parametrize("inv_h,count", [(int(r[0]), int(r[1])) for r in TABLE1])
def test_quadrature_counts_table1(inv_h, count):
    # Table 1, column "# quads": grid-line intersections with |n_i| >= cos 70 deg (section 2.2)
    assert ellipsoid_quadrature(SPHEROID, 1.0 / inv_h).n == count


@pytest.mark.parametrize("inv_h,count", [(int(r[0]), int(r[2])) for r in TABLE1[:2]])
def test_target_counts_table1(inv_h, count):
    # Table 1, column "# targets": grid points outside the spheroid within distance h (section 4.1)
    t = grid_targets_outside(SPHEROID, 1.0 / inv_h)
    assert t.m == count
    assert np.all(t.b >= 0) and np.all(t.b <= (1 + 1e-12) / inv_h)


@pytest.mark.parametrize("inv_h,tol", [(16, 1e-4), (32, 2e-6), (64, 1e-8)])
def test_sphere_weights_moments(inv_h, tol):
    # the quadrature integrates smooth functions to high order: area 4 pi and int x1^2 = 4 pi / 3
    s = sphere_quadrature(1.0 / inv_h)
    assert abs(s.w.sum() - 4 * np.pi) < tol
    assert abs((s.w * s.x[:, 0] ** 2).sum() - 4 * np.pi / 3) < tol


def test_spheroid_area():
    # prolate spheroid (a=1, b=1/2): area = 2 pi b^2 (1 + a arcsin(e) / (b e)), e = sqrt(1 - b^2/a^2)
    e = np.sqrt(0.75)
    area = 2 * np.pi * 0.25 * (1 + np.arcsin(e) / (0.5 * e))
    errs = [abs(ellipsoid_quadrature(SPHEROID, 1.0 / k).w.sum() - area) for k in (32, 64, 128)]
    assert errs[0] < 2e-4 and errs[1] < 1e-6 and errs[2] < 1e-7


def test_ellipsoid_area_matches_quadrature():
    ax = (1.0, 0.8, 0.6)
    a = workload.ellipsoid_area(ax)
    assert abs(ellipsoid_quadrature(ax, 1 / 64).w.sum() - a) < 1e-7


def test_partition_of_unity_and_families():
    s = ellipsoid_quadrature((1.0, 0.8, 0.6), 1 / 32)
    cth = np.cos(np.deg2rad(70.0))
    fam = s.family
    assert np.all(np.abs(s.normal[np.arange(s.n), fam]) >= cth)
    assert np.all(s.w >= 0)
    np.testing.assert_allclose(np.linalg.norm(s.normal, axis=1), 1.0, atol=1e-14)
    # points lie on the surface
    F = ((s.x / np.array([1.0, 0.8, 0.6])) ** 2).sum(1)
    np.testing.assert_allclose(F, 1.0, atol=1e-13)


def test_near_targets_closest_point():
    ax = (1.0, 0.8, 0.6)
    rng = np.random.default_rng(3)
    t = near_targets(ax, 500, 3 / 64, rng)
    x0, b = closest_point_ellipsoid(ax, t.y)
    np.testing.assert_allclose(x0, t.x0, atol=1e-12)
    np.testing.assert_allclose(b, t.b, atol=1e-12)
    np.testing.assert_allclose(ellipsoid_normal(ax, t.x0), t.n0, atol=1e-14)


def test_configs_sizes():
    c1 = workload.build_config("c1")
    assert c1["surf"].n == 4302 and c1["targets"].m == 5302
    c1b = workload.build_config("c1")
    np.testing.assert_array_equal(c1["f"], c1b["f"])  # seeded
    np.testing.assert_array_equal(c1["targets"].y, c1b["targets"].y)
    t = c1["targets"]
    assert np.all(t.b[: 4302] == 0) and np.all(np.abs(t.b[4302:]) <= 3 / 16)
