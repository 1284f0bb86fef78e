"""Named synthetic workloads.

Seeds are numpy.random.default_rng(250700156 + k) for workload k; draw order: density coefficients,
then the near-target base directions, then the signed distances b.

  c1      unit sphere, h = 1/16 (N = 4302); densities: degree <= 3 harmonics; targets: all quadrature
          points + 1000 near points with b ~ U[-3h, 3h]; rho = (2, 3, 4).
  c2      ellipsoid (1, 0.8, 0.6), h = 1/64 (N = 42342); degree <= 4; targets: all quadrature points
          + 20000 near points within +-3h (M = 62342).
  c3      ellipsoid (1, 0.8, 0.6), h = 1/128 (N = 169342); as c2 (M = 189342).
  table1  spheroid x1^2 + 4 x2^2 + 4 x3^2 = 1 at h (Table 1 of the paper): targets are the grid points
          within h outside; density f1 = 1/sqrt(1 - 3 x1^2 / 4), f2 = f3 = 0; rho = (3, 4, 5).
  small   ellipsoid (1, 0.8, 0.6), h = 1/24 (N ~ 6e3), degree <= 4, 800 near targets: a parity case
          that spans many tiles and a ragged tail at a size the oracle finishes in seconds.

The double-layer density q is the same field as f (q = f).
"""
from __future__ import annotations

import numpy as np

from .surface import ellipsoid_quadrature
from .targets import concat_targets, grid_targets_outside, near_targets, on_surface_targets
from .density import harmonic_coeffs, harmonic_field

SEED_BASE = 250700156

CONFIGS = {
    "c1": dict(k=1, axes=(1.0, 1.0, 1.0), h=1 / 16, L=3, m_near=1000, bmax_h=3.0, rho=(2.0, 3.0, 4.0)),
    "c2": dict(k=2, axes=(1.0, 0.8, 0.6), h=1 / 64, L=4, m_near=20000, bmax_h=3.0, rho=(2.0, 3.0, 4.0)),
    "c3": dict(k=3, axes=(1.0, 0.8, 0.6), h=1 / 128, L=4, m_near=20000, bmax_h=3.0, rho=(2.0, 3.0, 4.0)),
    "small": dict(k=11, axes=(1.0, 0.8, 0.6), h=1 / 24, L=4, m_near=800, bmax_h=3.0, rho=(2.0, 3.0, 4.0)),
    "tiny": dict(k=12, axes=(1.0, 0.8, 0.6), h=1 / 10, L=2, m_near=100, bmax_h=3.0, rho=(2.0, 3.0, 4.0)),
}


def build_config(name: str, h: float | None = None, m_near: int | None = None, seed_offset: int = 0) -> dict:
    """Return a dict: surf, targets, f, f0, q, q0, h, rho (and the generator parameters)."""
    if name.startswith("table1"):
        hh = h if h is not None else 1 / 32
        axes = (1.0, 0.5, 0.5)
        surf = ellipsoid_quadrature(axes, hh)
        t = grid_targets_outside(axes, hh)

        def fld(x):
            out = np.zeros_like(x)
            out[:, 0] = 1.0 / np.sqrt(1.0 - 0.75 * np.clip(x[:, 0], -1, 1) ** 2)
            return out

        f = fld(surf.x)
        f0 = fld(t.x0)
        return dict(name=name, surf=surf, targets=t, f=f, f0=f0, q=f.copy(), q0=f0.copy(), h=hh,
                    rho=(3.0, 4.0, 5.0), axes=axes)
    cfg = dict(CONFIGS[name])
    if h is not None:
        cfg["h"] = h
    if m_near is not None:
        cfg["m_near"] = m_near
    rng = np.random.default_rng(SEED_BASE + cfg["k"] + seed_offset)
    coeffs = harmonic_coeffs(cfg["L"], rng)
    surf = ellipsoid_quadrature(cfg["axes"], cfg["h"])
    t_on = on_surface_targets(surf)
    t_near = near_targets(cfg["axes"], cfg["m_near"], cfg["bmax_h"] * cfg["h"], rng)
    t = concat_targets(t_on, t_near)
    f = harmonic_field(coeffs, surf.x)
    f0 = harmonic_field(coeffs, t.x0)
    f0[: surf.n] = f  # on-surface targets: density at x0 is exactly the source value
    return dict(name=name, surf=surf, targets=t, f=f, f0=f0, q=f.copy(), q0=f0.copy(), h=cfg["h"],
                rho=tuple(cfg["rho"]), axes=cfg["axes"], coeffs=coeffs)


def two_spheres(h: float, gap: float, radius: float = 1.0):
    """Two spheres of the given radius, centres (0,0,0) and (2 radius + gap, 0, 0); each sphere's
    grid-line quadrature is generated in its own frame (identical point sets).  Returns
    (centers (2,3), radii (2,), surfaces [s1, s2])."""
    c1 = (0.0, 0.0, 0.0)
    c2 = (2.0 * radius + gap, 0.0, 0.0)
    s1 = ellipsoid_quadrature((radius, radius, radius), h, c1)
    s2 = ellipsoid_quadrature((radius, radius, radius), h, c2)
    return np.array([c1, c2]), np.array([radius, radius]), [s1, s2]


def rigid_motion(rng: np.random.Generator, nsph: int = 2) -> np.ndarray:
    """(nsph, 6) translation and rotation per sphere, N(0, 1)."""
    return rng.standard_normal((nsph, 6))


def two_drops(h: float, eps: float = 1.0 / 16 ** 3):
    """Two unit spheres centred at (0,0,0) and (2, 0, eps) (paper section 4.3; gap sqrt(4 + eps^2) - 2),
    each with the grid-line quadrature in its own frame.  Returns (centers (2,3), radii, [s1, s2])."""
    c1 = (0.0, 0.0, 0.0)
    c2 = (2.0, 0.0, float(eps))
    s1 = ellipsoid_quadrature((1.0, 1.0, 1.0), h, c1)
    s2 = ellipsoid_quadrature((1.0, 1.0, 1.0), h, c2)
    return np.array([c1, c2]), np.array([1.0, 1.0]), [s1, s2]


def drop_force(x: np.ndarray, center) -> np.ndarray:
    """Jump in surface force on a unit sphere with surface tension gamma = 1 + (x1 - c1)^2 (section 4.3):
    [f] = 2 gamma H n - grad_S gamma with mean curvature H = 1 and n the outward normal;
    grad_S gamma = (I - n n^T) grad gamma, grad gamma = (2 (x1 - c1), 0, 0)."""
    x = np.asarray(x, float)
    c = np.asarray(center, float)
    d = x - c
    n = d / np.linalg.norm(d, axis=1)[:, None]
    gam = 1.0 + d[:, 0] ** 2
    grad = np.zeros_like(x)
    grad[:, 0] = 2.0 * d[:, 0]
    grad_s = grad - n * (n * grad).sum(1)[:, None]
    return 2.0 * gam[:, None] * n - grad_s
