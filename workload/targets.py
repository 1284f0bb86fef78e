"""Target sets with their closest-point data (x0, n0, b), where y = x0 + b n0 (paper §2, the
expansion about the closest point; b > 0 outside, b = 0 on the surface)."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .surface import Surface, closest_point_ellipsoid, ellipsoid_normal, ellipsoid_project


@dataclass
class Targets:
    """y, x0, n0: (M,3); b: (M,); src: (M,) index of the coinciding quadrature point or -1."""
    y: np.ndarray
    x0: np.ndarray
    n0: np.ndarray
    b: np.ndarray
    src: np.ndarray

    @property
    def m(self) -> int:
        return int(self.y.shape[0])

    def subset(self, idx) -> "Targets":
        idx = np.asarray(idx)
        return Targets(self.y[idx].copy(), self.x0[idx].copy(), self.n0[idx].copy(), self.b[idx].copy(),
                       self.src[idx].copy())


def on_surface_targets(surf: Surface) -> Targets:
    """Every quadrature point as a target on the surface (x0 = y, n0 = its normal, b = 0)."""
    return Targets(surf.x.copy(), surf.x.copy(), surf.normal.copy(), np.zeros(surf.n),
                   np.arange(surf.n, dtype=np.int64))


def near_targets(axes, m: int, bmax: float, rng: np.random.Generator, center=(0.0, 0.0, 0.0)) -> Targets:
    """m targets y = x0 + b n0: x0 is the radial projection of a uniform random direction,
    b ~ U[-bmax, bmax].  Draw order: all directions first, then all b."""
    u = rng.standard_normal((m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    b = rng.uniform(-bmax, bmax, size=m)
    x0 = ellipsoid_project(axes, u, center)
    n0 = ellipsoid_normal(axes, x0, center)
    y = x0 + b[:, None] * n0
    return Targets(y, x0, n0, b, np.full(m, -1, dtype=np.int64))


def grid_targets_outside(axes, h: float, dist: float | None = None, center=(0.0, 0.0, 0.0)) -> Targets:
    """3-D grid points (aligned with the centre) outside the ellipsoid within distance `dist` (default h).

    'Outside' is F(y) >= 1 and the distance test is inclusive with a relative slack of 1e-12, so that
    grid points lying exactly at distance h (the axis vertices shifted by h) are kept despite rounding.
    This is the target set of the paper's Table 1.
    """
    A = np.asarray(axes, float)
    c = np.asarray(center, float)
    dist = h if dist is None else dist
    lims = [int(np.ceil((A[i] + dist) / h)) + 1 for i in range(3)]
    g = [np.arange(-L, L + 1) * h for L in lims]
    X, Y, Z = np.meshgrid(*g, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    F = ((P / A) ** 2).sum(1)
    P = P[F >= 1.0]
    # cheap prefilter: distance >= A_min (sqrt(F) - 1)
    P = P[A.min() * (np.sqrt(((P / A) ** 2).sum(1)) - 1.0) <= dist * 1.5]
    x0, b = closest_point_ellipsoid(A, P + c, c)
    keep = b <= dist * (1.0 + 1e-12)
    y = P[keep] + c
    x0 = x0[keep]
    n0 = ellipsoid_normal(A, x0, c)
    return Targets(y, x0, n0, b[keep], np.full(y.shape[0], -1, dtype=np.int64))


def concat_targets(*ts: Targets) -> Targets:
    return Targets(*(np.concatenate([getattr(t, f) for t in ts]) for f in ("y", "x0", "n0", "b", "src")))
