"""Grid-line-intersection surface quadrature on an ellipsoid (paper §2.2, eq. (quadrature)).

The surface F(x) = sum_i ((x_i - c_i)/A_i)^2 = 1 is covered by a 3-D grid of spacing h aligned with the
centre c.  Family i (i = 1, 2, 3) holds the points whose two other coordinates lie on the grid and whose
unit normal satisfies |n_i| >= cos(theta), theta = 70 degrees.  A point of family i gets the weight
w = psi_i(n) h^2 / |n_i|, where psi is the partition of unity on the unit sphere built from the bump
b(r) = exp(2 r^2 / (r^2 - 1)) (|r| < 1, else 0) through beta_i(n) = b(arccos|n_i| / theta),
psi_i = beta_i / sum_j beta_j.  (The printed formula for beta_i has an unbalanced parenthesis; the
reading b(arccos|n_i| / theta) reproduces the point counts of the paper's Table 1 exactly.)

These arrays are inputs of the evaluator: the caller hands over points, normals and weights.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

THETA_DEG = 70.0


@dataclass
class Surface:
    """Quadrature of a closed surface: x (N,3), normal (N,3) outward unit, w (N,), family (N,) in {0,1,2}."""
    x: np.ndarray
    normal: np.ndarray
    w: np.ndarray
    family: np.ndarray
    axes: tuple
    center: tuple
    h: float

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def _bump(r: np.ndarray) -> np.ndarray:
    out = np.zeros_like(r)
    m = np.abs(r) < 1.0
    rr = r[m] ** 2
    out[m] = np.exp(2.0 * rr / (rr - 1.0))
    return out


def partition_of_unity(nrm: np.ndarray, theta_deg: float = THETA_DEG) -> np.ndarray:
    """psi_i(n) for i = 1..3 at unit normals nrm (K,3) -> (K,3)."""
    th = np.deg2rad(theta_deg)
    beta = _bump(np.arccos(np.clip(np.abs(nrm), 0.0, 1.0)) / th)
    return beta / beta.sum(axis=1, keepdims=True)


def ellipsoid_normal(axes, x: np.ndarray, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Outward unit normal grad F / |grad F| at points x (K,3) of the ellipsoid."""
    A = np.asarray(axes, float)
    g = (np.asarray(x, float) - np.asarray(center, float)) / A ** 2
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def ellipsoid_project(axes, u: np.ndarray, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Radial projection of directions u (K,3) from the centre onto the ellipsoid."""
    A = np.asarray(axes, float)
    u = np.asarray(u, float)
    s = np.sqrt(((u / A) ** 2).sum(axis=1, keepdims=True))
    return np.asarray(center, float) + u / s


def ellipsoid_quadrature(axes, h: float, center=(0.0, 0.0, 0.0), theta_deg: float = THETA_DEG) -> Surface:
    """All three families of grid-line intersections with their partition-of-unity weights.

    Order: family 1, 2, 3; within a family, grid lines in lexicographic order of the two grid
    coordinates, then the + and - intersections.
    """
    A = np.asarray(axes, float)
    c = np.asarray(center, float)
    cth = np.cos(np.deg2rad(theta_deg))
    xs, ns, ws, fs = [], [], [], []
    for i in range(3):
        j, k = [a for a in range(3) if a != i]
        kj = int(np.floor(A[j] / h))
        kk = int(np.floor(A[k] / h))
        P, Q = np.meshgrid(np.arange(-kj, kj + 1), np.arange(-kk, kk + 1), indexing="ij")
        xj = P.ravel() * h
        xk = Q.ravel() * h
        s = 1.0 - (xj / A[j]) ** 2 - (xk / A[k]) ** 2
        m = s > 0.0
        xj, xk, s = xj[m], xk[m], s[m]
        root = A[i] * np.sqrt(s)
        for sg in (1.0, -1.0):
            x = np.empty((s.size, 3))
            x[:, i] = sg * root
            x[:, j] = xj
            x[:, k] = xk
            x += c
            nrm = ellipsoid_normal(A, x, c)
            keep = np.abs(nrm[:, i]) >= cth
            x, nrm = x[keep], nrm[keep]
            psi = partition_of_unity(nrm, theta_deg)
            w = psi[:, i] / np.abs(nrm[:, i]) * h * h
            xs.append(x)
            ns.append(nrm)
            ws.append(w)
            fs.append(np.full(x.shape[0], i, dtype=np.int32))
    return Surface(np.ascontiguousarray(np.concatenate(xs)), np.ascontiguousarray(np.concatenate(ns)),
                   np.concatenate(ws), np.concatenate(fs), tuple(float(a) for a in A),
                   tuple(float(v) for v in c), float(h))


def sphere_quadrature(h: float, radius: float = 1.0, center=(0.0, 0.0, 0.0)) -> Surface:
    return ellipsoid_quadrature((radius, radius, radius), h, center)


def closest_point_ellipsoid(axes, y: np.ndarray, center=(0.0, 0.0, 0.0), iters: int = 200):
    """Closest point x0 on the ellipsoid to each y (K,3) and the signed distance b (positive outside).

    x0_i = A_i^2 y_i / (A_i^2 + t) with t the root of sum_i (A_i y_i / (A_i^2 + t))^2 = 1 that lies
    above -min_i A_i^2 (Newton from the outer side, then bisection polish).  Valid for targets closer
    to the surface than its smallest radius of curvature, which is all that the target sets here use.
    """
    A = np.asarray(axes, float)
    A2 = A ** 2
    c = np.asarray(center, float)
    yy = np.asarray(y, float) - c
    K = yy.shape[0]
    lo = np.full(K, -A2.min() * (1.0 - 1e-15))
    hi = np.maximum(np.linalg.norm(yy, axis=1) * A.max(), 1.0)

    def F(t):
        return ((A * yy / (A2 + t[:, None])) ** 2).sum(1) - 1.0

    # bracket and bisect (robust), then Newton polish
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        f = F(mid)
        pos = f > 0
        lo = np.where(pos, mid, lo)
        hi = np.where(pos, hi, mid)
        if np.all(hi - lo <= 1e-16 * np.maximum(1.0, np.abs(hi))):
            break
    t = 0.5 * (lo + hi)
    for _ in range(3):
        den = A2 + t[:, None]
        f = ((A * yy / den) ** 2).sum(1) - 1.0
        df = (-2.0 * A2 * yy ** 2 / den ** 3).sum(1)
        ok = df != 0
        t = np.where(ok, t - np.where(ok, f / np.where(ok, df, 1.0), 0.0), t)
    x0 = A2 * yy / (A2 + t[:, None]) + c
    d = np.linalg.norm(np.asarray(y, float) - x0, axis=1)
    inside = ((yy / A) ** 2).sum(1) < 1.0
    return x0, np.where(inside, -d, d)


def ellipsoid_area(axes) -> float:
    """Surface area of an ellipsoid by adaptive quadrature over the parameter domain (reference value)."""
    from scipy import integrate

    a, b, c = (float(v) for v in axes)

    def integrand(phi, th):
        st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(phi), np.cos(phi)
        # |x_th x x_phi| for x = (a st cp, b st sp, c ct)
        return st * np.sqrt((b * c * st * cp) ** 2 + (a * c * st * sp) ** 2 + (a * b * ct) ** 2)

    val, _ = integrate.dblquad(integrand, 0.0, np.pi, 0.0, 2.0 * np.pi, epsabs=1e-13, epsrel=1e-13)
    return float(val)
