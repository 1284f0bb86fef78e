"""Oracle of the two-sphere rigid-motion solve (TEST INFRASTRUCTURE ONLY).

Completed double-layer equation for the exterior flow past rigid spheres (Power & Miranda, SIAM J.
Appl. Math. 47 (1987)); the paper's double-layer evaluation supplies every integral:

    (A q)(x) = -1/2 q(x) + sum_m DL_m[q_m](x) + sum_m C_m(x) = U_b + Omega_b x (x - c_b),   x on sphere b,

  DL_m[q_m](x)   the paper's extrapolated double layer of sphere m (eqs. (Stokes_DL2), (extrap_eqn));
                 for m == b the target is on the surface (b = 0, chi = 1/2: the principal value), for
                 m != b it is a nearly singular exterior evaluation (chi = 0) with x0 the closest point of
                 sphere m and q(x0) interpolated;
  C_m(x)         completion: (1/8 pi) [ S(x - c_m) F_m + L_m x (x - c_m) / |x - c_m|^3 ] with
                 F_m = sum_p q_p w_p and L_m = sum_p (x_p - c_m) x q_p w_p over sphere m.

-1/2 q + DL_PV is the exterior limit of the double layer (its jump is q, eq. (Stokes_DL1)); the
completion removes the rigid-motion null space.  q(x0): tensor Lagrange interpolation on the grid of a
quadrature family i on the sheet sign(n_i(x0)): the first of widths 6, 5, 4, 3, 2 points per axis
(6 x 6 points: O(h^6) where the full stencil exists), and for each width the families in decreasing
|n_i(x0)| order, whose stencil points all exist.  The paper does not say how q(x0) is obtained when
x0 is not a quadrature point; this is the reading taken, and the same routine prolongs a density from
the quadrature of spacing h to that of spacing h/2.  GMRES: the textbook algorithm with modified Gram-Schmidt and Givens rotations.
"""
from __future__ import annotations

import numpy as np

from . import dl as _dl
from . import dl_sharp as _dl_sharp
from . import sl as _sl
from . import sl_sharp as _sl_sharp

PI = np.pi
THETA = np.deg2rad(70.0)


class Sphere:
    """One sphere: centre, radius, quadrature (local family/grid keys built from the points)."""

    def __init__(self, surf, center, radius, h):
        self.x = np.asarray(surf.x, float)
        self.n = np.asarray(surf.normal, float)
        self.w = np.asarray(surf.w, float)
        self.c = np.asarray(center, float)
        self.a = float(radius)
        self.h = float(h)
        self.keys = {}
        loc = self.x - self.c
        for p in range(len(self.x)):
            for i in range(3):
                if abs(self.n[p, i]) < np.cos(THETA):
                    continue
                j, k = [d for d in range(3) if d != i]
                aj, ak = loc[p, j] / h, loc[p, k] / h
                if abs(aj - round(aj)) < 1e-9 and abs(ak - round(ak)) < 1e-9:
                    self.keys[(i, 1 if loc[p, i] > 0 else -1, int(round(aj)), int(round(ak)))] = p

    @property
    def size(self):
        return len(self.x)

    def closest(self, y):
        d = np.asarray(y, float) - self.c
        r = np.linalg.norm(d, axis=1)
        n0 = d / r[:, None]
        return self.c + self.a * n0, n0, r - self.a

    def stencils(self, x0):
        """Indices (K,36) and weights (K,36) of the interpolation stencils at surface points x0:
        width 6 (quintic), else 5, 4, 3, 2 points per axis, each tried over the families in decreasing
        |n_i| order; unused slots have weight 0 and index 0."""
        loc = np.asarray(x0, float) - self.c
        h = self.h
        K = len(loc)
        idx = np.zeros((K, 36), dtype=np.int64)
        wts = np.zeros((K, 36))
        for t in range(K):
            order = np.argsort(-np.abs(loc[t]), kind="stable")
            done = False
            for wdt in (6, 5, 4, 3, 2):
                for i in order:
                    j, k = [d for d in range(3) if d != i]
                    sg = 1 if loc[t, i] > 0 else -1
                    j0 = int(np.floor(loc[t, j] / h)) - (wdt - 1) // 2
                    k0 = int(np.floor(loc[t, k] / h)) - (wdt - 1) // 2
                    ids = [self.keys.get((int(i), sg, j0 + a, k0 + b)) for a in range(wdt) for b in range(wdt)]
                    if any(v is None for v in ids):
                        continue
                    lj = _lagrange(loc[t, j] / h - j0, wdt)
                    lk = _lagrange(loc[t, k] / h - k0, wdt)
                    idx[t, :wdt * wdt] = ids
                    wts[t, :wdt * wdt] = np.outer(lj, lk).ravel()
                    done = True
                    break
                if done:
                    break
            if not done:
                raise ValueError("no interpolation stencil")
        return idx, wts


def _lagrange(s, wdt):
    """Lagrange basis at nodes 0 .. wdt-1 evaluated at s."""
    L = np.ones(wdt)
    for a in range(wdt):
        for b in range(wdt):
            if a != b:
                L[a] *= (s - b) / (a - b)
    return L


class RigidProblem:
    """Targets = all quadrature points of all spheres, in sphere order."""

    def __init__(self, spheres, h, rho=(2.0, 3.0, 4.0), full=True, sharp=False, sharp_rho=3.0, a_id=-0.5, a_dl=1.0,
                 completion=True):
        self.S = spheres
        self.h = h
        self.rho = tuple(rho)
        # the operator a_id q + a_dl sum_m DL_m[q] (+ the completion): -1/2, 1, on for the rigid-motion
        # problem; lambda + 1, -2 (lambda - 1), off for the drops of section 4.3 (eq. (IE-2Surf) with the
        # 1/(4 pi) integrals written as twice the 1/(8 pi) layers)
        self.a_id, self.a_dl, self.completion_on = float(a_id), float(a_dl), bool(completion)
        # sharp: a sphere's own points (on its surface) use the modified smoothing at sharp_rho h
        # (paper section 2.1) instead of the extrapolation
        self.sharp, self.sharp_rho = bool(sharp), float(sharp_rho)
        self.y = np.concatenate([s.x for s in spheres])
        self.off = np.cumsum([0] + [s.size for s in spheres])
        self.ntot = int(self.off[-1])
        self.cross = []
        if not full:  # only matvec_rows / velocity will be used
            return
        for m, s in enumerate(spheres):
            x0, n0, b = s.closest(self.y)
            own = np.zeros(self.ntot, bool)
            own[self.off[m]:self.off[m + 1]] = True
            x0[own] = s.x
            n0[own] = s.n
            b[own] = 0.0
            idx, wts = s.stencils(x0[~own])
            self.cross.append(dict(x0=x0, n0=n0, b=b, own=own, idx=idx, wts=wts))

    def split(self, q):
        return [q[self.off[m]:self.off[m + 1]] for m in range(len(self.S))]

    def rhs(self, motion):
        """motion: (nsph, 6) = (U, Omega) per sphere."""
        out = np.zeros((self.ntot, 3))
        for m, s in enumerate(self.S):
            U, Om = motion[m, :3], motion[m, 3:]
            out[self.off[m]:self.off[m + 1]] = U + np.cross(Om, s.x - s.c)
        return out

    def completion_strengths(self, q):
        F, L = [], []
        for s, qm in zip(self.S, self.split(q)):
            F.append((qm * s.w[:, None]).sum(0))
            L.append((np.cross(s.x - s.c, qm) * s.w[:, None]).sum(0))
        return F, L

    def completion(self, q, y):
        F, L = self.completion_strengths(q)
        out = np.zeros((len(y), 3))
        for s, Fm, Lm in zip(self.S, F, L):
            d = y - s.c
            r = np.linalg.norm(d, axis=1)[:, None]
            Sf = Fm / r + d * (d @ Fm)[:, None] / r ** 3
            out += (Sf + np.cross(Lm, d) / r ** 3) / (8 * PI)
        return out

    def _layer(self, s, qm, y, x0, n0, b, q0, own):
        """Double layer of sphere s at targets y; rows `own` are its own points."""
        if not self.sharp or not own.any():
            return _dl(s.x, s.n, s.w, qm, y, x0, n0, b, q0, self.h, self.rho)
        out = np.empty((len(y), 3))
        out[own] = _dl_sharp(s.x, s.n, s.w, qm, y[own], n0[own], q0[own], self.sharp_rho * self.h)
        if (~own).any():
            out[~own] = _dl(s.x, s.n, s.w, qm, y[~own], x0[~own], n0[~own], b[~own], q0[~own], self.h, self.rho)
        return out

    def double_layers(self, q):
        out = np.zeros((self.ntot, 3))
        for s, qm, cr in zip(self.S, self.split(q), self.cross):
            q0 = np.empty((self.ntot, 3))
            q0[cr["own"]] = qm
            q0[~cr["own"]] = np.einsum("ks,ksc->kc", cr["wts"], qm[cr["idx"]])
            out += self._layer(s, qm, self.y, cr["x0"], cr["n0"], cr["b"], q0, cr["own"])
        return out

    def matvec(self, q):
        q = np.asarray(q, float).reshape(self.ntot, 3)
        out = self.a_id * q + self.a_dl * self.double_layers(q)
        return out + self.completion(q, self.y) if self.completion_on else out

    def single_layers(self, f):
        """sum_m SL_m[f_m] at every point: own points on the surface (the modified smoothing if sharp,
        else the extrapolation with b = 0), other points nearly singular with f(x0) interpolated by the
        same stencils as q(x0)."""
        f = np.asarray(f, float).reshape(self.ntot, 3)
        out = np.zeros((self.ntot, 3))
        for s, fm, cr in zip(self.S, self.split(f), self.cross):
            f0 = np.empty((self.ntot, 3))
            f0[cr["own"]] = fm
            f0[~cr["own"]] = np.einsum("ks,ksc->kc", cr["wts"], fm[cr["idx"]])
            own = cr["own"]
            if self.sharp:
                out[own] += _sl_sharp(s.x, s.n, s.w, fm, self.y[own], cr["n0"][own], f0[own], self.sharp_rho * self.h)
            else:
                out[own] += _sl(s.x, s.n, s.w, fm, self.y[own], cr["x0"][own], cr["n0"][own], cr["b"][own], f0[own],
                                self.h, self.rho)
            out[~own] += _sl(s.x, s.n, s.w, fm, self.y[~own], cr["x0"][~own], cr["n0"][~own], cr["b"][~own],
                             f0[~own], self.h, self.rho)
        return out

    def matvec_rows(self, q, rows):
        """(A q) at the target rows only (the same arithmetic as matvec, restricted)."""
        q = np.asarray(q, float).reshape(self.ntot, 3)
        rows = np.asarray(rows)
        y = self.y[rows]
        out = self.a_id * q[rows] + (self.completion(q, y) if self.completion_on else 0.0)
        dls = np.zeros((len(rows), 3))
        for m, (s, qm) in enumerate(zip(self.S, self.split(q))):
            own = (rows >= self.off[m]) & (rows < self.off[m + 1])
            x0, n0, b = s.closest(y)
            x0[own] = s.x[rows[own] - self.off[m]]
            n0[own] = s.n[rows[own] - self.off[m]]
            b[own] = 0.0
            q0 = np.empty((len(rows), 3))
            q0[own] = qm[rows[own] - self.off[m]]
            if (~own).any():
                idx, wts = s.stencils(x0[~own])
                q0[~own] = np.einsum("ks,ksc->kc", wts, qm[idx])
            dls += self._layer(s, qm, y, x0, n0, b, q0, own)
        return out + self.a_dl * dls

    def velocity(self, q, y):
        """Exterior flow at points y outside every sphere: sum_m DL_m (chi = 0) + completion."""
        y = np.asarray(y, float)
        out = self.completion(q, y)
        for s, qm in zip(self.S, self.split(q)):
            x0, n0, b = s.closest(y)
            idx, wts = s.stencils(x0)
            q0 = np.einsum("ks,ksc->kc", wts, qm[idx])
            out += _dl(s.x, s.n, s.w, qm, y, x0, n0, b, q0, self.h, self.rho)
        return out


def gmres(matvec, b, x0=None, tol=1e-10, maxit=200):
    """Textbook GMRES (no restart) with modified Gram-Schmidt and Givens rotations.
    Returns (x, iterations, relative residual estimate)."""
    b = np.asarray(b, float).ravel()
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, float).ravel().copy()
    r = b - matvec(x).ravel()
    bn = np.linalg.norm(b)
    beta = np.linalg.norm(r)
    if beta / bn <= tol:
        return x, 0, beta / bn
    V = [r / beta]
    H = np.zeros((maxit + 1, maxit))
    cs, sn = np.zeros(maxit), np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    k = 0
    for k in range(maxit):
        w = matvec(V[k]).ravel()
        for i in range(k + 1):
            H[i, k] = V[i] @ w
            w = w - H[i, k] * V[i]
        H[k + 1, k] = np.linalg.norm(w)
        V.append(w / H[k + 1, k])
        for i in range(k):
            t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
            H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
            H[i, k] = t
        d = np.hypot(H[k, k], H[k + 1, k])
        cs[k], sn[k] = H[k, k] / d, H[k + 1, k] / d
        H[k, k] = d
        H[k + 1, k] = 0.0
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k] * g[k]
        if abs(g[k + 1]) / bn <= tol:
            break
    y = np.linalg.solve(np.triu(H[:k + 1, :k + 1]), g[:k + 1])
    for i in range(k + 1):
        x = x + y[i] * V[i]
    return x, k + 1, abs(g[k + 1]) / bn
