"""Two drops nearly touching in Stokes flow (paper section 4.3, eq. (IE-2Surf)).

Interface velocity u of two spherical drops (viscosity ratio lambda, external viscosity 1) driven by
the jump in surface force [f] = 2 gamma H n - grad_S gamma, gamma = 1 + (x1 - x_c)^2:

    (lambda + 1) u - 2 (lambda - 1) sum_m DL_m[u] = -2 sum_m SL_m[[f]_m]

(the 1/(4 pi) integrals of the paper are twice the 1/(8 pi) layers of the library).  As in the paper,
integrals over a drop's own surface use the modified on-surface smoothing at delta = 3h, those over
the other drop the extrapolated regularization with delta = 3h, 4h, 5h; GMRES from zero to a relative
residual of 1e-10.  Every layer sum runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np

import workload
from .evaluator import RigidSpheres


def _dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


class TwoDrops:
    def __init__(self, h: float, lam: float = 2.0, eps: float = 1.0 / 16 ** 3, precision: int = 0,
                 far_method: int = 0, **kw):
        self.h, self.lam = float(h), float(lam)
        self.centers, self.radii, self.surfs = workload.two_drops(h, eps)
        self.counts = [s.n for s in self.surfs]
        self.x = _dev(np.concatenate([s.x for s in self.surfs]))
        self.R = RigidSpheres(h, rho=(3.0, 4.0, 5.0), precision=precision, far_method=far_method,
                              surface_sharp=True, sharp_rho=3.0, **kw)
        self.R.set_spheres(self.centers, self.radii, self.counts, self.x,
                           _dev(np.concatenate([s.normal for s in self.surfs])),
                           _dev(np.concatenate([s.w for s in self.surfs])))
        self.R.set_operator(self.lam + 1.0, -2.0 * (self.lam - 1.0), False)

    def rhs(self):
        f = np.concatenate([workload.drop_force(s.x, c) for s, c in zip(self.surfs, self.centers)])
        return -2.0 * self.R.single_layer(_dev(f))

    def solve(self, tol: float = 1e-10, maxit: int = 100):
        b = self.rhs()
        return self.R.solve(b, tol=tol, maxit=maxit, restart=maxit)

    def close(self):
        self.R.close()


def self_convergence(u_h, u_h2, h: float, eps: float = 1.0 / 16 ** 3):
    """e_h = u_h - u_{h/2} at the points of spacing h (a subset of those of spacing h/2: the grid lines
    of h are among those of h/2); returns (max |e|, (sum |e|^2 / N)^(1/2)) as in eq. (error_L2)."""
    _, _, sc = workload.two_drops(h, eps)
    _, _, sf = workload.two_drops(h / 2, eps)
    idx, off = [], 0
    for a, b in zip(sc, sf):
        pos = {tuple(p): i for i, p in enumerate(map(tuple, b.x))}
        idx.append(np.array([pos[tuple(p)] for p in map(tuple, a.x)], dtype=np.int64) + off)
        off += b.n
    idx = np.concatenate(idx)
    e = np.asarray(u_h).reshape(-1, 3) - np.asarray(u_h2).reshape(-1, 3)[idx]
    n = np.linalg.norm(e, axis=1)
    return float(n.max()), float(np.sqrt((n ** 2).mean()))
