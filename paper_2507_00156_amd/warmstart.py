"""Learned warm start for the two-sphere rigid-motion solve.

Pipeline (every step on the GPU through the library; torch only holds device memory):
  1. data: for each (gap, motion) sample, the mixed-precision GMRES solve of the completed
     double-layer equation on the fine quadrature (spacing h_f), kept at the coarse points
     (spacing h_c = 2 h_f, a subset of the fine points): 3 N_c values.  Solving on the coarse
     quadrature instead leaves the coarse/fine discretization difference in every prediction;
  2. training: the warm-start network (gap, 12 motion parameters) -> coarse density, Adam on
     random mini-batches drawn from the resident data set, cosine learning-rate decay;
  3. use: predict the coarse density, interpolate it to the fine quadrature (spacing h_f), and
     start the refined GMRES solve there; the solve replaces a guess no better than zero by zero.
"""
from __future__ import annotations

import math
import time

import numpy as np

import workload
from .evaluator import Prolongation, RigidSpheres, WarmStartNet


def _dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


class TwoSpheres:
    """Two unit spheres at a gap: quadrature on the device and the library's rigid-motion operator."""

    def __init__(self, h: float, gap: float, precision: int = 1, far_method: int = 0, **kw):
        self.h, self.gap = float(h), float(gap)
        self.centers, self.radii, surfs = workload.two_spheres(h, gap)
        self.counts = [s.n for s in surfs]
        self.x = _dev(np.concatenate([s.x for s in surfs]))
        self.nrm = _dev(np.concatenate([s.normal for s in surfs]))
        self.w = _dev(np.concatenate([s.w for s in surfs]))
        self.ntot = int(sum(self.counts))
        self.R = RigidSpheres(h, precision=precision, far_method=far_method, **kw)
        self.R.set_spheres(self.centers, self.radii, self.counts, self.x, self.nrm, self.w)

    def close(self):
        self.R.close()


def restriction(h_c: float, h_f: float, gap: float):
    """Indices of the coarse quadrature points within the fine quadrature, sphere by sphere.  The grid
    lines of spacing h_c are among those of spacing h_f = h_c / k, so every coarse point is a fine
    point with bit-identical coordinates; matching is exact."""
    _, _, sc = workload.two_spheres(h_c, gap)
    _, _, sf = workload.two_spheres(h_f, gap)
    out, off = [], 0
    for a, b in zip(sc, sf):
        pos = {tuple(p): i for i, p in enumerate(map(tuple, b.x))}
        try:
            out.append(np.array([pos[tuple(p)] for p in map(tuple, a.x)], dtype=np.int64) + off)
        except KeyError:
            raise ValueError("coarse points are not a subset of the fine points") from None
        off += b.n
    return np.concatenate(out)


def generate(h: float, gaps, motions, tol: float = 1e-6, restart: int = 100, maxit: int = 600, log=None,
             keep=None):
    """Solutions for the samples (gaps (n,), motions (n,2,6)) on the quadrature of spacing h;
    consecutive samples with the same gap share one operator.  keep(gap) -> point indices (or None:
    all points) selects the points stored.  Returns (Y (n, 3 K) FP64 device tensor, iterations)."""
    import torch

    gaps = np.asarray(gaps, float)
    n = len(gaps)
    Y = None
    its = np.zeros(n, dtype=np.int64)
    sys_ = None
    t0 = time.time()
    for i in range(n):
        if sys_ is None or gaps[i] != sys_.gap:
            if sys_ is not None:
                sys_.close()
            sys_ = TwoSpheres(h, gaps[i], precision=1)
            sel = None if keep is None else torch.from_numpy(keep(gaps[i])).cuda()
            if Y is None:
                Y = torch.empty((n, 3 * (sys_.ntot if sel is None else len(sel))), dtype=torch.float64, device="cuda")
        b = sys_.R.rhs(np.asarray(motions[i], float).reshape(2, 6))
        q, it, rr = sys_.R.solve(b, tol=tol, maxit=maxit, restart=restart)
        Y[i] = (q if sel is None else q[sel]).reshape(-1)
        its[i] = it
        if log and ((i + 1) % max(1, n // 20) == 0 or i + 1 == n):
            log(f"data {i + 1}/{n}: gap {gaps[i]:.4f} iterations {it} ({time.time() - t0:.1f} s)")
    if sys_ is not None:
        sys_.close()
    return Y, its


def train(net: WarmStartNet, gaps, motions, Y, steps: int, batch: int = 64, lr: float = 1e-3,
          lr_min: float = 1e-5, seed: int = 0, log=None, log_every: int = 500):
    """Adam on random mini-batches (indices drawn on the host from `seed`), cosine decay from lr to
    lr_min.  The output scale is fitted to Y first.  Returns the loss history (every log_every)."""
    import torch

    g = _dev(gaps)
    m = _dev(np.asarray(motions, float).reshape(len(gaps), 12))
    net.fit_output_scale(Y)
    rng = np.random.default_rng(seed)
    n = len(gaps)
    hist = []
    t0 = time.time()
    for it in range(steps):
        idx = torch.from_numpy(rng.integers(0, n, batch)).cuda()
        a = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * it / max(1, steps - 1)))
        want = (it % log_every == 0) or it == steps - 1
        loss = net.train_step(g, m, Y, a, idx=idx, batch=batch, want_loss=want)
        if want:
            hist.append((it, loss))
            if log:
                log(f"train step {it}/{steps}: loss {loss:.3e} lr {a:.2e} ({time.time() - t0:.1f} s)")
    return hist


class WarmStarter:
    """Predicts the fine-grid initial density for a (gap, motion): network on the coarse grid, then
    interpolation to the fine grid."""

    def __init__(self, net: WarmStartNet, h_c: float):
        self.net, self.h_c = net, float(h_c)
        self._coarse = {}

    def guess(self, fine: TwoSpheres, motion):
        import torch

        key = fine.gap
        if key not in self._coarse:
            cen, rad, sc = workload.two_spheres(self.h_c, fine.gap)
            xc = _dev(np.concatenate([s.x for s in sc]))
            nc = _dev(np.concatenate([s.normal for s in sc]))
            self._coarse = {key: Prolongation(cen, rad, self.h_c, [s.n for s in sc], xc, nc, fine.counts, fine.x)}
        pr = self._coarse[key]
        g = torch.tensor([fine.gap], dtype=torch.float64, device="cuda")
        m = _dev(np.asarray(motion, float).reshape(1, 12))
        qc = self.net.predict(g, m).reshape(-1, 3)
        return pr(qc)
