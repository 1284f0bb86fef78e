"""Learned warm start for the two-sphere rigid-motion solve.

Pipeline (every step on the GPU through the library; torch only holds device memory):
  0. physics part: the density of one sphere alone in the fluid for each of its 6 unit rigid
     motions (IsolatedSphere); for a pair of spheres with motion m it gives q_iso(m), the density
     without the interaction of the two spheres;
  1. data: for each (gap, motion) sample, the mixed-precision GMRES solve of the completed
     double-layer equation on the fine quadrature (spacing h_f), kept at the coarse points
     (spacing h_c = 2 h_f, a subset of the fine points): 3 N_c values.  Solving on the coarse
     quadrature instead leaves the coarse/fine discretization difference in every prediction.
     Samples are solved in increasing gap order and each starts from the solutions of the same
     motion at the previous gaps, extrapolated in log(gap);
  2. training: the warm-start network (gap, 12 motion parameters) -> the interaction part of the
     coarse density, q - q_iso(m) at the coarse points; Adam on random mini-batches drawn from the
     resident data set, cosine learning-rate decay;
  3. use: q_iso(m) on the fine quadrature plus the predicted interaction part interpolated from the
     coarse to the fine quadrature; the refined GMRES solve starts there and replaces a guess no
     better than zero by zero.
Controls at the same data: q_iso(m) alone (no learning), and the stored interaction parts at the
training gaps interpolated in log(gap) (BasisInterpolator, no learning).
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


_RESTRICTION = {}


def restriction(h_c: float, h_f: float, gap: float):
    """Indices of the coarse quadrature points within the fine quadrature, sphere by sphere.  The grid
    lines of spacing h_c are among those of spacing h_f = h_c / k, so every coarse point is a fine
    point with bit-identical coordinates; matching is exact.  Each sphere's points are the same set in
    its own frame at every gap, so the indices do not depend on the gap (computed once per (h_c, h_f))."""
    key = (float(h_c), float(h_f))
    if key not in _RESTRICTION:
        _RESTRICTION[key] = _restriction(h_c, h_f, gap)
    return _RESTRICTION[key]


def _restriction(h_c: float, h_f: float, gap: float):
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
             keep=None, chain: bool = True, order_x: int = 3):
    """Solutions for the samples (gaps (n,), motions (n,2,6)) on the quadrature of spacing h;
    consecutive samples with the same gap share one operator.  keep(gap) -> point indices (or None:
    all points) selects the points stored.  chain: when the motions are the 12 unit motions at each
    gap (the rows of warmstart_unit_dataset), solve the gaps in increasing order and start each solve
    from the same motion's solution at the previous gap, extrapolated in log(gap) by the Lagrange polynomial through
    the order_x previous gaps (the rows of Y stay in the caller's order).  Returns (Y (n, 3 K) FP64 device tensor,
    iterations)."""
    import torch

    gaps = np.asarray(gaps, float)
    motions = np.asarray(motions, float).reshape(len(gaps), 12)
    n = len(gaps)
    unit = (n % 12 == 0 and np.array_equal(motions, np.tile(np.eye(12), (n // 12, 1)))
            and np.all(gaps.reshape(-1, 12) == gaps.reshape(-1, 12)[:, :1]))
    chain = chain and unit
    order = np.arange(n)
    if chain:
        g_order = np.argsort(gaps[::12], kind="stable")
        order = (g_order[:, None] * 12 + np.arange(12)[None, :]).ravel()
    Y = None
    its = np.zeros(n, dtype=np.int64)
    sys_ = None
    hist = {}  # motion -> [(log gap, fine solution), ...] of the last order_x gaps
    t0 = time.time()
    t_solve = 0.0
    for c, i in enumerate(order):
        if sys_ is None or gaps[i] != sys_.gap:
            if sys_ is not None:
                sys_.close()
            sys_ = TwoSpheres(h, gaps[i], precision=1)
            sel = None if keep is None else torch.from_numpy(keep(gaps[i])).cuda()
            if Y is None:
                Y = torch.empty((n, 3 * (sys_.ntot if sel is None else len(sel))), dtype=torch.float64, device="cuda")
        b = sys_.R.rhs(motions[i].reshape(2, 6))
        x0 = None
        if chain:
            l = int(np.argmax(motions[i]))
            prev = hist.get(l, [])
            lg = math.log(gaps[i])
            # Lagrange extrapolation in log(gap) through the previous gaps (up to three)
            xs = [v[0] for v in prev]
            if prev and len(set(xs)) == len(xs):
                x0 = 0
                for j, (xj, qj) in enumerate(prev):
                    L = 1.0
                    for k2, xk in enumerate(xs):
                        if k2 != j:
                            L *= (lg - xk) / (xj - xk)
                    x0 = x0 + L * qj
            elif prev:
                x0 = prev[-1][1]
        t1 = time.time()
        q, it, rr = sys_.R.solve(b, x0=x0, tol=tol, maxit=maxit, restart=restart)
        t_solve += time.time() - t1
        if chain:
            hist[l] = (hist.get(l, []) + [(lg, q)])[-order_x:]
        Y[i] = (q if sel is None else q[sel]).reshape(-1)
        its[i] = it
        if log and ((c + 1) % max(1, n // 20) == 0 or c + 1 == n):
            log(f"data {c + 1}/{n}: gap {gaps[i]:.4f} iterations {it} ({time.time() - t0:.1f} s, {t_solve:.1f} s in "
                f"the solves)")
    if sys_ is not None:
        sys_.close()
    return Y, its


class IsolatedSphere:
    """The density of one unit sphere alone in the fluid for its 6 unit rigid motions (U = e_1, e_2,
    e_3, then Omega = e_1, e_2, e_3), on the grid-line quadrature of spacing h in the sphere's own frame:
    the same completed double-layer equation as the pair, with one sphere.  Every sphere of a pair
    carries the same point set in its own frame, so for the pair with motion m (2, 6) the density
    without interaction is q_iso(m) = [sum_l m[0, l] B_l ; sum_l m[1, l] B_l]."""

    def __init__(self, h: float, tol: float = 1e-10):
        import torch

        self.h = float(h)
        surf = workload.sphere_quadrature(h)
        R = RigidSpheres(h, precision=1)
        R.set_spheres(np.zeros((1, 3)), np.ones(1), [surf.n], _dev(surf.x), _dev(surf.normal), _dev(surf.w))
        self.n = surf.n
        B = torch.empty((6, surf.n, 3), dtype=torch.float64, device="cuda")
        self.iterations = []
        for l in range(6):
            mo = np.zeros((1, 6))
            mo[0, l] = 1.0
            b = R.rhs(mo)
            q, it, _, rr = R.solve_refined(b, tol=tol, restart=100)
            B[l] = q
            self.iterations.append(int(it))
        R.close()
        self.B = B

    def density(self, motion):
        """q_iso for a pair of spheres: (2 n, 3) for motion (2, 6)."""
        import torch

        m = torch.as_tensor(np.asarray(motion, float).reshape(2, 6), device="cuda")
        return torch.einsum("sl,lpc->spc", m, self.B).reshape(2 * self.n, 3)

    def densities(self, motions):
        """q_iso for a batch of motions (k, 2, 6): (k, 2 n, 3)."""
        import torch

        m = torch.as_tensor(np.asarray(motions, float).reshape(-1, 2, 6), device="cuda")
        return torch.einsum("ksl,lpc->kspc", m, self.B).reshape(m.shape[0], 2 * self.n, 3)


def train(net: WarmStartNet, gaps, motions, Y, steps: int, batch: int = 64, lr: float = 1e-3,
          lr_min: float = 1e-5, seed: int = 0, log=None, log_every: int = 500, scale=None):
    """Adam on random mini-batches (indices drawn on the host from `seed`), cosine decay from lr to
    lr_min.  The output scale is fitted to Y first (per output), or set to `scale` (a device vector,
    one value per output) when given.  Returns the loss history (every log_every)."""
    import torch

    g = _dev(gaps)
    m = _dev(np.asarray(motions, float).reshape(len(gaps), 12))
    if scale is None:
        net.fit_output_scale(Y)
    else:
        net.set_output_scale(scale)
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


def coarse_isolated(iso: IsolatedSphere, h_c: float, motions):
    """q_iso(m) at the coarse points of the pair, for motions (k, 2, 6): (k, 3 N_c), the layout of the
    data rows (sphere by sphere, point by point, component fastest)."""
    import torch

    sel = torch.from_numpy(restriction(h_c, iso.h, 0.1)).cuda()
    n1 = iso.n
    sel1 = sel[sel < n1]  # the first sphere's coarse points; the second sphere's are the same + n1
    if len(sel1) * 2 != len(sel) or not torch.equal(sel[len(sel1):], sel1 + n1):
        raise ValueError("the two spheres' coarse points are not the same point set")
    Bc = iso.B[:, sel1, :]  # (6, N_c1, 3)
    m = torch.as_tensor(np.asarray(motions, float).reshape(-1, 2, 6), device="cuda")
    return torch.einsum("ksl,lpc->kspc", m, Bc).reshape(m.shape[0], -1)


class BasisInterpolator:
    """A warm start without learning, from the same data: at each training gap the 12 unit-motion
    rows are the columns of the linear map from motion to (interaction part of the) coarse density;
    for a new gap each column is interpolated in log(gap) by a least-squares polynomial of degree `deg`
    through the `k` nearest training gaps, and applied to the motion."""

    def __init__(self, gaps, Y, k: int = 8, deg: int = 4):
        g = np.asarray(gaps, float).reshape(-1, 12)
        self.lg = np.log(g[:, 0])
        self.Q = Y.reshape(len(self.lg), 12, -1)
        self.k, self.deg = min(k, len(self.lg)), min(deg, min(k, len(self.lg)) - 1)

    def __call__(self, gap: float, motion):
        import torch

        lg = math.log(gap)
        near = np.argsort(np.abs(self.lg - lg), kind="stable")[:self.k]
        x = self.lg[near] - lg
        sc = max(np.abs(x).max(), 1e-12)
        V = np.vander(x / sc, self.deg + 1, increasing=True)
        w = np.linalg.pinv(V)[0]  # the fitted polynomial's value at x = 0
        dev = self.Q.device
        wt = torch.as_tensor(w, device=dev)
        Qg = torch.einsum("k,klp->lp", wt, self.Q[torch.from_numpy(near).to(dev)])
        m = torch.as_tensor(np.asarray(motion, float).reshape(12), device=dev)
        return m @ Qg


class WarmStarter:
    """Fine-grid initial density for a (gap, motion): q_iso(m) on the fine quadrature (when an
    IsolatedSphere is given) plus a coarse-grid prediction interpolated to the fine quadrature
    (predict(gap, motion) -> (3 N_c,) device tensor, or None for the isolated part alone)."""

    def __init__(self, predict, h_c: float, iso: IsolatedSphere | None = None):
        self.predict, self.h_c, self.iso = predict, float(h_c), iso
        self._prolong = None

    def guess(self, fine: TwoSpheres, motion):
        x = None
        if self.predict is not None:
            # the interpolation stencils of a sphere depend on its points in its own frame only, which
            # are the same at every gap: built once (on the host) and reused for every gap
            if self._prolong is None:
                cen, rad, sc = workload.two_spheres(self.h_c, fine.gap)
                xc = _dev(np.concatenate([s.x for s in sc]))
                nc = _dev(np.concatenate([s.normal for s in sc]))
                self._prolong = Prolongation(cen, rad, self.h_c, [s.n for s in sc], xc, nc, fine.counts, fine.x)
            x = self._prolong(self.predict(fine.gap, motion).reshape(-1, 3).contiguous())
        if self.iso is not None:
            qi = self.iso.density(motion)
            x = qi if x is None else x + qi
        return x


def _blocks(width: int, nout: int):
    """(name, shape) of the network's parameter blocks in the library's order."""
    W = width
    return [("W1", (W, 1)), ("b1", (W,)), ("W2", (W, W)), ("b2", (W,)), ("W3", (W, W)), ("b3", (W,)),
            ("W4", (12 * W, W)), ("b4", (12 * W,)), ("Wh", (nout, W))]


def fit_readout(net: WarmStartNet, gaps, T, scale, lambdas=None, log=None):
    """Least-squares fit of the network's two linear output layers for its trained hidden layers
    (variable projection).  The output is linear in [h3; 1] for each motion k: o = M_k [h3; 1] with
    M_k = Wh [W4_k | b4_k] (W4_k, b4_k: the rows 12 w + k).  With the unit-motion data (rows i*12 + k:
    gap g_i, motion e_k) each M_k is a ridge regression of the standardized targets T / scale on the
    features [h3(g_i); 1]; the ridge parameter is chosen by leave-one-gap-out error (closed form from
    the hat matrix).  Written back with Wh = [I_nout | 0] (needs nout <= width): W4 rows 12 w + k = row w
    of M_k.  Returns (chosen lambda, its leave-one-out RMS, the training RMS), in standardized units."""
    import torch

    W, P = net.width, net.nout
    if P > W:
        raise ValueError("fit_readout: needs nout <= width")
    flat = net.get_params().astype(np.float64)
    p, off = {}, 0
    for name, shp in _blocks(W, P):
        k = int(np.prod(shp))
        p[name] = flat[off:off + k].reshape(shp)
        off += k
    g = np.asarray(gaps, float).reshape(-1, 12)[:, 0]
    gt = ((np.log(g) - net.g_mid) / net.g_half)[:, None]
    h = np.tanh(gt @ p["W1"].T + p["b1"])
    h = np.tanh(h @ p["W2"].T + p["b2"])
    h = np.tanh(h @ p["W3"].T + p["b3"])
    F = np.concatenate([h, np.ones((len(g), 1))], axis=1)  # (n_g, W + 1)
    s = scale.cpu().numpy() if hasattr(scale, "cpu") else np.asarray(scale, float)
    Tn = (T.cpu().numpy() if hasattr(T, "cpu") else np.asarray(T)).reshape(len(g), 12, P) / s  # (n_g, 12, P)
    U, sv, Vt = np.linalg.svd(F, full_matrices=False)
    UT = np.einsum("ia,ikp->akp", U, Tn)  # U^T T per motion and output
    if lambdas is None:
        lambdas = [sv[0] ** 2 * 10.0 ** (-e) for e in range(4, 17)]
    best = None
    for lam in lambdas:
        f = sv ** 2 / (sv ** 2 + lam)
        fit = np.einsum("ia,a,akp->ikp", U, f, UT)
        hii = np.einsum("ia,a,ia->i", U, f, U)
        loo = (Tn - fit) / (1.0 - hii)[:, None, None]
        # leaving out the smallest or the largest gap is an extrapolation: judged on the others
        inner = np.ones(len(g), bool)
        inner[[int(np.argmin(g)), int(np.argmax(g))]] = False
        e = float(np.sqrt(np.mean(loo[inner] ** 2)))
        if log:
            log(f"readout lambda {lam:.1e}: leave-one-gap-out RMS {e:.2e}, training RMS "
                f"{float(np.sqrt(np.mean((Tn - fit) ** 2))):.2e}")
        if best is None or e < best[1]:
            best = (lam, e, float(np.sqrt(np.mean((Tn - fit) ** 2))))
    lam = best[0]
    coef = Vt.T @ np.diag(sv / (sv ** 2 + lam))  # (W + 1, n_g): F^+ regularized
    M = np.einsum("ca,akp->kpc", coef, UT)  # (12, P, W + 1)
    W4 = np.zeros((12 * W, W))
    b4 = np.zeros(12 * W)
    for k in range(12):
        W4[12 * np.arange(P) + k, :] = M[k, :, :W]
        b4[12 * np.arange(P) + k] = M[k, :, W]
    p["W4"], p["b4"] = W4, b4
    p["Wh"] = np.eye(P, W)
    net.set_params(np.concatenate([p[name].ravel() for name, _ in _blocks(W, P)]).astype(np.float32))
    net.set_output_scale(scale)
    return best


def host_forward(net: WarmStartNet, gaps, motions):
    """The network's standardized outputs o (k, nout) in FP64 on the host from its parameters (a check of
    the library's BF16 forward; not used for prediction)."""
    W, P = net.width, net.nout
    flat = net.get_params().astype(np.float64)
    p, off = {}, 0
    for name, shp in _blocks(W, P):
        k = int(np.prod(shp))
        p[name] = flat[off:off + k].reshape(shp)
        off += k
    gt = ((np.log(np.asarray(gaps, float)) - net.g_mid) / net.g_half)[:, None]
    h = np.tanh(gt @ p["W1"].T + p["b1"])
    h = np.tanh(h @ p["W2"].T + p["b2"])
    h = np.tanh(h @ p["W3"].T + p["b3"])
    C = (h @ p["W4"].T + p["b4"]).reshape(len(gt), W, 12)
    z = np.einsum("nwk,nk->nw", C, np.asarray(motions, float).reshape(len(gt), 12))
    return z @ p["Wh"].T


class PodDecoder:
    """The network's output layer expressed in principal directions of the training data: the rows of
    Y (n, P) span (to a relative energy rel^2) the columns of V (P, r), orthonormal; the network is
    trained to predict z = V^T y (r values) and the coarse density is V z.  V comes from the n x n Gram
    matrix Y Y^T (eigenvectors U, eigenvalues e: V = Y^T U e^-1/2), then one QR pass to restore
    orthogonality.  The data are linear in the motion and so is V z."""

    def __init__(self, Y, rel: float = 3e-7, rmax: int = 1536):
        import torch

        G = (Y @ Y.T).cpu().numpy()
        e, U = np.linalg.eigh(0.5 * (G + G.T))
        e, U = e[::-1].clip(min=0.0), U[:, ::-1]
        # the Gram matrix resolves energies down to ~1e-16 of the largest; below that the eigenpairs
        # are rounding noise and are never kept
        e = np.where(e > 1e-14 * e[0], e, 0.0)
        tail = np.concatenate([np.cumsum(e[::-1])[::-1][1:], [0.0]])  # energy beyond the first k+1 modes
        tot = e.sum()
        r = int(np.argmax(tail <= rel * rel * tot)) + 1 if tot > 0 else 1
        r = max(1, min(r, rmax, int((e > 0).sum())))
        Ur = torch.as_tensor(np.ascontiguousarray(U[:, :r] / np.sqrt(e[:r])), device=Y.device)
        V = Y.T @ Ur
        self.V, _ = torch.linalg.qr(V)
        self.V = self.V.contiguous()
        self.r = r
        self.energy_tail = float(tail[r - 1] / tot) if tot > 0 else 0.0
        self.eigenvalues = e

    @classmethod
    def from_basis(cls, V):
        """A decoder with the given orthonormal columns V (P, r) (e.g. as saved by save_model)."""
        obj = cls.__new__(cls)
        obj.V = V.contiguous()
        obj.r = int(V.shape[1])
        obj.energy_tail = float("nan")
        obj.eigenvalues = None
        return obj

    def encode(self, Y):
        return Y @ self.V

    def decode(self, z):
        return self.V @ z


def network_predictor(net: WarmStartNet, pod: PodDecoder | None = None):
    """predict(gap, motion) of the trained network (the coarse values it was trained on; through the
    PodDecoder when the network predicts its coefficients)."""
    import torch

    def predict(gap, motion):
        g = torch.tensor([gap], dtype=torch.float64, device="cuda")
        m = _dev(np.asarray(motion, float).reshape(1, 12))
        z = net.predict(g, m).reshape(-1)
        return z if pod is None else pod.decode(z)

    return predict


def save_model(path, net: WarmStartNet, pod: PodDecoder, gaps, motions, T, meta: dict):
    """Writes a trained warm start to the directory `path` (numpy .npy files and a JSON file): the
    network's parameters and output scale, the principal directions (FP32: their rounding, 6e-8
    relative, is far below the data's accuracy), and the training data as coefficients T (so that the
    log(gap) interpolation control can be rebuilt) with its gaps and motions."""
    import json
    import os

    import torch

    os.makedirs(path, exist_ok=True)
    np.save(os.path.join(path, "params.npy"), net.get_params())
    np.save(os.path.join(path, "scale.npy"), net.output_scale().cpu().numpy())
    np.save(os.path.join(path, "pod_v.npy"), pod.V.to(dtype=torch.float32).cpu().numpy())
    np.save(os.path.join(path, "coeffs.npy"), T.cpu().numpy())
    np.save(os.path.join(path, "gaps.npy"), np.asarray(gaps, float))
    np.save(os.path.join(path, "motions.npy"), np.asarray(motions, float))
    with open(os.path.join(path, "meta.json"), "w") as f:
        json.dump(dict(meta, width=net.width, nout=net.nout, passes=meta.get("passes", 3)), f)


def load_model(path):
    """Reads what save_model wrote: (net, pod, gaps, motions, T, meta)."""
    import json
    import os

    import torch

    with open(os.path.join(path, "meta.json")) as f:
        meta = json.load(f)
    net = WarmStartNet(meta["width"], meta["nout"], max_batch=64, passes=meta["passes"])
    net.set_params(np.load(os.path.join(path, "params.npy")).astype(np.float32))
    net.set_output_scale(torch.as_tensor(np.load(os.path.join(path, "scale.npy")), dtype=torch.float64, device="cuda"))
    V = torch.as_tensor(np.load(os.path.join(path, "pod_v.npy")), dtype=torch.float64, device="cuda")
    T = torch.as_tensor(np.load(os.path.join(path, "coeffs.npy")), dtype=torch.float64, device="cuda")
    return (net, PodDecoder.from_basis(V), np.load(os.path.join(path, "gaps.npy")),
            np.load(os.path.join(path, "motions.npy")), T, meta)
