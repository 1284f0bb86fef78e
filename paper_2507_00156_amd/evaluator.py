"""Convenience wrapper around one library context: owns it, allocates output tensors, forwards calls."""
from __future__ import annotations

from . import binding as B


class Evaluator:
    """One surface on one GPU.  All tensors are float64 CUDA tensors; outputs are allocated here."""

    def __init__(self, h: float, rho=(2.0, 3.0, 4.0), cutoff: float = 6.0, precision: int = B.SR_FP64,
                 far_method: int = B.SR_DIRECT, tree_degree: int = 8, tree_theta: float = 0.7,
                 tree_leaf: int = 2000, surface_sharp: bool = False, sharp_rho: float = 3.0, device: int = 0):
        import torch

        self.device = torch.device("cuda", device)
        self.ctx = B.sr_create(device)
        p = B.sr_default_params()
        p.h = float(h)
        for j in range(3):
            p.rho[j] = float(rho[j])
        p.cutoff = float(cutoff)
        p.precision = int(precision)
        p.far_method = int(far_method)
        p.tree_degree = int(tree_degree)
        p.tree_theta = float(tree_theta)
        p.tree_leaf = int(tree_leaf)
        p.surface_sharp = int(bool(surface_sharp))
        p.sharp_rho = float(sharp_rho)
        try:
            B.sr_set_params(self.ctx, p)
        except Exception:
            B.sr_destroy(self.ctx)
            self.ctx = None
            raise
        self.params = p
        self.n = 0

    def close(self) -> None:
        if self.ctx is not None:
            B.sr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, **kw) -> None:
        p = self.params
        for k, v in kw.items():
            if k == "rho":
                for j in range(3):
                    p.rho[j] = float(v[j])
            else:
                setattr(p, k, v)
        B.sr_set_params(self.ctx, p)

    def tree_work(self, y_host):
        """(target-proxy interactions, leaf pairs, points in accepted clusters) of the treecode far field
        for host targets y_host."""
        return B.sr_tree_work(self.ctx, y_host)

    def set_surface(self, x, nrm, w, stream=None) -> None:
        B.sr_set_surface(self.ctx, x, nrm, w, stream)
        self.n = int(x.shape[0])

    def set_density(self, layer: int, dens, stream=None) -> None:
        B.sr_set_density(self.ctx, layer, dens, stream)

    def eval(self, layers: int, y, x0, n0, b, f0=None, q0=None, want_delta: bool = False, stream=None, out=None):
        """Returns (u, v[, u_delta, v_delta]); entries for layers not requested are None."""
        import torch

        m = int(y.shape[0])
        kw = dict(dtype=torch.float64, device=y.device)
        if out is not None:
            u, v, ud, vd = out
        else:
            u = torch.empty((m, 3), **kw) if layers & B.SR_SL else None
            v = torch.empty((m, 3), **kw) if layers & B.SR_DL else None
            ud = torch.empty((m, 3, 3), **kw) if (want_delta and layers & B.SR_SL) else None
            vd = torch.empty((m, 3, 3), **kw) if (want_delta and layers & B.SR_DL) else None
        B.sr_eval(self.ctx, layers, y, x0, n0, b, f0, q0, u, v, ud, vd, stream)
        return (u, v, ud, vd) if want_delta else (u, v)

    def eval_far(self, layers: int, y, stream=None, out=None):
        """Plain sums at targets with no closest point; returns (u, v) (None for a layer not asked for).
        A target within the near radius of a source is reported by check()."""
        import torch

        m = int(y.shape[0])
        kw = dict(dtype=torch.float64, device=y.device)
        if out is not None:
            u, v = out
        else:
            u = torch.empty((m, 3), **kw) if layers & B.SR_SL else None
            v = torch.empty((m, 3), **kw) if layers & B.SR_DL else None
        B.sr_eval_far(self.ctx, layers, y, u, v, stream)
        return u, v

    def eval_host(self, layers: int, y, x0, n0, b, f0=None, q0=None):
        """sr_eval on host (numpy) arrays; returns numpy (u, v)."""
        import numpy as np

        m = int(y.shape[0])
        u = np.empty((m, 3)) if layers & B.SR_SL else None
        v = np.empty((m, 3)) if layers & B.SR_DL else None
        c = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)  # noqa: E731
        B.sr_eval_host(self.ctx, layers, c(y), c(x0), c(n0), c(b), c(f0), c(q0), u, v)
        return u, v

    def check(self, stream=None) -> None:
        """Raises SrError (SR_ENEAR) if a target treated as far lay within the near radius of a source."""
        B.sr_check(self.ctx, stream)


class RigidSpheres:
    """Rigid spheres in Stokes flow (completed double layer, GMRES); thin wrapper of sr_rigid_*."""

    def __init__(self, h: float, rho=(2.0, 3.0, 4.0), cutoff: float = 6.0, precision: int = B.SR_FP64,
                 far_method: int = B.SR_DIRECT, tree_degree: int = 8, tree_theta: float = 0.7,
                 tree_leaf: int = 2000, surface_sharp: bool = False, sharp_rho: float = 3.0, device: int = 0):
        self.r = B.sr_rigid_create(device)
        p = B.sr_default_params()
        p.h = float(h)
        for j in range(3):
            p.rho[j] = float(rho[j])
        p.cutoff = float(cutoff)
        p.precision = int(precision)
        p.far_method = int(far_method)
        p.tree_degree = int(tree_degree)
        p.tree_theta = float(tree_theta)
        p.tree_leaf = int(tree_leaf)
        p.surface_sharp = int(bool(surface_sharp))
        p.sharp_rho = float(sharp_rho)
        try:
            B.sr_rigid_set_params(self.r, p)
        except Exception:
            B.sr_rigid_destroy(self.r)
            self.r = None
            raise
        self.ntot = 0

    def close(self) -> None:
        if self.r is not None:
            B.sr_rigid_destroy(self.r)
            self.r = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_spheres(self, centers, radii, counts, x, nrm, w, stream=None) -> None:
        B.sr_rigid_set_spheres(self.r, centers, radii, counts, x, nrm, w, stream)
        self.ntot = int(x.shape[0])

    def rhs(self, motion, stream=None):
        import torch

        out = torch.empty((self.ntot, 3), dtype=torch.float64, device="cuda")
        B.sr_rigid_rhs(self.r, motion, out, stream)
        return out

    def matvec(self, q, stream=None):
        import torch

        out = torch.empty_like(q)
        B.sr_rigid_matvec(self.r, q, out, stream)
        return out

    def set_operator(self, a_id: float, a_dl: float, completion: bool) -> None:
        B.sr_rigid_set_operator(self.r, a_id, a_dl, completion)

    def single_layer(self, f, stream=None):
        import torch

        out = torch.empty_like(f)
        B.sr_rigid_single_layer(self.r, f, out, stream)
        return out

    def solve(self, rhs, x0=None, tol=1e-8, maxit=200, restart=60, stream=None):
        """Returns (x, iterations, relative residual)."""
        import torch

        x = torch.zeros_like(rhs) if x0 is None else x0.clone()
        it, rr = B.sr_rigid_solve(self.r, rhs, x, x0 is not None, tol, maxit, restart, stream)
        return x, it, rr

    def solve_refined(self, rhs, x0=None, tol=1e-10, inner_tol=1e-6, maxit=400, restart=60, stream=None):
        """Iterative refinement (FP64 residuals, working-precision GMRES corrections).
        Returns (x, inner iterations, outer corrections, FP64 relative residual)."""
        import torch

        x = torch.zeros_like(rhs) if x0 is None else x0.clone()
        it, no, rr = B.sr_rigid_solve_refined(self.r, rhs, x, x0 is not None, tol, inner_tol, maxit, restart, stream)
        return x, it, no, rr

    def velocity(self, q, y, stream=None):
        import torch

        u = torch.empty_like(y)
        B.sr_rigid_velocity(self.r, q, y, u, stream)
        return u


class Prolongation:
    """Coarse-to-fine interpolation of densities on spheres (sr_prolong_*)."""

    def __init__(self, centers, radii, hc, counts_c, xc, nc, counts_f, xf, device: int = 0, stream=None):
        self.p = B.sr_prolong_create(centers, radii, hc, counts_c, xc, nc, counts_f, xf, device, stream)
        self.nf = int(xf.shape[0])

    def __call__(self, qc, stream=None):
        import torch

        qf = torch.empty((self.nf, 3), dtype=torch.float64, device=qc.device)
        B.sr_prolong_apply(self.p, qc, qf, stream)
        return qf

    def close(self) -> None:
        if self.p is not None:
            B.sr_prolong_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class WarmStartNet:
    """The warm-start network (sr_mlp_*): gap + 12 motion parameters -> coarse density."""

    def __init__(self, width: int, nout: int, max_batch: int, passes: int = 3, g_mid: float = -2.760730458931123,
                 g_half: float = 1.151292546497023, device: int = 0):
        self.width, self.nout, self.max_batch = int(width), int(nout), int(max_batch)
        self.g_mid, self.g_half = float(g_mid), float(g_half)
        self.net = B.sr_mlp_create(width, nout, max_batch, device)
        self.nparam = B.sr_mlp_num_params(width, nout)
        B.sr_mlp_set_options(self.net, passes, g_mid, g_half)

    def close(self) -> None:
        if self.net is not None:
            B.sr_mlp_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_options(self, passes: int = 3, g_mid: float = -2.760730458931123, g_half: float = 1.151292546497023) -> None:
        B.sr_mlp_set_options(self.net, passes, g_mid, g_half)
        self.g_mid, self.g_half = float(g_mid), float(g_half)

    def set_params(self, flat) -> None:
        B.sr_mlp_set_params(self.net, flat)

    def get_params(self):
        return B.sr_mlp_get_params(self.net, self.nparam)

    def fit_output_scale(self, y, stream=None) -> None:
        B.sr_mlp_fit_output_scale(self.net, y, stream)

    def set_output_scale(self, s, stream=None) -> None:
        B.sr_mlp_set_output_scale(self.net, s, stream)

    def output_scale(self, stream=None):
        import torch

        s = torch.empty(self.nout, dtype=torch.float64, device="cuda")
        B.sr_mlp_get_output_scale(self.net, s, stream)
        return s

    def forward(self, gap, motion, stream=None):
        import torch

        out = torch.empty((gap.shape[0], self.nout), dtype=torch.float32, device=gap.device)
        B.sr_mlp_forward(self.net, gap, motion, out, stream)
        return out

    def predict(self, gap, motion, stream=None):
        import torch

        q = torch.empty((gap.shape[0], self.nout), dtype=torch.float64, device=gap.device)
        B.sr_mlp_predict(self.net, gap, motion, q, stream)
        return q

    def gradients(self, gap, motion, y, idx=None, batch=None, stream=None):
        import torch

        g = torch.empty(self.nparam, dtype=torch.float32, device=gap.device)
        b = int(gap.shape[0] if batch is None else batch)
        loss = B.sr_mlp_gradients(self.net, b, idx, gap, motion, y, g, stream)
        return g, loss

    def set_profiling(self, on: bool) -> None:
        B.sr_mlp_set_profiling(self.net, on)

    def get_profile(self):
        return B.sr_mlp_get_profile(self.net)

    def train_step(self, gap, motion, y, lr, idx=None, batch=None, want_loss=True, stream=None):
        b = int(gap.shape[0] if batch is None else batch)
        return B.sr_mlp_train_step(self.net, b, idx, gap, motion, y, lr, want_loss, stream)
