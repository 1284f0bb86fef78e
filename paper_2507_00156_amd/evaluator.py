"""Convenience wrapper around one library context: owns it, allocates output tensors, forwards calls."""
from __future__ import annotations

from . import binding as B


class Evaluator:
    """One surface on one GPU.  All tensors are float64 CUDA tensors; outputs are allocated here."""

    def __init__(self, h: float, rho=(2.0, 3.0, 4.0), cutoff: float = 6.0, precision: int = B.SR_FP64,
                 far_method: int = B.SR_DIRECT, tree_degree: int = 8, tree_theta: float = 0.7,
                 tree_leaf: int = 2000, device: int = 0):
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


class RigidSpheres:
    """Rigid spheres in Stokes flow (completed double layer, GMRES); thin wrapper of sr_rigid_*."""

    def __init__(self, h: float, rho=(2.0, 3.0, 4.0), cutoff: float = 6.0, precision: int = B.SR_FP64,
                 far_method: int = B.SR_DIRECT, tree_degree: int = 8, tree_theta: float = 0.7,
                 tree_leaf: int = 2000, device: int = 0):
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

    def solve(self, rhs, x0=None, tol=1e-8, maxit=200, restart=60, stream=None):
        """Returns (x, iterations, relative residual)."""
        import torch

        x = torch.zeros_like(rhs) if x0 is None else x0.clone()
        it, rr = B.sr_rigid_solve(self.r, rhs, x, x0 is not None, tol, maxit, restart, stream)
        return x, it, rr

    def solve_refined(self, rhs, x0=None, tol=1e-10, inner_tol=1e-4, maxit=400, restart=60, stream=None):
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
