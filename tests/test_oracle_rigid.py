"""Pins of the rigid-sphere oracle (oracle/rigid.py) against facts that do not come from it.

- completion closed forms on one unit sphere: A U = (1/8 pi) (sum w) (U + n (n.U)) exactly for a
  constant density (the subtracted double layer of a constant is chi q = q/2 on the surface), and
  A (Omega x d) ~ (1/3) Omega x d (rotlet of L = (8 pi / 3) Omega);
- interpolation stencil: the 6 x 6 tensor stencil's error at points off the grid falls like h^6, and
  it reproduces polynomials of degree 5 in each grid coordinate exactly;
- single translating / rotating sphere: the solved density's exterior flow equals Stokes' solution;
- GMRES: matches a dense solve on a small nonsymmetric system.
"""
import numpy as np
import pytest

import workload
from oracle.rigid import RigidProblem, Sphere, gmres


def one_sphere(h):
    s = workload.sphere_quadrature(h)
    return RigidProblem([Sphere(s, np.zeros(3), 1.0, h)], h), s


def test_completion_of_constant_density():
    prob, s = one_sphere(1 / 8)
    U = np.array([0.3, -1.2, 0.7])
    q = np.tile(U, (prob.ntot, 1))
    got = prob.matvec(q)
    n = s.normal
    ex = s.w.sum() / (8 * np.pi) * (U + n * (n @ U)[:, None])
    assert np.abs(got - ex).max() <= 1e-13
    # and sum w is the sphere's area to the quadrature's accuracy
    assert abs(workload.sphere_quadrature(1 / 16).w.sum() - 4 * np.pi) <= 1e-4


def test_completion_of_rotation():
    prob, s = one_sphere(1 / 12)
    Om = np.array([0.4, 0.9, -0.5])
    q = np.cross(Om, s.x)
    got = prob.matvec(q)
    ex = np.cross(Om, s.x) / 3.0
    err = np.abs(got - ex).max()
    print(f"rotation: {err:.2e}")
    assert err <= 2e-3


def test_stencil_error_is_sixth_order():
    errs = []
    rng = np.random.default_rng(7)
    d = rng.standard_normal((40, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]

    def field(x):
        return np.stack([np.sin(1.3 * x[:, 0] + 0.4 * x[:, 1]), np.cos(x[:, 2] - 0.7 * x[:, 0]),
                         np.exp(0.5 * x[:, 1]) * x[:, 2]], axis=1)

    for h in (1 / 16, 1 / 32, 1 / 64):
        s = workload.sphere_quadrature(h)
        sp = Sphere(s, np.zeros(3), 1.0, h)
        idx, wts = sp.stencils(d)
        # near the corners of the families' sheets a coarse grid has no 6 x 6 stencil (narrower ones
        # are taken there); from h = 1/32 on every point has one
        assert (np.count_nonzero(wts, axis=1) == 36).all() or h == 1 / 16
        q = field(s.x)
        est = np.einsum("ks,ksc->kc", wts, q[idx])
        errs.append(np.abs(est - field(d)).max())
    print("stencil errors", errs, "ratios", errs[0] / errs[1], errs[1] / errs[2])
    # h^6: a factor 64 per halving (asymptotically); h^4 would give 16
    assert errs[1] / errs[2] >= 40 and errs[2] <= 1e-8


def test_stencil_reproduces_quintic_polynomials():
    """On a sheet of family i the grid coordinates are (x_j, x_k); a polynomial of degree <= 5 in
    each of them is interpolated exactly by the 6 x 6 tensor stencil (to rounding)."""
    h = 1 / 16
    s = workload.sphere_quadrature(h)
    sp = Sphere(s, np.zeros(3), 1.0, h)
    rng = np.random.default_rng(11)
    d = rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    idx, wts = sp.stencils(d)
    full = np.count_nonzero(wts, axis=1) == 36
    assert full.mean() > 0.9
    # the family of each stencil: the axis whose coordinate is not a grid coordinate of all its points
    C = rng.standard_normal((6, 6))

    def poly(a, b):
        return sum(C[i, j] * a ** i * b ** j for i in range(6) for j in range(6))

    bad = 0
    for t in np.nonzero(full)[0]:
        pts = s.x[idx[t]]
        fam = [i for i in range(3) if np.allclose(np.round(pts[:, [j for j in range(3) if j != i]] / h),
                                                    pts[:, [j for j in range(3) if j != i]] / h, atol=1e-9)]
        i = fam[0]
        j, k = [e for e in range(3) if e != i]
        got = wts[t] @ poly(pts[:, j], pts[:, k])
        ex = poly(d[t, j], d[t, k])
        bad += abs(got - ex) > 1e-10 * max(1.0, abs(ex))
    assert bad == 0


@pytest.mark.parametrize("kind", ["translate", "rotate"])
def test_single_sphere_stokes_flow(kind):
    h = 1 / 12
    prob, s = one_sphere(h)
    U = np.array([0.3, -0.5, 0.8])
    Om = np.array([0.4, 0.1, -0.6])
    motion = np.r_[U, 0, 0, 0] if kind == "translate" else np.r_[0, 0, 0, Om]
    b = prob.rhs(motion[None, :])
    q, it, rr = gmres(prob.matvec, b, tol=1e-10, maxit=80)
    y = np.array([[1.5, 0.2, 0.1], [0.0, -2.0, 0.5], [1.1, 1.1, 1.1], [0.0, 0.0, 3.0]])
    u = prob.velocity(q.reshape(-1, 3), y)
    r = np.linalg.norm(y, axis=1)[:, None]
    if kind == "translate":
        Uy = (y @ U)[:, None]
        ex = 0.75 * (U / r + Uy * y / r ** 3) + 0.25 * (U / r ** 3 - 3 * Uy * y / r ** 5)
    else:
        ex = np.cross(Om, y) / r ** 3
    err = np.abs(u - ex).max()
    print(f"{kind}: iters {it} flow error {err:.2e}")
    assert rr <= 1e-10 and err <= 2e-3


def test_gmres_matches_dense_solve():
    rng = np.random.default_rng(3)
    n = 60
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    x, it, rr = gmres(lambda v: A @ v, b, tol=1e-13, maxit=n)
    assert np.abs(x - np.linalg.solve(A, b)).max() <= 1e-11
    assert rr <= 1e-13 and it <= n
