"""GPU treecode far field (paper section 3.4) against the oracle treecode, which takes the same
per-target steps (same octree, same MAC, same proxies), and against the direct sums.

Bars: FP64 path <= 1e-10, mixed path <= 1e-7 relative to the oracle treecode; theta = 0 reproduces
the direct evaluation; the treecode error against the direct sum falls with the degree p.
"""
import numpy as np
import pytest

import oracle
import workload
from tests.gpu_helpers import gpu_eval, rel_err, to_dev, tree_mac_radius

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-7}


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2507_00156_amd as P

    P.load_library()
    return P


def tree_eval(P, cfg, precision, p, theta, leaf, idx=None):
    import torch

    s, t = cfg["surf"], cfg["targets"]
    ev = P.Evaluator(cfg["h"], cfg["rho"], precision=precision, far_method=P.SR_TREE, tree_degree=p,
                     tree_theta=theta, tree_leaf=leaf)
    ev.set_surface(to_dev(s.x), to_dev(s.normal), to_dev(s.w))
    ev.set_density(P.SR_SL, to_dev(cfg["f"]))
    ev.set_density(P.SR_DL, to_dev(cfg["q"]))
    sel = slice(None) if idx is None else np.asarray(idx)
    u, v = ev.eval(P.SR_SL | P.SR_DL, to_dev(t.y[sel]), to_dev(t.x0[sel]), to_dev(t.n0[sel]), to_dev(t.b[sel]),
                   to_dev(cfg["f0"][sel]), to_dev(cfg["q0"][sel]))
    torch.cuda.synchronize()
    out = u.cpu().numpy(), v.cpu().numpy()
    ev.close()
    return out


@pytest.fixture(scope="module")
def small():
    return workload.build_config("small")


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("p,theta,leaf", [(6, 0.7, 200), (4, 0.5, 60), (8, 0.9, 500)])
def test_tree_matches_oracle_tree(P, small, precision, p, theta, leaf):
    cfg = small
    gu, gv = tree_eval(P, cfg, precision, p, theta, leaf)
    ou, ov = oracle.tree_cfg(cfg, None, p=p, theta=theta, leaf=leaf, mac_rnear=tree_mac_radius(cfg, precision))
    e1, e2 = rel_err(gu, ou), rel_err(gv, ov)
    print(f"tree p={p} theta={theta} leaf={leaf} prec={precision}: SL {e1:.3e} DL {e2:.3e}", flush=True)
    assert e1 <= TOL[precision] and e2 <= TOL[precision]


def test_theta_zero_is_direct(P, small):
    gu, gv = tree_eval(P, small, 0, 4, 0.0, 100)
    du, dv = gpu_eval(small, 3, 0)
    assert rel_err(gu, du) <= 1e-12 and rel_err(gv, dv) <= 1e-12


@pytest.mark.parametrize("precision", [0, 1])
def test_theta_zero_is_direct_with_modified_smoothing(P, small, precision):
    """With the on-surface modified smoothing, surface targets have a smaller near radius than the
    others; at theta = 0 the treecode's leaf sums must take exactly the pairs the direct far field
    takes (each target's own radius), so the two far fields agree to rounding."""
    import torch

    cfg = small
    s, t = cfg["surf"], cfg["targets"]
    outs = []
    for far in (P.SR_DIRECT, P.SR_TREE):
        ev = P.Evaluator(cfg["h"], cfg["rho"], precision=precision, far_method=far, tree_degree=4, tree_theta=0.0,
                         tree_leaf=100, surface_sharp=True, sharp_rho=3.0)
        ev.set_surface(to_dev(s.x), to_dev(s.normal), to_dev(s.w))
        ev.set_density(P.SR_SL, to_dev(cfg["f"]))
        ev.set_density(P.SR_DL, to_dev(cfg["q"]))
        u, v = ev.eval(P.SR_SL | P.SR_DL, to_dev(t.y), to_dev(t.x0), to_dev(t.n0), to_dev(t.b), to_dev(cfg["f0"]),
                       to_dev(cfg["q0"]))
        torch.cuda.synchronize()
        outs.append((u.cpu().numpy(), v.cpu().numpy()))
        ev.close()
    e1, e2 = rel_err(outs[1][0], outs[0][0]), rel_err(outs[1][1], outs[0][1])
    print(f"theta 0 with modified smoothing, precision {precision}: SL {e1:.2e} DL {e2:.2e}", flush=True)
    bar = 1e-12 if precision == 0 else 1e-6
    assert e1 <= bar and e2 <= bar


def test_tree_error_vs_direct_decreases_with_p(P):
    cfg = workload.build_config("c2", m_near=2000)
    du, dv = gpu_eval(cfg, 3, 0)
    errs = []
    for p in (4, 6, 8):
        gu, gv = tree_eval(P, cfg, 0, p, 0.7, 2000)
        errs.append(max(rel_err(gu, du), rel_err(gv, dv)))
    print("tree vs direct errors", errs, flush=True)
    # theta = 0.7 is a loose MAC: at p = 8 the error is at the level of the h = 1/64 discretization error
    assert errs[1] < errs[0] / 5 and errs[2] < errs[1] / 5 and errs[2] < 1e-5


def test_tree_c3_sampled(P):
    # the treecode workload: ellipsoid h = 1/128 (N = 169342), p = 8, theta = 0.7, N0 = 2000, mixed;
    # all targets on the GPU, 160 of them recomputed by the oracle treecode
    cfg = workload.build_config("c3")
    t = cfg["targets"]
    n = cfg["surf"].n
    rng = np.random.default_rng(7)
    idx = np.concatenate([rng.choice(n, 80, replace=False), n + rng.choice(t.m - n, 80, replace=False)])
    gu, gv = tree_eval(P, cfg, 1, 8, 0.7, 2000)
    ou, ov = oracle.tree_cfg(cfg, idx, p=8, theta=0.7, leaf=2000, mac_rnear=tree_mac_radius(cfg, 1))
    e1, e2 = rel_err(gu[idx], ou), rel_err(gv[idx], ov)
    print(f"c3 tree mixed: SL {e1:.3e} DL {e2:.3e}", flush=True)
    assert e1 <= 1e-7 and e2 <= 1e-7


def _count_tree_work(x, y, leaf, p, theta, rnear):
    """Independent count of the treecode work: the octree of section 3.4 (midpoint split into 8
    octants, upper half when x >= mid, empty octants dropped, boxes the bounding boxes of their
    points, no split when all points fall in one octant) and the MAC r_c^2 <= theta^2 R^2 with the
    box farther than rnear (the MAC's near radius), in FP64 operation by operation."""
    nodes = []

    def build(idx):
        lo, hi = x[idx].min(0), x[idx].max(0)
        nd = {"lo": lo, "hi": hi, "n": len(idx), "ch": []}
        nodes.append(nd)
        if len(idx) > leaf:
            mid = (lo + hi) * 0.5
            oc = (x[idx, 0] >= mid[0]) * 1 + (x[idx, 1] >= mid[1]) * 2 + (x[idx, 2] >= mid[2]) * 4
            parts = [idx[oc == o] for o in range(8) if (oc == o).any()]
            if len(parts) > 1:
                nd["ch"] = [build(q) for q in parts]
        rc2 = 0.0
        for d in range(3):
            e = hi[d] - lo[d]
            rc2 += 0.25 * e * e
        nd["rc2"] = rc2
        return nd

    root = build(np.arange(len(x)))
    theta2, rnear2, nprox = theta * theta, rnear * rnear, (p + 1) ** 3
    npx = nlf = ncl = 0
    stack = [(root, np.arange(len(y)))]
    while stack:
        nd, ti = stack.pop()
        yt = y[ti]
        R2 = np.zeros(len(ti))
        g2 = np.zeros(len(ti))
        for d in range(3):
            dc = yt[:, d] - 0.5 * (nd["lo"][d] + nd["hi"][d])
            R2 += dc * dc
            a, b = nd["lo"][d] - yt[:, d], yt[:, d] - nd["hi"][d]
            gap = np.where(a > 0.0, a, np.where(b > 0.0, b, 0.0))
            g2 += gap * gap
        acc = (nd["rc2"] <= theta2 * R2) & (g2 > rnear2)
        npx += int(acc.sum()) * nprox
        ncl += int(acc.sum()) * nd["n"]
        rest = ti[~acc]
        if len(rest):
            if nd["ch"]:
                stack.extend((c, rest) for c in nd["ch"])
            else:
                nlf += len(rest) * nd["n"]
    return npx, nlf, ncl


@pytest.mark.parametrize("p,theta,leaf", [(4, 0.0, 100), (6, 0.7, 200), (4, 0.5, 60)])
def test_tree_work_counts(P, small, p, theta, leaf):
    """sr_tree_work (the interaction counts behind the treecode roofline) against an independent
    count; accepted points plus leaf pairs cover every pair.  (theta = 0 still accepts clusters of
    zero extent, single points, whose proxy sum is exact.)"""
    cfg = small
    s, t = cfg["surf"], cfg["targets"]
    ev = P.Evaluator(cfg["h"], cfg["rho"], precision=1, far_method=P.SR_TREE, tree_degree=p, tree_theta=theta,
                     tree_leaf=leaf)
    ev.set_surface(to_dev(s.x), to_dev(s.normal), to_dev(s.w))
    ev.set_density(P.SR_SL, to_dev(cfg["f"]))
    ev.set_density(P.SR_DL, to_dev(cfg["q"]))
    ev.eval(P.SR_SL | P.SR_DL, to_dev(t.y), to_dev(t.x0), to_dev(t.n0), to_dev(t.b), to_dev(cfg["f0"]),
            to_dev(cfg["q0"]))
    npx, nlf, ncl = ev.tree_work(t.y)
    ev.close()
    ref = _count_tree_work(s.x, t.y, leaf, p, theta, tree_mac_radius(cfg, 1))
    print(f"tree work p={p} theta={theta} leaf={leaf}: proxy {npx} leaf {nlf} clustered {ncl}", flush=True)
    assert (npx, nlf, ncl) == ref
    assert ncl + nlf == t.m * s.n
    assert npx % (p + 1) ** 3 == 0


@pytest.fixture(scope="module")
def spheroid128():
    return workload.build_config("table1", h=1 / 128)


@pytest.mark.parametrize("precision,p,theta,leaf", [(1, 10, 0.6, 2000), (1, 12, 0.6, 2000), (0, 12, 0.6, 2000),
                                                    (1, 8, 0.6, 4000), (1, 8, 0.6, 16000), (0, 8, 0.6, 16000),
                                                    (1, 8, 0.4, 2000), (1, 8, 0.8, 2000)])
def test_tree_sweep_configurations_match_oracle(P, spheroid128, precision, p, theta, leaf):
    """The configurations of the treecode sweep (paper section 4.2: theta, N0 and p around theta 0.6,
    N0 2000, p 8, on the h = 1/128 spheroid of Table 1, N = 112006), including the largest degrees and
    leaves, against the oracle treecode on 150 sampled grid targets."""
    cfg = spheroid128
    rng = np.random.default_rng(p * 1000 + leaf + int(theta * 10))
    idx = np.sort(rng.choice(cfg["targets"].m, 150, replace=False))
    gu, gv = tree_eval(P, cfg, precision, p, theta, leaf, idx)
    ou, ov = oracle.tree_cfg(cfg, idx, p=p, theta=theta, leaf=leaf, mac_rnear=tree_mac_radius(cfg, precision))
    e1, e2 = rel_err(gu, ou), rel_err(gv, ov)
    print(f"sweep config p={p} theta={theta} N0={leaf} prec={precision}: SL {e1:.3e} DL {e2:.3e}", flush=True)
    assert e1 <= TOL[precision] and e2 <= TOL[precision]
