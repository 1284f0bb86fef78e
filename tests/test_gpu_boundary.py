"""The boundary's target kinds and its consistency report, on the GPU through the C ABI.

- sr_eval_far (targets with no closest point: the plain sums of eqs. (Stokes_SL), (Stokes_DL)) against
  the oracle's plain sums at targets far from the surface;
- SR_ENEAR (sr_check) for a far-kind target inside the near radius, and for an sr_eval target whose
  stated |b| selects the far rule while a source is closer (paper section 3.3: the regularization
  acts within cutoff * delta of a source), and no report for honest targets;
- the host-pointer mode (SR_HOST) gives the device mode's results bit for bit;
- an evaluation of more than 2^20 targets (run in chunks) equals its targets' single evaluations.
"""
import numpy as np
import pytest

import oracle
import workload
from tests.gpu_helpers import rel_err, to_dev

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-7}


def _setup(cfg, precision):
    import paper_2507_00156_amd as P

    s = cfg["surf"]
    ev = P.Evaluator(cfg["h"], cfg["rho"], precision=precision)
    ev.set_surface(to_dev(s.x), to_dev(s.normal), to_dev(s.w))
    ev.set_density(P.SR_SL, to_dev(cfg["f"]))
    ev.set_density(P.SR_DL, to_dev(cfg["q"]))
    return ev


def _far_points(m, radius, seed):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((m, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return radius * d * rng.uniform(1.0, 1.5, (m, 1))


@pytest.mark.parametrize("precision", [0, 1])
def test_eval_far_matches_oracle_plain_sums(precision):
    import torch

    import paper_2507_00156_amd as P

    cfg = workload.build_config("small")
    s = cfg["surf"]
    y = _far_points(700, 2.5, 11)  # beyond 1.5 from the ellipsoid (1, 0.8, 0.6); near radius 24 h = 1.0
    ev = _setup(cfg, precision)
    u, v = ev.eval_far(P.SR_SL | P.SR_DL, to_dev(y))
    torch.cuda.synchronize()
    ev.check()  # no target inside the near radius
    uo, vo = oracle.plain(s.x, s.normal, s.w, cfg["f"], cfg["q"], y)
    assert rel_err(u.cpu().numpy(), uo) <= TOL[precision]
    assert rel_err(v.cpu().numpy(), vo) <= TOL[precision]
    # single layers alone, host-pointer mode
    uh, _ = (np.empty((y.shape[0], 3)), None)
    P.binding.sr_eval_far_host(ev.ctx, P.SR_SL, np.ascontiguousarray(y), uh, None)
    assert np.array_equal(uh, u.cpu().numpy())
    ev.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_far_target_inside_near_radius_reported(precision):
    import paper_2507_00156_amd as P

    cfg = workload.build_config("small")
    t = cfg["targets"]
    y = _far_points(300, 2.5, 12)
    y[137] = t.y[-5]  # a near target given as a far one
    ev = _setup(cfg, precision)
    ev.eval_far(P.SR_SL | P.SR_DL, to_dev(y))
    with pytest.raises(P.SrError) as ei:
        ev.check()
    assert ei.value.status == P.SR_ENEAR and "target 137 " in str(ei.value)
    ev.check()  # the report was cleared
    ev.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_wrong_far_rule_b_reported_and_honest_far_rule_not(precision):
    import torch

    import paper_2507_00156_amd as P

    cfg = workload.build_config("small")
    t = cfg["targets"]
    h, rho = cfg["h"], cfg["rho"]
    rcut = 6.0 * max(rho) * h
    idx = np.arange(t.m - 200, t.m)  # near targets (|b| <= 3h)
    y, x0, n0, b = t.y[idx].copy(), t.x0[idx].copy(), t.n0[idx].copy(), t.b[idx].copy()
    f0, q0 = cfg["f0"][idx], cfg["q0"][idx]
    # honest far-rule targets: on the outward normal of a convex surface at distance 1.2 rcut
    y[:50] = x0[:50] + 1.2 * rcut * n0[:50]
    b[:50] = 1.2 * rcut
    ev = _setup(cfg, precision)
    u, v = ev.eval(P.SR_SL | P.SR_DL, to_dev(y), to_dev(x0), to_dev(n0), to_dev(b), to_dev(f0), to_dev(q0))
    torch.cuda.synchronize()
    ev.check()
    s = cfg["surf"]
    uo = oracle.sl(s.x, s.normal, s.w, cfg["f"], y, x0, n0, b, f0, h, rho)
    vo = oracle.dl(s.x, s.normal, s.w, cfg["q"], y, x0, n0, b, q0, h, rho)
    assert rel_err(u.cpu().numpy(), uo) <= TOL[precision]
    assert rel_err(v.cpu().numpy(), vo) <= TOL[precision]
    # a near target whose b claims the far rule: reported, the first such index named
    bw = b.copy()
    bw[120] = np.sign(b[120] if b[120] != 0 else 1.0) * 1.1 * rcut
    bw[170] = -1.5 * rcut
    ev.eval(P.SR_SL | P.SR_DL, to_dev(y), to_dev(x0), to_dev(n0), to_dev(bw), to_dev(f0), to_dev(q0))
    with pytest.raises(P.SrError) as ei:
        ev.check()
    assert ei.value.status == P.SR_ENEAR and "target 120 " in str(ei.value)
    ev.check()
    ev.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_host_pointer_mode_equals_device_mode(precision):
    import torch

    import paper_2507_00156_amd as P

    cfg = workload.build_config("small")
    t = cfg["targets"]
    ev = _setup(cfg, precision)
    u, v = ev.eval(P.SR_SL | P.SR_DL, to_dev(t.y), to_dev(t.x0), to_dev(t.n0), to_dev(t.b), to_dev(cfg["f0"]),
                   to_dev(cfg["q0"]))
    torch.cuda.synchronize()
    uh, vh = ev.eval_host(P.SR_SL | P.SR_DL, t.y, t.x0, t.n0, t.b, cfg["f0"], cfg["q0"])
    assert np.array_equal(uh, u.cpu().numpy()) and np.array_equal(vh, v.cpu().numpy())
    _, vd = ev.eval_host(P.SR_DL, t.y, t.x0, t.n0, t.b, None, cfg["q0"])
    assert np.array_equal(vd, v.cpu().numpy())
    ev.close()


def test_evaluation_in_chunks_equals_one_chunk():
    """More than 2^20 targets are evaluated in chunks of 2^20 one after the other: every target's
    result equals (bit for bit) that of an evaluation of its own copy alone, and a report of the second
    chunk names the target's index in the whole call."""
    import torch

    import paper_2507_00156_amd as P

    cfg = workload.build_config("small")
    t = cfg["targets"]
    reps = (1 << 20) // t.m + 2  # more than 2^20 targets in all
    m = reps * t.m
    ev = _setup(cfg, 1)
    args1 = [to_dev(a) for a in (t.y, t.x0, t.n0, t.b, cfg["f0"], cfg["q0"])]
    u1, v1 = ev.eval(P.SR_SL | P.SR_DL, *args1)
    torch.cuda.synchronize()
    argsn = [a.repeat((reps, 1)) if a.dim() == 2 else a.repeat(reps) for a in args1]
    un, vn = ev.eval(P.SR_SL | P.SR_DL, *argsn)
    torch.cuda.synchronize()
    ev.check()
    assert un.shape[0] == m > (1 << 20)
    assert torch.equal(un, u1.repeat((reps, 1))) and torch.equal(vn, v1.repeat((reps, 1)))
    # a copy, in the second chunk, of a surface target (its own point is a source) whose b claims the
    # far rule
    h, rho = cfg["h"], cfg["rho"]
    on = int(np.nonzero(t.b == 0.0)[0][0])
    k = ((1 << 20) // t.m + 1) * t.m + on
    assert k > (1 << 20)
    bw = argsn[3].clone()
    bw[k] = 1.5 * 6.0 * max(rho) * h
    ev.eval(P.SR_SL | P.SR_DL, argsn[0], argsn[1], argsn[2], bw, argsn[4], argsn[5])
    with pytest.raises(P.SrError) as ei:
        ev.check()
    assert ei.value.status == P.SR_ENEAR and f"target {k} " in str(ei.value)
    ev.check()
    ev.close()
