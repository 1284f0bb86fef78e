"""On-surface targets with the modified smoothing (paper section 2.1) on the GPU vs the oracle:
targets on the surface against oracle.sl_sharp / dl_sharp at delta = 3h, the other targets against
the extrapolated oracle; FP64 <= 1e-10 and mixed <= 1e-7 relative; the per-delta outputs of an
on-surface target repeat its single value; the rigid-sphere operator with this option vs the oracle's."""
import numpy as np
import pytest

import oracle
import workload
from oracle.rigid import RigidProblem, Sphere
from tests.gpu_helpers import rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2507_00156_amd as P

    P.load_library()
    return P


def oracle_mixed(cfg, layer):
    s, t = cfg["surf"], cfg["targets"]
    on = t.b == 0.0
    h = cfg["h"]
    out = np.empty((t.m, 3))
    if layer == "sl":
        out[on] = oracle.sl_sharp(s.x, s.normal, s.w, cfg["f"], t.y[on], t.n0[on], cfg["f0"][on], 3 * h)
        out[~on] = oracle.sl(s.x, s.normal, s.w, cfg["f"], t.y[~on], t.x0[~on], t.n0[~on], t.b[~on],
                             cfg["f0"][~on], h, cfg["rho"])
    else:
        out[on] = oracle.dl_sharp(s.x, s.normal, s.w, cfg["q"], t.y[on], t.n0[on], cfg["q0"][on], 3 * h)
        out[~on] = oracle.dl(s.x, s.normal, s.w, cfg["q"], t.y[~on], t.x0[~on], t.n0[~on], t.b[~on],
                             cfg["q0"][~on], h, cfg["rho"])
    return out


@pytest.mark.parametrize("name", ["c1", "small"])
@pytest.mark.parametrize("precision", [0, 1])
def test_sharp_matches_oracle(P, name, precision):
    cfg = workload.build_config(name)
    s, t = cfg["surf"], cfg["targets"]
    ev = P.Evaluator(cfg["h"], cfg["rho"], precision=precision, surface_sharp=True, sharp_rho=3.0)
    ev.set_surface(to_dev(s.x), to_dev(s.normal), to_dev(s.w))
    ev.set_density(P.SR_SL, to_dev(cfg["f"]))
    ev.set_density(P.SR_DL, to_dev(cfg["q"]))
    u, v, ud, vd = ev.eval(P.SR_SL | P.SR_DL, to_dev(t.y), to_dev(t.x0), to_dev(t.n0), to_dev(t.b),
                           to_dev(cfg["f0"]), to_dev(cfg["q0"]), want_delta=True)
    u, v, ud, vd = (x.cpu().numpy() for x in (u, v, ud, vd))
    eu, ev_ = rel_err(u, oracle_mixed(cfg, "sl")), rel_err(v, oracle_mixed(cfg, "dl"))
    print(f"{name} sharp prec={precision}: SL {eu:.3e} DL {ev_:.3e}", flush=True)
    tol = 1e-10 if precision == 0 else 1e-7
    assert eu <= tol and ev_ <= tol
    on = t.b == 0.0
    for arr, full in ((ud, u), (vd, v)):
        for j in range(3):
            np.testing.assert_array_equal(arr[on, j, :], full[on] if arr is ud else arr[on, 0, :])
    ev.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_rigid_sharp_matvec_matches_oracle(P, precision):
    h, gap = 1 / 16, 0.1
    cen, rad, surfs = workload.two_spheres(h, gap)
    x = np.concatenate([s.x for s in surfs])
    n = np.concatenate([s.normal for s in surfs])
    w = np.concatenate([s.w for s in surfs])
    R = P.RigidSpheres(h, precision=precision, surface_sharp=True)
    R.set_spheres(cen, rad, [s.n for s in surfs], to_dev(x), to_dev(n), to_dev(w))
    rng = np.random.default_rng(5)
    q = np.concatenate([workload.harmonic_field(workload.harmonic_coeffs(3, rng), s.x, c) for s, c in zip(surfs, cen)])
    g = R.matvec(to_dev(q)).cpu().numpy()
    prob = RigidProblem([Sphere(s, c, a, h) for s, c, a in zip(surfs, cen, rad)], h, sharp=True)
    o = prob.matvec(q)
    e = rel_err(g, o)
    print(f"rigid sharp matvec prec={precision}: {e:.3e}", flush=True)
    assert e <= (1e-10 if precision == 0 else 1e-7)
    R.close()
