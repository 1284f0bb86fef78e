"""Failure handling of the rigid-sphere solve, the interpolation and the network through the C ABI:
bad arguments give SR_EINVAL, calls out of order SR_ESTATE, an iteration cap SR_ENOCONV with the last
iterate kept; nothing faults and every error leaves the object usable."""
import numpy as np
import pytest

import workload
from tests.gpu_helpers import to_dev

pytestmark = pytest.mark.gpu
EINVAL, ESTATE, ENOCONV = -1, -4, -6


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2507_00156_amd as P

    P.load_library()
    return P


def spheres(h=1 / 8, gap=0.2):
    cen, rad, surfs = workload.two_spheres(h, gap)
    x = np.concatenate([s.x for s in surfs])
    n = np.concatenate([s.normal for s in surfs])
    w = np.concatenate([s.w for s in surfs])
    return cen, rad, surfs, x, n, w


def test_rigid_errors(P):
    import torch

    h = 1 / 8
    cen, rad, surfs, x, n, w = spheres(h)
    R = P.RigidSpheres(h)
    b = torch.zeros((len(x), 3), dtype=torch.float64, device="cuda")
    with pytest.raises(P.SrError) as ei:  # spheres not set
        R.matvec(b)
    assert ei.value.status == ESTATE
    with pytest.raises(ValueError):  # counts that do not add up to the points: caught before the call
        R.set_spheres(cen, rad, [surfs[0].n, surfs[1].n + 5], to_dev(x), to_dev(n), to_dev(w))
    R.set_spheres(cen, rad, [s.n for s in surfs], to_dev(x), to_dev(n), to_dev(w))
    with pytest.raises(P.SrError) as ei:
        R.set_operator(float("nan"), 1.0, True)
    assert ei.value.status == EINVAL
    rhs = R.rhs(workload.rigid_motion(np.random.default_rng(1)))
    with pytest.raises(P.SrError) as ei:  # three iterations cannot reach 1e-12
        B = P.binding
        xx = torch.zeros_like(rhs)
        B.sr_rigid_solve(R.r, rhs, xx, False, 1e-12, 3, 3)
    assert ei.value.status == ENOCONV
    assert torch.isfinite(xx).all() and xx.abs().max() > 0  # the last iterate is kept
    with pytest.raises(P.SrError) as ei:  # a point inside a sphere
        R.velocity(R.solve(rhs, tol=1e-6)[0], to_dev(np.array([[0.1, 0.0, 0.0]])))
    assert ei.value.status == EINVAL
    q, it, rr = R.solve(rhs, tol=1e-8)  # still usable
    assert rr <= 1e-8
    R.close()


def test_prolongation_rejects_wrong_spacing(P):
    hc, hf = 1 / 8, 1 / 16
    cen, rad, sc = workload.two_spheres(hc, 0.2)
    _, _, sf = workload.two_spheres(hf, 0.2)
    xc = np.concatenate([s.x for s in sc])
    nc = np.concatenate([s.normal for s in sc])
    xf = np.concatenate([s.x for s in sf])
    with pytest.raises(P.SrError) as ei:  # hc that is not the coarse points' spacing
        P.Prolongation(cen, rad, hc * 1.37, [s.n for s in sc], to_dev(xc), to_dev(nc), [s.n for s in sf], to_dev(xf))
    assert ei.value.status == EINVAL


def test_network_errors(P):
    import torch

    B = P.binding
    with pytest.raises(P.SrError) as ei:
        P.WarmStartNet(33, 10, 4)
    assert ei.value.status == EINVAL
    net = P.WarmStartNet(32, 10, 4)
    g = torch.tensor([0.05, 0.1], dtype=torch.float64, device="cuda")
    m = torch.zeros((2, 12), dtype=torch.float64, device="cuda")
    with pytest.raises(P.SrError) as ei:  # no parameters yet
        net.forward(g, m)
    assert ei.value.status == ESTATE
    with pytest.raises(P.SrError) as ei:
        net.set_options(passes=2)
    assert ei.value.status == EINVAL
    net.set_params(np.zeros(net.nparam, np.float32))
    y = torch.zeros((2, 10), dtype=torch.float64, device="cuda")
    bad = torch.tensor([0, 7], dtype=torch.int64, device="cuda")
    with pytest.raises(P.SrError) as ei:  # index outside the two resident rows
        net.train_step(g, m, y, 1e-3, idx=bad, batch=2)
    assert ei.value.status == EINVAL
    g5 = torch.full((5,), 0.1, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SrError) as ei:  # batch above max_batch
        net.forward(g5, torch.zeros((5, 12), dtype=torch.float64, device="cuda"))
    assert ei.value.status == EINVAL
    assert torch.isfinite(net.forward(g, m)).all()  # still usable
    net.close()


def test_sharp_parameter_errors(P):
    with pytest.raises(P.SrError) as ei:
        P.Evaluator(1 / 8, surface_sharp=True, sharp_rho=-1.0)
    assert ei.value.status == EINVAL
