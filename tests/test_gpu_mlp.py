"""Warm-start network and coarse-to-fine interpolation on the GPU, through the C ABI.

- BF16 matrix-core product vs an FP64 product: |C - C_ref| <= tol * (|A| |B|^T) elementwise with
  tol = 2^-8 (one pass: both operands rounded to BF16), 2^-15 (three passes: hi*hi + hi*lo + lo*hi)
  or 2^-25 (six passes: the whole FP32 operands, |lo| <= 2^-9 |x| and |lo2| <= 2^-18 |x|, so the
  dropped lo*lo2, lo2*lo, lo2*lo2 are below 2^-26 |a||b|) plus K 2^-23 for FP32 accumulation;
  ragged sizes and the head's shape;
- forward outputs and loss gradients vs the numpy FP64 oracle (ragged batch and output count);
- one Adam step vs the oracle's Adam applied to the kernel's own gradient;
- padding rows never leak: a batch of 7 gives the same gradient through idx as the rows themselves;
- coarse-to-fine interpolation vs the oracle's stencils, and its accuracy on a smooth field;
- the refined solve replaces a useless guess by zero.
"""
import numpy as np
import pytest

import workload

GMID, GHALF = np.log(0.02 * 0.2) / 2, np.log(0.2 / 0.02) / 2  # ln g over [0.02, 0.2] -> [-1, 1]
from oracle import mlp as omlp
from oracle.rigid import Sphere
from tests.gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2507_00156_amd as P

    P.load_library()
    return P


def flat(p):
    return np.concatenate([p[k].astype(np.float64).ravel() for k in omlp.NAMES])


def unflat(v, width, nout):
    out, o = {}, 0
    for k in omlp.NAMES:
        shp = omlp.shapes(width, nout)[k]
        n = int(np.prod(shp))
        out[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


@pytest.mark.parametrize("passes", [1, 3, 6])
@pytest.mark.parametrize("mnk", [(70, 100, 300), (1, 33, 5), (64, 2000, 256), (64, 256, 4100)])
def test_gemm_bound(P, passes, mnk):
    import torch

    m, n, k = mnk
    rng = np.random.default_rng(m * 7 + n + k)
    A = rng.standard_normal((m, k)).astype(np.float32)
    B = rng.standard_normal((n, k)).astype(np.float32)
    C = torch.empty((m, n), dtype=torch.float32, device="cuda")
    P.sr_mlp_gemm_test(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), C, passes=passes)
    ref = A.astype(np.float64) @ B.astype(np.float64).T
    S = np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64).T
    tol = {1: 2.0 ** -8, 3: 2.0 ** -15, 6: 2.0 ** -25}[passes] + k * 2.0 ** -23
    ratio = (np.abs(C.cpu().numpy() - ref) / S).max()
    print(f"gemm {mnk} passes={passes}: max |err| / (|A||B|) = {ratio:.3e} (bound {tol:.2e})", flush=True)
    assert ratio <= tol


def setup_net(P, width, nout, batch, passes=3, seed=3):
    import torch

    p = workload.mlp_init(width, nout, seed)
    rng = np.random.default_rng(seed + 1)
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = rng.standard_normal(p[k].shape) * 0.2
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}  # the values the GPU holds
    net = P.WarmStartNet(width, nout, max_batch=max(batch, 8), passes=passes)
    net.set_params(flat(p).astype(np.float32))
    g, m = workload.warmstart_samples(batch, seed + 2)
    y = rng.standard_normal((batch, nout)) * (1.0 + np.arange(nout) % 5)
    return net, p, g, m.reshape(batch, 12), y


@pytest.mark.parametrize("passes", [3, 1, 6])
def test_forward_matches_oracle(P, passes):
    width, nout, batch = 64, 301, 7
    net, p, g, m, _ = setup_net(P, width, nout, batch, passes)
    o = net.forward(to_dev(g), to_dev(m)).cpu().numpy()
    ref = omlp.forward(p, g, m, GMID, GHALF)[0]
    e = np.abs(o - ref).max() / np.abs(ref).max()
    print(f"forward passes={passes}: {e:.3e}", flush=True)
    assert e <= {3: 1e-4, 1: 2e-2, 6: 2e-6}[passes]
    net.close()


def test_gradients_match_oracle(P):
    import torch

    width, nout, batch = 64, 301, 7
    net, p, g, m, y = setup_net(P, width, nout, batch, 3)
    yd = to_dev(y)
    net.fit_output_scale(yd)
    s = net.output_scale().cpu().numpy()
    np.testing.assert_allclose(s, np.sqrt((y ** 2).mean(0)), rtol=1e-14)
    grad, loss = net.gradients(to_dev(g), to_dev(m), yd)
    o, cache = omlp.forward(p, g, m, GMID, GHALF)
    t = y / s
    gr = omlp.backward(p, cache, o, t)
    assert abs(loss - omlp.loss(o, t)) <= 1e-5 * omlp.loss(o, t)
    gg = unflat(grad.cpu().numpy(), width, nout)
    for k in omlp.NAMES:
        e = np.linalg.norm(gg[k] - gr[k]) / max(np.linalg.norm(gr[k]), 1e-30)
        print(f"grad {k}: {e:.2e}", flush=True)
        assert e <= 1e-3, k
    # rows chosen by idx from a larger resident set give the same gradient as the rows themselves
    big = np.concatenate([np.zeros((5, 12)), m]), np.concatenate([np.full(5, 0.07), g])
    ybig = np.concatenate([np.zeros((5, nout)), y])
    idx = torch.arange(5, 5 + batch, dtype=torch.int64, device="cuda")
    grad2, loss2 = net.gradients(to_dev(big[1]), to_dev(big[0]), to_dev(ybig), idx=idx, batch=batch)
    assert torch.equal(grad, grad2) and loss == loss2
    net.close()


def test_adam_step_matches_oracle(P):
    width, nout, batch = 64, 301, 7
    net, p, g, m, y = setup_net(P, width, nout, batch, 3)
    yd = to_dev(y)
    net.fit_output_scale(yd)
    grad, _ = net.gradients(to_dev(g), to_dev(m), yd)
    lr = 3e-3
    net.train_step(to_dev(g), to_dev(m), yd, lr)
    after = net.get_params().astype(np.float64)
    opt = omlp.Adam(lr=lr)
    ref = opt.step({k: v.copy() for k, v in p.items()}, unflat(grad.cpu().numpy(), width, nout))
    d = np.abs(after - flat(ref)).max()
    print(f"adam step: max |theta_gpu - theta_ref| = {d:.2e} (lr {lr})", flush=True)
    assert d <= 1e-3 * lr + 1e-6
    net.close()


def test_training_reduces_loss(P):
    import torch

    width, nout, n = 64, 400, 256
    rng = np.random.default_rng(11)
    g, m = workload.warmstart_samples(n, 12)
    m = m.reshape(n, 12)
    A = rng.standard_normal((12, nout))
    Bc = rng.standard_normal((12, nout)) * 0.05
    y = np.einsum("nk,nkp->np", m, A[None] + Bc[None] / (g[:, None, None] + 0.02))
    net = P.WarmStartNet(width, nout, max_batch=32, passes=3)
    net.set_params(flat(workload.mlp_init(width, nout, 4)).astype(np.float32))
    gd, md, yd = to_dev(g), to_dev(m), to_dev(y)
    net.fit_output_scale(yd)
    losses = []
    for it in range(400):
        idx = torch.from_numpy(rng.integers(0, n, 32)).cuda()
        losses.append(net.train_step(gd, md, yd, 2e-3, idx=idx, batch=32))
    print(f"training: loss {losses[0]:.3e} -> {losses[-1]:.3e}", flush=True)
    assert losses[-1] <= 0.05 * losses[0]
    net.close()


def test_prolongation_matches_oracle_stencils(P):
    hc, hf = 1 / 16, 1 / 32
    cen, rad, sc = workload.two_spheres(hc, 0.1)
    _, _, sf = workload.two_spheres(hf, 0.1)
    xc = np.concatenate([s.x for s in sc])
    nc = np.concatenate([s.normal for s in sc])
    xf = np.concatenate([s.x for s in sf])
    pr = P.Prolongation(cen, rad, hc, [s.n for s in sc], to_dev(xc), to_dev(nc), [s.n for s in sf], to_dev(xf))

    def field(x):
        return np.stack([np.sin(1.3 * x[:, 0] + 0.4 * x[:, 1]), np.cos(x[:, 2] - 0.7 * x[:, 0]),
                         np.exp(0.5 * x[:, 1]) * x[:, 2]], axis=1)

    qc = field(xc)
    got = pr(to_dev(qc)).cpu().numpy()
    ref = []
    off = 0
    for s, c, a in zip(sc, cen, rad):
        sp = Sphere(s, c, a, hc)
        fpts = sf[len(ref)].x
        x0, _, _ = sp.closest(fpts)
        idx, wts = sp.stencils(x0)
        ref.append(np.einsum("ks,ksc->kc", wts, qc[off:off + s.n][idx]))
        off += s.n
    ref = np.concatenate(ref)
    d = np.abs(got - ref).max()
    acc = np.abs(got - field(xf)).max()
    print(f"prolongation: vs oracle stencils {d:.2e}, vs the field {acc:.2e}", flush=True)
    assert d <= 1e-13 and acc <= 1e-3
    pr.close()


def test_refined_solve_rejects_useless_guess(P):
    import torch

    h, gap = 1 / 12, 0.2
    cen, rad, surfs = workload.two_spheres(h, gap)
    x = np.concatenate([s.x for s in surfs])
    n = np.concatenate([s.normal for s in surfs])
    w = np.concatenate([s.w for s in surfs])
    R = P.RigidSpheres(h, precision=1)
    R.set_spheres(cen, rad, [s.n for s in surfs], to_dev(x), to_dev(n), to_dev(w))
    b = R.rhs(workload.rigid_motion(np.random.default_rng(8)))
    q0, it0, no0, rr0 = R.solve_refined(b, tol=1e-8)
    bad = torch.full_like(b, 1e6)
    q1, it1, no1, rr1 = R.solve_refined(b, x0=bad, tol=1e-8)
    nanguess = torch.full_like(b, float("nan"))
    q2, it2, no2, rr2 = R.solve_refined(b, x0=nanguess, tol=1e-8)
    print(f"zero start {it0}/{no0}, bad guess {it1}/{no1}, NaN guess {it2}/{no2}", flush=True)
    assert rr1 <= 1e-8 and rr2 <= 1e-8 and it1 == it0 and it2 == it0
    assert torch.equal(q0, q1) and torch.equal(q0, q2)
    R.close()


def test_real_head_shape_matches_oracle(P):
    """The network at its real shape: width 256, 102420 outputs (the two h = 1/32 spheres' unknowns),
    batch 64.  The head's backward product dz = dout Wh then contracts over 102420 outputs and takes the
    explicit K split of the GEMM (200 partial products summed in a fixed order) that the small shapes
    above never reach.  Forward, every gradient block and one Adam step against the FP64 oracle."""
    width, nout, batch = 256, 102420, 64
    net, p, g, m, y = setup_net(P, width, nout, batch, 3, seed=21)
    yd = to_dev(y)
    net.fit_output_scale(yd)
    s = net.output_scale().cpu().numpy()
    o_gpu = net.forward(to_dev(g), to_dev(m)).cpu().numpy()
    o, cache = omlp.forward(p, g, m, GMID, GHALF)
    e = np.abs(o_gpu - o).max() / np.abs(o).max()
    print(f"real shape forward: {e:.3e}", flush=True)
    assert e <= 1e-4
    grad, loss = net.gradients(to_dev(g), to_dev(m), yd)
    t = y / s
    gr = omlp.backward(p, cache, o, t)
    assert abs(loss - omlp.loss(o, t)) <= 1e-5 * omlp.loss(o, t)
    gg = unflat(grad.cpu().numpy(), width, nout)
    for k in omlp.NAMES:
        e = np.linalg.norm(gg[k] - gr[k]) / max(np.linalg.norm(gr[k]), 1e-30)
        print(f"real shape grad {k}: {e:.2e}", flush=True)
        assert e <= 1e-3, k
    lr = 1e-3
    net.train_step(to_dev(g), to_dev(m), yd, lr)
    after = net.get_params().astype(np.float64)
    ref = omlp.Adam(lr=lr).step({k: v.copy() for k, v in p.items()}, gg)
    d = np.abs(after - flat(ref)).max()
    print(f"real shape adam step: {d:.2e}", flush=True)
    assert d <= 1e-3 * lr + 1e-6
    net.close()


def test_switch_to_six_products_after_set_params(P):
    """The weights' third BF16 pieces are written only in the six-product mode: switching to it after
    the parameters are set must rebuild them (same outputs as a network made in that mode)."""
    width, nout, batch = 64, 301, 7
    net_a, p, g, m, _ = setup_net(P, width, nout, batch, 6)
    net_b, _, _, _, _ = setup_net(P, width, nout, batch, 3)
    net_b.set_options(passes=6, g_mid=GMID, g_half=GHALF)
    oa = net_a.forward(to_dev(g), to_dev(m)).cpu().numpy()
    ob = net_b.forward(to_dev(g), to_dev(m)).cpu().numpy()
    assert np.array_equal(oa, ob)
    ref = omlp.forward(p, g, m, GMID, GHALF)[0]
    assert np.abs(ob - ref).max() / np.abs(ref).max() <= 2e-6
    net_a.close()
    net_b.close()
