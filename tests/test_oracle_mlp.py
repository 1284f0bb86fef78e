"""Pins of the warm-start network oracle (oracle/mlp.py).

- analytic gradients vs central finite differences of the FP64 loss (every parameter block);
- the output is exactly linear in the motion parameters and independent of them through the gap
  branch (the structure the network is built to have);
- Adam under a constant gradient moves every parameter by lr * g / (|g| + eps) per step (m_hat = g,
  v_hat = g^2 after bias correction);
- zero head weights give the loss mean(t^2).
"""
import numpy as np
import pytest

import workload

GMID, GHALF = np.log(0.02 * 0.2) / 2, np.log(0.2 / 0.02) / 2  # ln g over [0.02, 0.2] -> [-1, 1]
from oracle import mlp


def tiny(width=6, nout=5, seed=1):
    p = workload.mlp_init(width, nout, seed)
    rng = np.random.default_rng(seed + 1)
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = rng.standard_normal(p[k].shape) * 0.3
    g, m = workload.warmstart_samples(4, seed + 2)
    return p, g, m.reshape(4, 12), rng.standard_normal((4, nout))


@pytest.mark.parametrize("name", mlp.NAMES)
def test_gradient_matches_finite_differences(name):
    p, g, m, t = tiny()
    o, cache = mlp.forward(p, g, m, GMID, GHALF)
    gr = mlp.backward(p, cache, o, t)
    rng = np.random.default_rng(5)
    flat = p[name].reshape(-1)
    idx = rng.choice(flat.size, size=min(8, flat.size), replace=False)
    eps = 1e-6
    for i in idx:
        old = flat[i]
        flat[i] = old + eps
        lp = mlp.loss(mlp.forward(p, g, m, GMID, GHALF)[0], t)
        flat[i] = old - eps
        lm = mlp.loss(mlp.forward(p, g, m, GMID, GHALF)[0], t)
        flat[i] = old
        fd = (lp - lm) / (2 * eps)
        an = gr[name].reshape(-1)[i]
        assert abs(fd - an) <= 1e-8 + 1e-6 * abs(fd), (name, i, fd, an)


def test_output_is_linear_in_motion():
    p, g, m, _ = tiny()
    rng = np.random.default_rng(9)
    m2 = rng.standard_normal(m.shape)
    a, b = 0.7, -1.9
    o1 = mlp.forward(p, g, m, GMID, GHALF)[0]
    o2 = mlp.forward(p, g, m2, GMID, GHALF)[0]
    o3 = mlp.forward(p, g, a * m + b * m2, GMID, GHALF)[0]
    np.testing.assert_allclose(o3, a * o1 + b * o2, rtol=1e-12, atol=1e-12)
    assert np.abs(mlp.forward(p, g, 0 * m, GMID, GHALF)[0]).max() == 0.0


def test_adam_constant_gradient_closed_form():
    rng = np.random.default_rng(2)
    p = {k: rng.standard_normal((3, 2)) for k in mlp.NAMES}
    gr = {k: rng.standard_normal((3, 2)) for k in mlp.NAMES}
    p0 = {k: v.copy() for k, v in p.items()}
    opt = mlp.Adam(lr=0.01, eps=1e-8)
    steps = 7
    for _ in range(steps):
        opt.step(p, gr)
    for k in mlp.NAMES:
        ex = p0[k] - steps * 0.01 * gr[k] / (np.abs(gr[k]) + 1e-8)
        np.testing.assert_allclose(p[k], ex, rtol=0, atol=1e-13)


def test_zero_head_loss():
    p, g, m, t = tiny()
    p["Wh"][:] = 0.0
    o = mlp.forward(p, g, m, GMID, GHALF)[0]
    assert mlp.loss(o, t) == pytest.approx(np.mean(t ** 2), rel=1e-15)
