"""Host-side pieces of the warm-start pipeline (no GPU): the principal-direction decoder, the
least-squares output layers and the log(gap) interpolation control, each against a fact fixed
independently of it.

- PodDecoder: on data of known rank k it keeps exactly k orthonormal directions and reconstructs the
  data to rounding; on data with a known singular spectrum it keeps the modes whose tail energy
  exceeds the threshold;
- fit_readout: the parameters it writes, run through a plain FP64 forward pass of the network
  (written here from the layer definitions), reproduce the ridge fit it reports; with a trunk whose
  features span the targets exactly the fit is exact;
- BasisInterpolator: a map from motion to values that is a polynomial of degree <= 4 in log(gap) is
  reproduced exactly between the training gaps.
"""
import numpy as np
import pytest
import torch

from paper_2507_00156_amd import warmstart as W


def test_pod_decoder_rank_and_reconstruction():
    rng = np.random.default_rng(3)
    n, P, k = 60, 500, 7
    Y = torch.as_tensor(rng.standard_normal((n, k)) @ rng.standard_normal((k, P)))
    pod = W.PodDecoder(Y, rel=1e-9)
    assert pod.r == k
    V = pod.V
    assert torch.allclose(V.T @ V, torch.eye(k, dtype=V.dtype), atol=1e-12)
    Yr = pod.encode(Y) @ V.T
    assert ((Yr - Y).norm() / Y.norm()).item() < 1e-12


def test_pod_decoder_truncates_by_energy():
    rng = np.random.default_rng(4)
    n, P = 40, 300
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Vt, _ = np.linalg.qr(rng.standard_normal((P, n)))
    sv = 10.0 ** -np.arange(n, dtype=float)  # energies 1, 1e-2, 1e-4, ...
    Y = torch.as_tensor((U * sv) @ Vt.T)
    # the energy beyond the first r modes is ~ sv[r]^2 (1 + 1e-2 + ...); rel = 3e-4 -> rel^2 = 9e-8
    # keeps modes up to sv = 1e-3 (tail ~1e-8 < 9e-8) and no fewer (tail beyond 3 modes ~1e-6)
    pod = W.PodDecoder(Y, rel=3e-4)
    assert pod.r == 4


class _HostNet:
    """Stand-in for WarmStartNet with the attributes fit_readout uses (host parameter vector)."""

    def __init__(self, width, nout, seed=0):
        self.width, self.nout, self.g_mid, self.g_half = width, nout, -2.760730458931123, 1.151292546497023
        rng = np.random.default_rng(seed)
        self.p = np.concatenate([rng.standard_normal(int(np.prod(sh))) * 0.3
                                 for _, sh in W._blocks(width, nout)]).astype(np.float32)
        self.scale = None

    def get_params(self):
        return self.p.copy()

    def set_params(self, f):
        self.p = np.asarray(f, np.float32)

    def set_output_scale(self, s):
        self.scale = s


def _forward(net, gaps, motions):
    """The network of the header's definition, FP64: tanh layers on the normalized log gap, C(g) m, Wh."""
    W_, P = net.width, net.nout
    flat, p, off = net.p.astype(np.float64), {}, 0
    for name, shp in W._blocks(W_, P):
        k = int(np.prod(shp))
        p[name] = flat[off:off + k].reshape(shp)
        off += k
    gt = ((np.log(gaps) - net.g_mid) / net.g_half)[:, None]
    h = np.tanh(np.tanh(np.tanh(gt @ p["W1"].T + p["b1"]) @ p["W2"].T + p["b2"]) @ p["W3"].T + p["b3"])
    C = (h @ p["W4"].T + p["b4"]).reshape(len(gaps), W_, 12)
    return np.einsum("nwk,nk->nw", C, motions) @ p["Wh"].T


@pytest.mark.parametrize("lam", [1e-3, 1e-8])
def test_fit_readout_writes_the_ridge_fit(lam):
    width, P, ng = 32, 5, 20
    net = _HostNet(width, P)
    rng = np.random.default_rng(1)
    g = np.sort(rng.uniform(0.02, 0.2, ng))
    gaps = np.repeat(g, 12)
    motions = np.tile(np.eye(12), (ng, 1))
    lg = np.log(g)
    T = np.stack([np.stack([np.sin((k + 1) * lg + q) for q in range(P)], 1) for k in range(12)], 1).reshape(ng * 12, P)
    scale = np.full(P, 2.0)
    _, _, fit_rms = W.fit_readout(net, gaps, T, scale, lambdas=[lam])
    o = _forward(net, gaps, motions)
    rms = np.sqrt(np.mean((o - T / 2.0) ** 2))
    assert abs(rms - fit_rms) <= 1e-6 * max(fit_rms, 1e-300) + 1e-12
    # linear in the motion: a combination of unit motions gives the same combination of outputs
    m = rng.standard_normal((3, 12))
    o3 = _forward(net, g[:3], m)
    ou = _forward(net, np.repeat(g[:3], 12), np.tile(np.eye(12), (3, 1))).reshape(3, 12, P)
    assert np.abs(o3 - np.einsum("nk,nkp->np", m, ou)).max() <= 1e-10 * np.abs(ou).max() * np.abs(m).sum(1).max()


def test_fit_readout_exact_when_targets_are_in_the_feature_span():
    width, P, ng = 32, 3, 24
    net = _HostNet(width, P, seed=2)
    rng = np.random.default_rng(5)
    g = np.sort(rng.uniform(0.02, 0.2, ng))
    gaps = np.repeat(g, 12)
    # targets = fixed linear maps of the trunk's own features (plus a constant): exactly representable
    probe = _HostNet(width, width, seed=2)
    flat, p, off = probe.p.astype(np.float64), {}, 0
    for name, shp in W._blocks(width, width):
        k = int(np.prod(shp))
        p[name] = flat[off:off + k].reshape(shp)
        off += k
    gt = ((np.log(g) - net.g_mid) / net.g_half)[:, None]
    h = np.tanh(np.tanh(np.tanh(gt @ p["W1"].T + p["b1"]) @ p["W2"].T + p["b2"]) @ p["W3"].T + p["b3"])
    A = rng.standard_normal((12, P, width)) * 0.1
    T = (np.einsum("kpw,nw->nkp", A, h) + 0.3).reshape(ng * 12, P)
    _, _, fit_rms = W.fit_readout(net, gaps, T, np.ones(P), lambdas=[1e-14])
    assert fit_rms <= 1e-8


def test_basis_interpolator_exact_for_quartic_in_log_gap():
    rng = np.random.default_rng(9)
    ng, P = 30, 40
    g = np.sort(rng.uniform(0.02, 0.2, ng))
    coef = rng.standard_normal((5, 12, P))

    def Q(gap):
        x = np.log(gap)
        return sum(coef[d] * x ** d for d in range(5))  # (12, P)

    Y = torch.as_tensor(np.concatenate([Q(x) for x in g]).reshape(ng * 12, P))
    interp = W.BasisInterpolator(np.repeat(g, 12), Y, k=8, deg=4)
    for gap in (0.031, 0.077, 0.15):
        m = rng.standard_normal(12)
        got = interp(gap, m).numpy()
        ex = m @ Q(gap)
        assert np.abs(got - ex).max() <= 1e-9 * np.abs(ex).max()
