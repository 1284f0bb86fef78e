"""Oracle of the warm-start network (TEST INFRASTRUCTURE ONLY): plain numpy FP64.

The network maps a gap g and the 12 rigid-motion parameters m (translation and rotation of the two
spheres) to the density at the coarse quadrature points.  The density solves a linear equation
whose right-hand side is linear in m, so the network is made exactly linear in m: four layers of
width 256 act on the gap alone, and the fourth is a 256 x 12 matrix C(g) contracted with m.

    gt = (ln g - g_mid) / g_half          (near contact the flow varies like log(gap))
    h1 = tanh(W1 gt + b1)                 W1 (W,1)
    h2 = tanh(W2 h1 + b2)                 W2 (W,W)
    h3 = tanh(W3 h2 + b3)                 W3 (W,W)
    a4 = W4 h3 + b4                       W4 (12W,W);  C[w,k] = a4[12 w + k]
    z  = C m                              (W)
    o  = Wh z                             Wh (P,W);  density q[p] = s[p] o[p]
    loss = mean over the batch and the P outputs of (o - y / s)^2

Adam: Kingma & Ba, ICLR 2015 (bias-corrected first and second moments).
Parameter order everywhere: W1, b1, W2, b2, W3, b3, W4, b4, Wh.
"""
from __future__ import annotations

import numpy as np

NMOT = 12
NAMES = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "Wh")


def shapes(width: int, nout: int):
    W = width
    return {"W1": (W, 1), "b1": (W,), "W2": (W, W), "b2": (W,), "W3": (W, W), "b3": (W,),
            "W4": (NMOT * W, W), "b4": (NMOT * W,), "Wh": (nout, W)}


def forward(p, g, m, g_mid, g_half):
    """p: dict of parameters; g (B,), m (B,12).  Returns (o (B,P), cache)."""
    gt = ((np.log(np.asarray(g, float)) - g_mid) / g_half)[:, None]
    h1 = np.tanh(gt @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    h3 = np.tanh(h2 @ p["W3"].T + p["b3"])
    a4 = h3 @ p["W4"].T + p["b4"]
    B, W = h3.shape
    C = a4.reshape(B, W, NMOT)
    z = np.einsum("nwk,nk->nw", C, np.asarray(m, float))
    o = z @ p["Wh"].T
    return o, dict(gt=gt, h1=h1, h2=h2, h3=h3, a4=a4, z=z, m=np.asarray(m, float))


def loss(o, t):
    """Mean squared error against standardized targets t = y / s."""
    return float(np.mean((o - t) ** 2))


def backward(p, cache, o, t):
    """Gradients of loss(o, t) with respect to every parameter (same keys as p)."""
    B, P = o.shape
    do = 2.0 * (o - t) / (B * P)
    z, m, h3, h2, h1, gt = cache["z"], cache["m"], cache["h3"], cache["h2"], cache["h1"], cache["gt"]
    gr = {}
    gr["Wh"] = do.T @ z
    dz = do @ p["Wh"]
    da4 = (dz[:, :, None] * m[:, None, :]).reshape(B, -1)
    gr["W4"] = da4.T @ h3
    gr["b4"] = da4.sum(0)
    dh3 = da4 @ p["W4"]
    d3 = dh3 * (1.0 - h3 ** 2)
    gr["W3"] = d3.T @ h2
    gr["b3"] = d3.sum(0)
    dh2 = d3 @ p["W3"]
    d2 = dh2 * (1.0 - h2 ** 2)
    gr["W2"] = d2.T @ h1
    gr["b2"] = d2.sum(0)
    dh1 = d2 @ p["W2"]
    d1 = dh1 * (1.0 - h1 ** 2)
    gr["W1"] = d1.T @ gt
    gr["b1"] = d1.sum(0)
    return gr


class Adam:
    """Adam with bias correction; state per parameter name."""

    def __init__(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.t = 0
        self.m = {}
        self.v = {}

    def step(self, p, gr, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        for k in NAMES:
            if k not in self.m:
                self.m[k] = np.zeros_like(p[k])
                self.v[k] = np.zeros_like(p[k])
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * gr[k]
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * gr[k] ** 2
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            p[k] = p[k] - lr * mh / (np.sqrt(vh) + self.eps)
        return p
