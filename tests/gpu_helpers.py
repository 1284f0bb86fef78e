"""Helpers shared by the GPU tests: move a workload to the device, run the library, compare."""
from __future__ import annotations

import numpy as np


def to_dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel_err(got, ref):
    """max_y |got - ref| / max_y |ref| with the Euclidean norm per target."""
    got = np.asarray(got).reshape(-1, 3)
    ref = np.asarray(ref).reshape(-1, 3)
    return float(np.linalg.norm(got - ref, axis=1).max() / max(np.linalg.norm(ref, axis=1).max(), 1e-300))


def gpu_eval(cfg, layers, precision, want_delta=False, idx=None, ev=None):
    """Evaluate cfg on the GPU; returns numpy (u, v[, ud, vd]) for the targets idx (default all)."""
    import torch

    import paper_2507_00156_amd as P

    s, t = cfg["surf"], cfg["targets"]
    own = ev is None
    if own:
        ev = P.Evaluator(cfg["h"], cfg["rho"], precision=precision)
        ev.set_surface(to_dev(s.x), to_dev(s.normal), to_dev(s.w))
        ev.set_density(P.SR_SL, to_dev(cfg["f"]))
        ev.set_density(P.SR_DL, to_dev(cfg["q"]))
    sel = slice(None) if idx is None else np.asarray(idx)
    res = ev.eval(layers, to_dev(t.y[sel]), to_dev(t.x0[sel]), to_dev(t.n0[sel]), to_dev(t.b[sel]),
                  to_dev(cfg["f0"][sel]), to_dev(cfg["q0"][sel]), want_delta=want_delta)
    torch.cuda.synchronize()
    out = tuple(None if r is None else r.cpu().numpy() for r in res)
    if own:
        ev.close()
    return out


def tree_mac_radius(cfg, precision, cutoff=6.0):
    """The radius the library's treecode MAC requires a cluster's box to lie beyond (the tree_theta
    entry of sr_params in include/stokesreg.h): the near radius on the FP64 path; on the mixed path
    the near radius widened by the reach of the single-precision pair test."""
    import numpy as np

    x = np.asarray(cfg["surf"].x, dtype=np.float64)
    rnear = cutoff * max(cfg["rho"]) * cfg["h"]
    if precision == 0:
        return rnear
    ext = max(0.5 * (float(x[:, d].max()) - float(x[:, d].min())) for d in range(3))
    return rnear * (1.0 + 1e-5) + 4.0 * 2.0 ** -24 * (2.0 * ext + rnear)
