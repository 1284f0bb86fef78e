"""Pins of the oracle treecode (paper section 3.4) against the oracle's direct sums.

- theta = 0 never accepts a cluster: every leaf is summed directly, so the treecode must reproduce
  the direct extrapolated sums to rounding;
- barycentric interpolation at Chebyshev points converges geometrically in p for well-separated
  clusters: the error against the direct sum must fall by a large factor per step p -> p + 2;
- a larger theta accepts more clusters: the error at theta = 0.9 exceeds the one at theta = 0.3
  (at this coarse h the near-radius condition dominates between 0.5 and 0.9).
"""
import numpy as np
import pytest

import oracle
import workload


@pytest.fixture(scope="module")
def small():
    cfg = workload.build_config("small")
    idx = np.arange(0, cfg["targets"].m, 17)
    return cfg, idx, oracle.sl_cfg(cfg, idx), oracle.dl_cfg(cfg, idx)


def _err(a, b):
    return np.linalg.norm(a - b, axis=1).max() / np.linalg.norm(b, axis=1).max()


def test_theta_zero_reproduces_direct(small):
    cfg, idx, u, v = small
    tu, tv = oracle.tree_cfg(cfg, idx, p=4, theta=0.0, leaf=150)
    assert _err(tu, u) < 1e-12 and _err(tv, v) < 1e-12


def test_error_decays_with_degree(small):
    cfg, idx, u, v = small
    errs = []
    for p in (4, 6, 8):
        tu, tv = oracle.tree_cfg(cfg, idx, p=p, theta=0.7, leaf=200)
        errs.append((_err(tu, u), _err(tv, v)))
    for k in range(2):
        assert errs[k + 1][0] < errs[k][0] / 10 and errs[k + 1][1] < errs[k][1] / 10
    assert errs[-1][0] < 1e-8 and errs[-1][1] < 1e-7


def test_larger_theta_larger_error(small):
    cfg, idx, u, v = small
    e5 = _err(oracle.tree_cfg(cfg, idx, p=4, theta=0.3, leaf=100)[0], u)
    e9 = _err(oracle.tree_cfg(cfg, idx, p=4, theta=0.9, leaf=100)[0], u)
    assert e9 > e5


def test_single_leaf_is_direct(small):
    # leaf size >= N: the root is a leaf and is never accepted (targets lie on or near the surface)
    cfg, idx, u, v = small
    tu, tv = oracle.tree_cfg(cfg, idx, p=3, theta=0.7, leaf=10 ** 7)
    assert _err(tu, u) < 1e-12 and _err(tv, v) < 1e-12


def test_mac_radius_beyond_the_surface_is_direct(small):
    """A MAC radius larger than the surface's diameter accepts no cluster, whatever theta: the treecode
    is then the direct sum; a radius between the two moves only some clusters to the leaf sums, so the
    error lies between the paper's MAC's and zero."""
    cfg, idx, u, v = small
    x = cfg["surf"].x
    diam = float(np.linalg.norm(x.max(0) - x.min(0)))
    tu, tv = oracle.tree_cfg(cfg, idx, p=4, theta=0.9, leaf=100, mac_rnear=2.0 * diam)
    assert _err(tu, u) < 1e-12 and _err(tv, v) < 1e-12
    rnear = 6.0 * max(cfg["rho"]) * cfg["h"]
    e_paper = _err(oracle.tree_cfg(cfg, idx, p=4, theta=0.9, leaf=100)[0], u)
    e_wide = _err(oracle.tree_cfg(cfg, idx, p=4, theta=0.9, leaf=100, mac_rnear=2.0 * rnear)[0], u)
    assert e_wide < e_paper
