"""Seeded draws for the warm-start network: initial parameters and (gap, motion) samples.

Only random draws live here; the network's arithmetic is elsewhere.
"""
from __future__ import annotations

import numpy as np

GAP_RANGE = (0.02, 0.2)


def mlp_init(width: int, nout: int, seed: int) -> dict:
    """Glorot-uniform weights U(-a, a), a = sqrt(6 / (fan_in + fan_out)), zero biases; FP64 arrays in the
    order W1, b1, W2, b2, W3, b3, W4 (12 width x width), b4, Wh (nout x width)."""
    rng = np.random.default_rng(seed)

    def glorot(fo, fi):
        a = np.sqrt(6.0 / (fi + fo))
        return rng.uniform(-a, a, size=(fo, fi))

    W = width
    return {"W1": glorot(W, 1), "b1": np.zeros(W), "W2": glorot(W, W), "b2": np.zeros(W),
            "W3": glorot(W, W), "b3": np.zeros(W), "W4": glorot(12 * W, W), "b4": np.zeros(12 * W),
            "Wh": glorot(nout, W)}


def warmstart_samples(n: int, seed: int, gap_range=GAP_RANGE):
    """n gaps uniform in gap_range and n motions (n, 2, 6) = (U, Omega) per sphere, N(0, 1)."""
    rng = np.random.default_rng(seed)
    gaps = rng.uniform(gap_range[0], gap_range[1], size=n)
    motions = rng.standard_normal((n, 2, 6))
    return gaps, motions


def warmstart_dataset(n_gaps: int, per_gap: int, seed: int, gap_range=GAP_RANGE):
    """n_gaps gaps uniform in gap_range, each with per_gap motions (n_gaps * per_gap, 2, 6) ~ N(0, 1);
    the gaps are repeated per_gap times in a row, so one geometry serves per_gap solves."""
    rng = np.random.default_rng(seed)
    gaps = rng.uniform(gap_range[0], gap_range[1], size=n_gaps)
    motions = rng.standard_normal((n_gaps * per_gap, 2, 6))
    return np.repeat(gaps, per_gap), motions
