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


def warmstart_unit_dataset(n_gaps: int, seed: int, gap_range=GAP_RANGE, spacing: str = "random",
                           ends: bool = False):
    """n_gaps gaps in gap_range, each with the 12 unit rigid motions (one per parameter), so the
    solutions at one gap are the 12 columns of the solution map at that gap: (n_gaps * 12,) gaps and
    (n_gaps * 12, 2, 6) motions, the gaps repeated 12 times in a row.  spacing "random": uniform draws;
    "log": the midpoints of n_gaps equal intervals of log(gap) (even cover of the network's input).
    ends: the first two gaps are the ends of gap_range (the rest as drawn)."""
    rng = np.random.default_rng(seed)
    if spacing == "log":
        lo, hi = np.log(gap_range[0]), np.log(gap_range[1])
        gaps = np.exp(lo + (np.arange(n_gaps) + 0.5) / n_gaps * (hi - lo))
    else:
        gaps = rng.uniform(gap_range[0], gap_range[1], size=n_gaps)
    if ends and n_gaps >= 2:
        gaps[0], gaps[1] = gap_range[0], gap_range[1]
    motions = np.tile(np.eye(12).reshape(12, 2, 6), (n_gaps, 1, 1))
    return np.repeat(gaps, 12), motions
