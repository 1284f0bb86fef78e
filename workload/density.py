"""Smooth vector densities: each component is a combination of real solid harmonics r^l Y_lm of
degree <= L about the surface centre, with seeded N(0,1) coefficients."""
from __future__ import annotations

import numpy as np
from scipy.special import sph_harm_y


def harmonic_coeffs(L: int, rng: np.random.Generator) -> np.ndarray:
    """(3, (L+1)^2) N(0,1) coefficients, ordered (l, m) with m = -l..l."""
    return rng.standard_normal((3, (L + 1) ** 2))


def harmonic_field(coeffs: np.ndarray, x: np.ndarray, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Evaluate the vector field with the given coefficients at points x (K,3) -> (K,3)."""
    coeffs = np.asarray(coeffs, float)
    nb = coeffs.shape[1]
    L = int(round(np.sqrt(nb))) - 1
    assert (L + 1) ** 2 == nb
    p = np.asarray(x, float) - np.asarray(center, float)
    r = np.linalg.norm(p, axis=1)
    rs = np.where(r > 0, r, 1.0)
    polar = np.arccos(np.clip(p[:, 2] / rs, -1.0, 1.0))
    azim = np.arctan2(p[:, 1], p[:, 0])
    basis = np.empty((p.shape[0], nb))
    col = 0
    for l in range(L + 1):
        rl = r ** l
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), polar, azim)
            if m > 0:
                yr = np.sqrt(2.0) * (-1) ** m * Y.real
            elif m < 0:
                yr = np.sqrt(2.0) * (-1) ** m * Y.imag
            else:
                yr = Y.real
            basis[:, col] = rl * yr
            col += 1
    return basis @ coeffs.T
