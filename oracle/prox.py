"""Proximal maps of Sec. 3.2, float64 (test infrastructure only).

Dual vectors of the regulariser blocks are stored as (c, N) arrays: c rows per
pixel (2 for grad / D grad, 4 for the symmetrised gradient), N pixels.
"""
from __future__ import annotations

import numpy as np


def prox_f1_conj(z: np.ndarray, f: np.ndarray, gamma) -> np.ndarray:
    """prox of gamma F1*, F1 = 1/2 ||. - f||^2: (z - gamma f) / (1 + gamma).

    gamma may be a scalar or an array of per-bin step sizes.
    """
    return (z - gamma * f) / (1.0 + gamma)


def project_ball(z: np.ndarray, radius: float) -> np.ndarray:
    """prox of the indicator of {|z_p|_2 <= radius pointwise}, i.e. the prox of
    gamma F2* (and F3*) for F2 = radius * ||.||_1 with the pointwise 2-norm:
    radius * z / max(radius, |z|_2), independent of gamma."""
    nrm = np.sqrt(np.sum(z * z, axis=0))
    return z * (radius / np.maximum(radius, nrm))


def prox_zero(x: np.ndarray, gamma=None) -> np.ndarray:
    """prox of gamma G for G = 0: the identity."""
    return x


def prox_tikhonov(x: np.ndarray, gamma, alpha: float) -> np.ndarray:
    """prox of gamma G for G = alpha/2 ||.||^2: x / (1 + gamma alpha)."""
    return x / (1.0 + gamma * alpha)
