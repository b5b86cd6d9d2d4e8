"""Closed-form results used to pin the oracle (independent of its code).

Each function is textbook mathematics, not a retyping of an oracle formula:

* circle-circle intersection: the fraction of a circle of radius r about a
  detector at distance rho from a disc centre that lies inside a disc of
  radius R is alpha/pi with cos(alpha) = (r^2 + rho^2 - R^2) / (2 r rho);
* the circular mean of an isotropic Gaussian exp(-|x-c|^2 / 2 s^2) over a
  circle of radius r about a point at distance rho from c is
  exp(-(r^2 + rho^2)/2s^2) I0(r rho / s^2) (Bessel I0 from its integral form);
* the eigenvalues of the Neumann forward-difference Laplacian in 1-D are
  4 sin^2(pi k / 2n), k = 0..n-1.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def disc_circular_mean(r, rho, R):
    """Mean of the indicator of a disc (radius R) over circles of radius r whose
    centre lies at distance rho from the disc centre."""
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros_like(r)
    inside = r <= R - rho                      # circle entirely inside the disc
    out[inside] = 1.0
    cut = (r > abs(R - rho)) & (r < R + rho)
    rc = r[cut]
    cosa = (rc * rc + rho * rho - R * R) / (2.0 * rc * rho)
    out[cut] = np.arccos(np.clip(cosa, -1.0, 1.0)) / np.pi
    return out


def gaussian_circular_mean(r, rho, s):
    """Mean of exp(-|x - c|^2 / 2 s^2) over circles of radius r centred at
    distance rho from c."""
    r = np.asarray(r, dtype=np.float64)
    z = r * rho / (s * s)
    return np.exp(-(r - rho) ** 2 / (2 * s * s)) * special.i0e(z)


def grad_norm_squared(nx: int, ny: int) -> float:
    """||grad||^2 for unit-spacing forward differences with Neumann boundary."""
    return 4.0 * np.cos(np.pi / (2 * nx)) ** 2 + 4.0 * np.cos(np.pi / (2 * ny)) ** 2


def textbook_divergence(px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """Discrete divergence of Chambolle (2004), written out with loops:
    (div p)_i = p_i [i < n-1] - p_{i-1} [i > 0] in each direction."""
    ny, nx = px.shape
    out = np.zeros((ny, nx))
    for j in range(ny):
        for i in range(nx):
            a = px[j, i] if i < nx - 1 else 0.0
            b = px[j, i - 1] if i > 0 else 0.0
            c = py[j, i] if j < ny - 1 else 0.0
            d = py[j - 1, i] if j > 0 else 0.0
            out[j, i] = (a - b) + (c - d)
    return out
