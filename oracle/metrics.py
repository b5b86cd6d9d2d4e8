"""Image quality measure of Sec. 5.4 (test infrastructure only)."""
from __future__ import annotations

import numpy as np


def psnr_as_printed(u_hat: np.ndarray, u_gt: np.ndarray) -> float:
    """10 log10(max(u_gt) / (||u_hat - u_gt||^2 / N)), with max not squared,
    as the formula is printed."""
    mse = np.sum((u_hat - u_gt) ** 2) / u_gt.size
    return float(10.0 * np.log10(np.max(u_gt) / mse))


def psnr(u_hat: np.ndarray, u_gt: np.ndarray) -> float:
    """Standard PSNR: 10 log10(max(u_gt)^2 / MSE)."""
    mse = np.sum((u_hat - u_gt) ** 2) / u_gt.size
    return float(10.0 * np.log10(np.max(u_gt) ** 2 / mse))
