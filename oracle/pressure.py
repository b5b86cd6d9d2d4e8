"""Calibrated forward model and preprocessing (Sec. 4.1 eq. FW_full, Sec. 4.2
eqs. FW_conv, f_rewrite, conv_thm2, deconv), float64.

Test infrastructure only (see the package docstring).

The measured pressure at detector x_d is the time convolution of the
circular projection of the image with the calibration measurement p_cal of
a point source at x_p, taken at the retarded time t' = t - |x_d - x_p| / c
and scaled by |x_d - x_p| / t:

  p = (|x_d - x_p| / t) (K u)  *_t  p_cal(x_d, t').

K is the circular integral; the operator A of this build is the circular
mean, K u = 2 pi c t (A u) on the circle of radius c t, so (1 / t) K u =
2 pi c A u and

  p_d = s_d (A u)_d *_t pcal_d(. + tau_d),  s_d = 2 pi c |x_d - x_p|,
  tau_d = |x_d - x_p| / c.

The convolution of sampled signals is the Riemann sum dt sum_j a_j b_{k-j}.
Preprocessing inverts it with the regularised filter of eq. deconv,

  f_t = F^-1{ F{p} conj(D) / (|D|^2 + eps) },  D = F{pcal(. + tau_d)} dt,

and f = f_t / s_d (eq. f_rewrite), which is A u again when the filter
inverts D. Transforms are discrete Fourier transforms of length L >= 2 n_t
(zero padding), so the convolution of the n_t-sample window is linear up to
what lies beyond L; the retarded shift is applied as the phase ramp
exp(i omega tau_d), omega the angular frequencies of the L-point transform
(a circular, band-limited shift: the part of the pulse before t' = 0 wraps to
the end of the buffer, i.e. to negative lags).
"""
from __future__ import annotations

import math

import numpy as np


def fft_length(n_t: int) -> int:
    """Smallest power of two >= 2 n_t."""
    L = 1
    while L < 2 * n_t:
        L *= 2
    return L


def omegas(L: int, dt: float) -> np.ndarray:
    """Angular frequencies of the L-point DFT bins (negative above L/2)."""
    return 2.0 * math.pi * np.fft.fftfreq(L, d=dt)


def source_distances(det_xy: np.ndarray, xp: float, yp: float) -> np.ndarray:
    return np.hypot(det_xy[:, 0] - xp, det_xy[:, 1] - yp)


def calibration_spectra(pcal: np.ndarray, det_xy: np.ndarray, xp: float, yp: float, c: float,
                        dt: float, L: int) -> np.ndarray:
    """D_d = dt F{pcal_d} exp(i omega tau_d): the spectrum of the calibration
    trace at retarded time (pulse moved to t' = 0), per detector [n_det][L]."""
    tau = source_distances(det_xy, xp, yp) / c
    P = np.fft.fft(pcal, n=L, axis=1)
    return dt * P * np.exp(1j * omegas(L, dt)[None, :] * tau[:, None])


def pressure_forward(Au: np.ndarray, pcal: np.ndarray, det_xy: np.ndarray, xp: float, yp: float,
                     c: float, dt: float) -> np.ndarray:
    """Eq. FW_full on the samples: Au [n_det][n_t] (the circular means),
    pcal [n_det][n_t] -> pressure [n_det][n_t]."""
    n_det, n_t = Au.shape
    L = fft_length(n_t)
    D = calibration_spectra(pcal, det_xy, xp, yp, c, dt, L)
    s = 2.0 * math.pi * c * source_distances(det_xy, xp, yp)
    y = np.fft.ifft(np.fft.fft(Au, n=L, axis=1) * D, axis=1).real[:, :n_t]
    return s[:, None] * y


def preprocess(p: np.ndarray, pcal: np.ndarray, det_xy: np.ndarray, xp: float, yp: float, c: float,
               dt: float, eps: float) -> np.ndarray:
    """Eqs. deconv and f_rewrite: regularised deconvolution of the measured
    pressure by the calibration spectrum, then division by s_d -> data f
    [n_det][n_t] in the units of A u."""
    n_det, n_t = p.shape
    L = fft_length(n_t)
    D = calibration_spectra(pcal, det_xy, xp, yp, c, dt, L)
    H = np.conj(D) / (np.abs(D) ** 2 + eps)
    ft = np.fft.ifft(np.fft.fft(p, n=L, axis=1) * H, axis=1).real[:, :n_t]
    s = 2.0 * math.pi * c * source_distances(det_xy, xp, yp)
    return ft / s[:, None]
