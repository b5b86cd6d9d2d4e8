"""Pins of the calibrated forward model and preprocessing oracle (Sec. 4.1,
4.2) against computations it does not do itself: a time-domain convolution
by explicit loops, the round trip through the deconvolution, the bound of
the regularised filter, and an analytically shifted pulse."""
import math

import numpy as np
import pytest

from oracle import pressure as PR


def _dets_at(dist, xp=0.1, yp=-0.2):
    """Detectors at the given distances from the source, on different rays."""
    ang = np.linspace(0.3, 2.9, len(dist))
    return np.stack([xp + dist * np.cos(ang), yp + dist * np.sin(ang)], axis=1)


def test_forward_is_the_time_domain_sum():
    """Integer retarded shifts m_d (tau_d = m_d dt): p_k = s_d dt sum_j
    Au_j pcal[k - j + m_d], s_d = 2 pi c |x_d - x_p|, by explicit loops."""
    rng = np.random.default_rng(1)
    n_det, n_t, c, dt = 3, 16, 1.3, 0.05
    m = np.array([0, 3, 7])
    det = _dets_at(m * c * dt + 1e-15 * 0)
    Au = rng.standard_normal((n_det, n_t))
    pcal = np.zeros((n_det, n_t))
    for d in range(n_det):  # a pulse arriving at m_d
        pcal[d, m[d]:m[d] + 5] = rng.standard_normal(5)
    got = PR.pressure_forward(Au, pcal, det, 0.1, -0.2, c, dt)
    want = np.zeros((n_det, n_t))
    for d in range(n_det):
        s = 2 * math.pi * c * math.hypot(det[d, 0] - 0.1, det[d, 1] + 0.2)
        for k in range(n_t):
            acc = 0.0
            for j in range(n_t):
                i = k - j + m[d]
                if 0 <= i < n_t:
                    acc += Au[d, j] * pcal[d, i]
            want[d, k] = s * dt * acc
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_deconvolution_recovers_the_projection():
    """A minimum-phase pulse (decaying exponential, no spectral zero) arriving
    at m_d samples: with a vanishing eps, preprocess(pressure_forward(Au))
    gives Au back (up to the truncation of the n_t-sample window)."""
    rng = np.random.default_rng(2)
    n_det, n_t, c, dt = 4, 64, 1.0, 0.02
    m = np.array([2, 5, 9, 11])
    det = _dets_at(m * c * dt)
    Au = rng.standard_normal((n_det, n_t))
    k = np.arange(n_t)
    pcal = np.zeros((n_det, n_t))
    for d in range(n_det):
        pcal[d, m[d]:] = np.exp(-(k[:n_t - m[d]]) / 3.0)
    p = PR.pressure_forward(Au, pcal, det, 0.1, -0.2, c, dt)
    f = PR.preprocess(p, pcal, det, 0.1, -0.2, c, dt, eps=1e-24)
    assert np.max(np.abs(f - Au)) <= 1e-8 * np.max(np.abs(Au))


def test_regularised_filter_bound():
    """|conj(D) / (|D|^2 + eps)| <= 1 / (2 sqrt(eps)) at every frequency (so
    noise at zeros of the calibration spectrum is not amplified without
    bound); a pulse with a zero at DC ([1, -1]) passes no DC at all."""
    rng = np.random.default_rng(3)
    n_det, n_t, c, dt, eps = 2, 32, 1.0, 0.1, 1e-3
    det = _dets_at(np.array([0.5, 0.8]))
    pcal = np.zeros((n_det, n_t))
    pcal[:, 0], pcal[:, 1] = 1.0, -1.0
    p = rng.standard_normal((n_det, n_t)) + 3.0
    L = PR.fft_length(n_t)
    s = 2 * math.pi * c * np.hypot(det[:, 0] - 0.1, det[:, 1] + 0.2)
    f = PR.preprocess(p, pcal, det, 0.1, -0.2, c, dt, eps) * s[:, None]
    # f_t is the first n_t samples of a length-L signal whose spectrum is the
    # filtered one; rebuild that signal and check its spectrum bin by bin
    D = PR.calibration_spectra(pcal, det, 0.1, -0.2, c, dt, L)
    H = np.conj(D) / (np.abs(D) ** 2 + eps)
    assert np.all(np.abs(H) <= 1.0 / (2.0 * math.sqrt(eps)) * (1 + 1e-12))
    full = np.fft.ifft(np.fft.fft(p, n=L, axis=1) * H, axis=1)
    assert np.allclose(full.real[:, :n_t], f, rtol=0, atol=1e-12)
    assert np.max(np.abs(np.fft.fft(full, axis=1)[:, 0])) <= 1e-9


def test_fractional_retarded_shift():
    """A Gaussian pulse centred at t_c + tau (tau not a multiple of dt): the
    spectrum at retarded time, transformed back, is the same Gaussian centred
    at t_c (to the Gaussian's own band-limit error)."""
    n_t, c, dt = 128, 1.0, 0.01
    tau = np.array([0.123456, 0.31])
    det = _dets_at(tau * c)
    t = np.arange(n_t) * dt
    tc, w = 0.2, 3.3 * dt
    pcal = np.exp(-((t[None, :] - tc - tau[:, None]) ** 2) / (2 * w * w))
    L = PR.fft_length(n_t)
    D = PR.calibration_spectra(pcal, det, 0.1, -0.2, c, dt, L)
    back = np.fft.ifft(D, axis=1).real / dt
    want = np.exp(-((np.arange(L) * dt - tc) ** 2) / (2 * w * w))
    assert np.max(np.abs(back[:, :n_t // 2] - want[None, :n_t // 2])) <= 1e-9
