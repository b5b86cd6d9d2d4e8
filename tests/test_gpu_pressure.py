"""Calibrated pressure model and preprocessing (Sec. 4.1, 4.2) through the C
ABI against the oracle: the forward model of measured pressure, the
regularised deconvolution, their round trip, and argument checks."""
import math

import numpy as np
import pytest
import torch

from oracle import geometry as OG
from oracle import pressure as OPR

from gpu_common import DT, desc_for, host, rel, to_dev

pytestmark = pytest.mark.gpu

pat = pytest.importorskip("paper_1707_02245_amd.pat")
TOL = {"f64": 1e-12, "f32": 2e-5}
XP, YP = 0.05, -0.03


def _pulses(og, c, kind, width=3.0):
    """Calibration traces: the pulse of a point source at (XP, YP) arriving
    at each detector's travel time. 'bipolar': a derivative of a Gaussian;
    'causal': a decaying exponential starting on arrival (no spectral
    zero)."""
    dist = np.hypot(og.det_xy[:, 0] - XP, og.det_xy[:, 1] - YP)
    dt = og.radii[1] - og.radii[0]  # c = 1: radii step = dt
    t = np.arange(og.n_t) * dt
    lag = t[None, :] - (dist / c)[:, None]
    if kind == "bipolar":
        w = width * dt
        s = lag - 4 * w
        return -s / (w * w) * np.exp(-s * s / (2 * w * w))
    return np.where(lag >= 0, np.exp(-np.maximum(lag, 0) / (width * dt)), 0.0)


@pytest.mark.parametrize("dt_name", ["f64", "f32"])
def test_pressure_and_preprocess_match_oracle(dt_name):
    d = desc_for(64, 32, 128)
    og = OG.make_geometry(d)
    A = OG.forward_matrix(og)
    g = pat.Geometry(dtype=DT[dt_name], **d)
    rng = np.random.default_rng(5)
    u = np.clip(rng.uniform(-0.2, 1.0, (64, 64)), 0, None)
    pcal = _pulses(og, 1.0, "bipolar")
    eps = 1e-3
    cal = pat.Calibration(g, to_dev(pcal, DT[dt_name]), XP, YP, eps)
    print(f"pressure {dt_name}: L = {OPR.fft_length(128)}", flush=True)
    p = host(cal.pressure(to_dev(u, DT[dt_name])))
    p_ref = OPR.pressure_forward((A @ u.ravel()).reshape(32, 128), pcal, og.det_xy, XP, YP, 1.0, d["dt"])
    assert rel(p, p_ref) <= TOL[dt_name], rel(p, p_ref)
    # preprocessing of the oracle's pressure (plus noise)
    pn = p_ref + 0.01 * np.linalg.norm(p_ref) / math.sqrt(p_ref.size) * rng.standard_normal(p_ref.shape)
    f = host(cal.preprocess(to_dev(pn, DT[dt_name])))
    f_ref = OPR.preprocess(pn, pcal, og.det_xy, XP, YP, 1.0, d["dt"], eps)
    assert rel(f, f_ref) <= TOL[dt_name], rel(f, f_ref)
    cal.close()


def test_round_trip_gives_the_projection():
    """A causal pulse without spectral zeros arriving on a whole sample (the
    source at the ring's centre, 97 samples: travel time 48 dt) and a tiny
    eps: preprocessing the modelled pressure gives A u back (FP64). (A pulse
    starting between samples is not band-limited, so its shifted spectrum
    does not describe a causal pulse and the window's truncation is not
    undone.)"""
    d = desc_for(48, 16, 97)
    og = OG.make_geometry(d)
    A = OG.forward_matrix(og)
    g = pat.Geometry(dtype=torch.float64, **d)
    u = np.clip(np.random.default_rng(6).uniform(-0.2, 1.0, (48, 48)), 0, None)
    dist = np.hypot(og.det_xy[:, 0], og.det_xy[:, 1])
    k0 = np.rint(dist / d["dt"]).astype(int)
    assert np.all(k0 == 48) and np.allclose(dist / d["dt"], 48, rtol=0, atol=1e-9)
    k = np.arange(97)
    pcal = np.where(k[None, :] >= k0[:, None], np.exp(-np.maximum(k[None, :] - k0[:, None], 0) / 3.0), 0.0)
    cal = pat.Calibration(g, to_dev(pcal, torch.float64), 0.0, 0.0, 1e-24)
    f = host(cal.preprocess(cal.pressure(to_dev(u, torch.float64))))
    e = rel(f, A @ u.ravel())
    print(f"round trip: rel {e:.2e}", flush=True)
    assert e <= 1e-7


def test_calibration_arguments():
    d = desc_for(32, 8, 40)
    g = pat.Geometry(dtype=torch.float64, **d)
    pc = g.data(1.0)
    for bad in (dict(eps=0.0), dict(eps=-1.0), dict(eps=math.nan), dict(xp=math.inf)):
        kw = dict(xp=XP, yp=YP, eps=1e-3)
        kw.update(bad)
        with pytest.raises(pat.L.PatError) as e:
            pat.Calibration(g, pc, **kw)
        assert e.value.status == pat.L.PAT_ERR_INVALID_ARG
    det = g.info  # the first detector of a closed ring sits at (1.2, 0)
    with pytest.raises(pat.L.PatError) as e:
        pat.Calibration(g, pc, 1.2, 0.0, 1e-3)
    assert e.value.status == pat.L.PAT_ERR_INVALID_ARG
    big = pat.Geometry(dtype=torch.float64, **desc_for(8, 2, 2049))
    with pytest.raises(pat.L.PatError) as e:
        pat.Calibration(big, big.data(1.0), XP, YP, 1e-3)
    assert e.value.status == pat.L.PAT_ERR_UNSUPPORTED
