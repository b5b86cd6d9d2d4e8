"""GPU checks of the warm-start plumbing through the C ABI: the network input
and targets (pat_warmstart_normalize) and the starting point
(pat_warmstart_infer) against host arithmetic on the oracle's A.

The network output itself is checked in the U-Net parity tests; here it is
read back through pat_warmstart_forward and everything around it is compared
in FP64 (1e-12 relative: the only differences are summation order).
"""
import numpy as np
import pytest
import torch

from oracle import geometry as OG
from oracle import pdhg as OP

from gpu_common import desc_for, host, oracle_problem, rel, split_state, synth_data, to_dev

pytestmark = pytest.mark.gpu

pat = pytest.importorskip("paper_1707_02245_amd.pat")
ws = pytest.importorskip("paper_1707_02245_amd.warmstart")


def _case(n=32, n_det=24, n_t=64, seed=4):
    d = desc_for(n, n_det, n_t)
    og = OG.make_geometry(d)
    A = OG.forward_matrix(og)
    f, _ = synth_data(d, "mixed", seed)
    g = pat.Geometry(dtype=torch.float64, **d)
    return d, A, f, g


def _normalised_bp(A, f):
    atf = A.T @ f
    at1 = A.T @ np.ones(A.shape[0])
    bp = np.where(at1 > 0, atf / np.where(at1 > 0, at1, 1.0), 0.0)
    s = max(np.mean(np.abs(bp)), 1e-12)
    return bp / s, s


def test_normalize_input_and_targets():
    d, A, f, g = _case()
    n = d["nx"]
    lam = 0.02
    reg = pat.Reg("tv", lam)
    so = torch.empty(g.state_elems("tv"), dtype=torch.float64, device="cuda")
    fd = to_dev(f, torch.float64)
    pat.solve(g, fd, reg, max_iter=200, gap_tol=0.0, gap_every=50, state_out=so)
    x, t, s = ws.normalize(g, fd, reg, so, 3)
    bp, s_ref = _normalised_bp(A, f)
    assert host(s)[0] == pytest.approx(s_ref, rel=1e-6)          # stored as FP32
    assert rel(host(x).ravel(), bp) <= 1e-6
    st = split_state(host(so), "tv", n * n, A.shape[0])
    tt = host(t).reshape(3, n * n)
    assert rel(tt[0], st["u"] / s_ref) <= 1e-6
    assert rel(tt[1:], st["r"] / lam) <= 1e-6
    x1, t1, _ = ws.normalize(g, fd, reg, so, 1)
    assert torch.equal(x1, x) and torch.equal(t1[0], t[0])
    x2, t2, _ = ws.normalize(g, fd)
    assert t2 is None and torch.equal(x2, x)


def test_infer_builds_primal_and_dual_start():
    d, A, f, g = _case(seed=6)
    n = d["nx"]
    lam = 0.02
    reg = pat.Reg("tv", lam)
    net = ws.WarmStartNet(3, 8, 3, seed=11)
    fd = to_dev(f, torch.float64)
    u0, y0 = net.infer(g, fd, reg, dual=True)
    x, _, s = ws.normalize(g, fd)
    y = torch.empty(1, 3, n, n, dtype=torch.float32, device="cuda")
    pat.L.check(pat.L.load().pat_warmstart_forward(net._h, 1, n, n, pat._ptr(x), pat._ptr(y), pat._stream()))
    yh = host(y).reshape(3, n * n)
    sc = float(host(s)[0])
    u_ref = yh[0] * sc
    assert rel(host(u0).ravel(), u_ref) <= 1e-7
    y0h = host(y0)
    nb = A.shape[0]
    q_ref = A @ host(u0).ravel() - f
    assert rel(y0h[:nb], q_ref) <= 1e-12
    m = np.maximum(1.0, np.hypot(yh[1], yh[2]))
    r_ref = lam * yh[1:] / m
    r = y0h[nb:].reshape(2, n * n)
    assert rel(r, r_ref) <= 1e-7
    assert np.all(np.hypot(r[0], r[1]) <= lam * (1 + 1e-12))
    u1, none = net.infer(g, fd, reg, dual=False)
    assert none is None and torch.equal(u1, u0)
    one = ws.WarmStartNet(3, 8, 1, seed=11)
    with pytest.raises(pat.L.PatError):
        one.infer(g, fd, reg, dual=True)
    with pytest.raises(pat.L.PatError):
        net.infer(g, fd, pat.Reg("tgv", lam, 2 * lam), dual=True)


def test_network_start_runs_the_oracle_iteration():
    """PDHG from the network's (u0, y0) is the oracle's iteration from that
    state. The weights are zero but the head biases (0.1, 0.3, -0.2), so the
    start is u0 = 0.1 s, r0 = lambda (0.3, -0.2), q0 = A u0 - f."""
    d, A, f, g = _case(seed=8)
    n = d["nx"]
    lam = 0.02
    reg = pat.Reg("tv", lam)
    net = ws.WarmStartNet(3, 8, 3, seed=2)
    v = np.zeros(net.n_params, dtype=np.float32)
    v[-3:] = [0.1, 0.3, -0.2]
    net.set_params(v)
    fd = to_dev(f, torch.float64)
    u0, y0 = net.infer(g, fd, reg, dual=True)
    _, s = _normalised_bp(A, f)
    uh, yh = host(u0).ravel(), host(y0)
    nb = A.shape[0]
    assert np.allclose(uh, 0.1 * s, rtol=1e-6)
    assert np.allclose(yh[nb:].reshape(2, -1), [[0.3 * lam], [-0.2 * lam]], rtol=1e-6)
    p = oracle_problem(A, f, n, "tv", lam)
    pc = OP.precond_diag(p)
    assert not OP.warm_start_rejected(p, uh)
    st = OP.init_state(p, uh)
    st["q"], st["r"] = yh[:nb].copy(), yh[nb:].reshape(2, -1).copy()
    ref = OP.pdhg_solve(p, pc, iters=30, state=st)
    u, info, _ = pat.solve(g, fd, reg, max_iter=30, gap_tol=0.0, gap_every=10, graph_block=10,
                           u0=u0, y0=y0)
    assert info["fallback"] == 0 and rel(host(u).ravel(), ref["u"]) <= 1e-10


def test_trained_network_on_held_out_phantoms():
    """The committed network (trained on seeds 10000-10767 for the current
    operator) against plain PDHG from zero on three held-out 256^2 TV cases,
    FP64 to rel_gap 1e-4: its start is never rejected, costs no more
    iterations than the start from zero (one gap interval of slack), and both
    runs certify the same objective within the gap. (At this gap the start
    buys little: the measured 64-seed means are in the weights' manifest.)"""
    import os
    import phantoms
    wl = phantoms.WORKLOADS["tv256"]
    desc = phantoms.geometry_desc(wl.n, wl.n_det, wl.n_t)
    g = pat.Geometry(dtype=torch.float64, **desc)
    net = ws.WarmStartNet(4, 32, 3, seed=0)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    net.load_weights(os.path.join(root, "paper_1707_02245_amd", "weights", "warmstart_tv256.npy"))
    reg = pat.Reg("tv", wl.lam)
    pc = pat.Precond(g, reg, "diag")
    kw = dict(max_iter=60000, gap_tol=1e-4, gap_every=50, graph_block=50, precond=pc)
    for seed in (50100, 50101, 50102):
        f, _, noise = ws.synth_data(desc, seed)
        _, i0, s0 = pat.solve(g, f, reg, **kw)
        u0, y0 = net.infer(g, f, reg, dual=True)
        _, i1, s1 = pat.solve(g, f, reg, u0=u0, y0=y0, **kw)
        print(f"held-out seed {seed} (noise {noise:.3f}): zero {i0['iters']} iterations, network "
              f"{i1['iters']}", flush=True)
        assert s0 == 0 and s1 == 0 and i1["fallback"] == 0
        assert i1["iters"] <= i0["iters"] + 50
        assert abs(i1["primal"] - i0["primal"]) <= 2e-4 * i0["primal"]


def test_weights_of_another_operator_are_refused(tmp_path):
    """The weights' manifest names the operator they were trained on; a
    different fingerprint is refused on load."""
    import json
    import os
    import shutil
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = os.path.join(root, "paper_1707_02245_amd", "weights", "warmstart_tv256")
    shutil.copy(src + ".npy", tmp_path / "w.npy")
    with open(src + ".json") as fh:
        man = json.load(fh)
    assert man["operator_fingerprint"] == ws.operator_fingerprint()
    man["operator_fingerprint"] = "0" * 16
    with open(tmp_path / "w.json", "w") as fh:
        json.dump(man, fh)
    net = ws.WarmStartNet(4, 32, 3, seed=0)
    with pytest.raises(ValueError, match="another forward operator"):
        net.load_weights(str(tmp_path / "w.npy"))
    net.load_weights(str(tmp_path / "w.npy"), check_operator=False)
