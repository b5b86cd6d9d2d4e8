"""The forward in quarter-turn form (GPU, through the C ABI) against the FP64
oracle: on a ring of 4m detectors about a square grid the bins of detector
d + t m are those of detector d on the image turned by t quarter turns, so
the gather runs over the first quarter of the detectors with four images.
Checked: every bin against the oracle's matrix, the slot mapping bit for bit
(quarter t of A u equals quarter 0 of A applied to u turned t times), the
direct evaluation, both block orders, and the solver's state and gap terms
after a fixed number of iterations, alone and batched.
"""
import numpy as np
import pytest
import torch

from oracle import geometry as OG
from oracle import pdhg as OP

from gpu_common import DT, desc_for, host, oracle_problem, rel, split_state, to_dev

pytestmark = pytest.mark.gpu

pat = pytest.importorskip("paper_1707_02245_amd.pat")

TOL_APPLY = {"f64": 1e-12, "f32": 1e-5}

# (n, n_det, n_t): a quarter of 8, 3, 1 and 2 detectors, odd and even grids
SHAPES = [(64, 32, 128), (45, 12, 70), (37, 4, 41), (3, 8, 9)]


def _setup(shape, dt):
    n, n_det, n_t = shape
    d = desc_for(n, n_det, n_t)
    og = OG.make_geometry(d)
    g = pat.Geometry(dtype=DT[dt], **d)
    return d, og, g


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES)
def test_quarter_turn_forward_matches_oracle(shape, dt):
    n, n_det, n_t = shape
    d, og, g = _setup(shape, dt)
    print(f"quarter-turn forward {shape} {dt}", flush=True)
    assert g.info["sym_rot"] == 4 and g.info["fwd_sym"] == 1  # off by default
    g.set_forward_symmetry(True)
    assert g.info["fwd_sym"] == 4
    A = OG.forward_matrix(og)
    u = np.random.default_rng(21).standard_normal((n, n))
    ref = A @ u.ravel()
    ud = to_dev(u, DT[dt])
    out = {}
    for lanes in (4, 5, 6):
        per_path = []
        for path in (0, 1):
            g.set_launch(lanes, g.info["adj_tile"], g.info["adj_det_group"])
            g.set_forward_path(path)
            per_path.append(host(g.forward(ud)))
        # the two block orders give each bin the same sum
        assert np.array_equal(per_path[0], per_path[1]), lanes
        assert rel(per_path[0], ref) <= TOL_APPLY[dt], lanes
        out[lanes] = per_path[0]
    # the padded entry point reads the same padded image
    upad = torch.zeros((n + 2, n + 2), dtype=DT[dt], device="cuda")
    upad[1:-1, 1:-1] = ud
    assert np.array_equal(host(g.forward_padded(upad)), out[6])
    # the direct evaluation of every detector: same operator
    g.set_forward_symmetry(False)
    assert g.info["fwd_sym"] == 1
    direct = host(g.forward(ud))
    assert rel(direct, ref) <= TOL_APPLY[dt]
    assert rel(direct, out[6]) <= TOL_APPLY[dt]
    g.set_forward_symmetry(True)
    assert g.info["fwd_sym"] == 4
    # the tiled path has no quarter-turn form
    g.set_forward_path(2)
    assert g.info["fwd_sym"] == 1
    assert rel(host(g.forward(ud)), ref) <= TOL_APPLY[dt]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_quarter_turn_slots_bitwise(dt):
    """Slot t of the forward of u computes exactly what slot 0 computes for u
    turned t quarter turns (u_t(p) = u(R^t p), R(i, j) = (n-1-j, i))."""
    shape = (45, 12, 70)
    n, n_det, n_t = shape
    d, og, g = _setup(shape, dt)
    g.set_forward_symmetry(True)
    q = n_det // 4
    u = np.random.default_rng(22).standard_normal((n, n))
    base = host(g.forward(to_dev(u, DT[dt]))).reshape(n_det, n_t)
    for t in range(4):
        ut = np.rot90(u, t)  # ut[j, i] = u at the pixel R^t (i, j)
        turned = host(g.forward(to_dev(ut, DT[dt]))).reshape(n_det, n_t)
        assert np.array_equal(turned[:q], base[t * q:(t + 1) * q]), t


def test_not_symmetric_stays_direct():
    d = desc_for(40, 16, 60, det_cx=0.01)
    og = OG.make_geometry(d)
    g = pat.Geometry(dtype=torch.float64, **d)
    assert g.info["sym_rot"] == 1 and g.info["fwd_sym"] == 1
    u = np.random.default_rng(23).standard_normal((40, 40))
    assert rel(host(g.forward(to_dev(u, torch.float64))), OG.forward_matrix(og) @ u.ravel()) <= 1e-12


def _problem(og, kind, dt, seed=4):
    A = OG.forward_matrix(og)
    rng = np.random.default_rng(seed)
    f = A @ np.clip(rng.uniform(-0.2, 1, og.n_pix), 0, None) + 0.01 * rng.standard_normal(og.n_bins)
    th = np.random.default_rng(3).uniform(-1.5, 1.5, (og.ny, og.nx))
    reg = pat.Reg(kind, 0.02, 0.04, 0.1, to_dev(th, DT[dt]) if kind == "dtv" else None)
    p = oracle_problem(A, f, og.nx, kind, reg.lam, reg.alpha0, reg.eta, th, ny=og.ny)
    return f, reg, p


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["tv", "tgv", "dtv", "tikhonov"])
def test_solver_state_in_quarter_turn_form(kind, dt):
    """60 iterations with the forward in quarter-turn form (the primal step
    writes the turned copies; the gap's forward uses four slots of partials):
    full state and gap terms against Alg. 1/2, and the direct forward's solve
    agrees."""
    d, og, g = _setup((45, 12, 70), dt)
    g.set_forward_symmetry(True)
    assert g.info["fwd_sym"] == 4
    f, reg, p = _problem(og, kind, dt)
    ref = OP.pdhg_solve(p, OP.precond_diag(p), iters=60)
    tol = 1e-10 if dt == "f64" else 1e-4
    for sym in (True, False):
        g.set_forward_symmetry(sym)
        st = torch.zeros(g.state_elems(kind), dtype=DT[dt], device="cuda")
        u, info, status = pat.solve(g, to_dev(f, DT[dt]), reg, max_iter=60, gap_tol=0.0,
                                   gap_every=10, graph_block=20, state_out=st)
        got = split_state(host(st), kind, og.n_pix, og.n_bins)
        print(f"{kind} {dt} quarter-turn {sym}: rel u {rel(got['u'], ref['u']):.2e} "
              f"gap {info['gap']:.6e}", flush=True)
        assert info["iters"] == 60
        for key in ("u", "ubar", "q", "r", "v", "vbar", "s"):
            if key in got and key in ref:
                e = rel(got[key], ref[key])
                assert e <= tol, (sym, key, e)
        g_ref = OP.gap_terms(p, ref, 2.0)
        assert info["primal"] == pytest.approx(g_ref["P"], rel=1e-9 if dt == "f64" else 1e-4)
        assert abs(info["gap"] - g_ref["gap"]) <= (1e-10 if dt == "f64" else 1e-5) * g_ref["P"]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_batched_quarter_turn_beside_direct_instances(dt):
    """A batch mixing instances in quarter-turn form (two on one geometry)
    with instances of an asymmetric geometry (grouped by geometry): every
    result is bitwise its single solve, and warm-started from a state (the
    turned copies rebuilt from it) the resumed solve is bitwise the
    uninterrupted one."""
    _, og_s, g_s = _setup((45, 12, 70), dt)
    g_s.set_forward_symmetry(True)
    d_a = desc_for(40, 12, 60, det_cx=0.01)
    og_a = OG.make_geometry(d_a)
    g_a = pat.Geometry(dtype=DT[dt], **d_a)
    assert g_s.info["fwd_sym"] == 4 and g_a.info["fwd_sym"] == 1
    problems = []
    for og, g, kind, seed in ((og_s, g_s, "tgv", 1), (og_a, g_a, "tv", 2), (og_s, g_s, "tv", 3),
                              (og_a, g_a, "tgv", 4)):
        f, reg, _ = _problem(og, kind, dt, seed)
        problems.append((g, to_dev(f, DT[dt]), reg))
    us, infos, _ = pat.solve_batched(problems, max_iter=200, gap_tol=1e-3, gap_every=10, graph_block=50)
    for (g, f, reg), u, info in zip(problems, us, infos):
        u1, i1, _ = pat.solve(g, f, reg, max_iter=200, gap_tol=1e-3, gap_every=10, graph_block=50)
        assert info["iters"] == i1["iters"]
        assert np.array_equal(host(u), host(u1))
    g, f, reg = problems[0]
    mid = torch.zeros(g.state_elems("tgv"), dtype=DT[dt], device="cuda")
    pat.solve(g, f, reg, max_iter=40, gap_tol=0.0, gap_every=20, graph_block=20, state_out=mid)
    u_res, _, _ = pat.solve(g, f, reg, max_iter=40, gap_tol=0.0, gap_every=20, graph_block=20, state_in=mid)
    u_all, _, _ = pat.solve(g, f, reg, max_iter=80, gap_tol=0.0, gap_every=20, graph_block=20)
    assert np.array_equal(host(u_res), host(u_all))
