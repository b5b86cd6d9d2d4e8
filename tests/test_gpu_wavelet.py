"""GPU parity of the wavelet model (Sec. 2.2 eq. min_wav: lam ||W u||_1 with the
dual-tree transform W; Algorithm 1 with grad -> W and div -> W^T) through the C
ABI against the FP64 oracle (oracle.wavelet, oracle.pdhg with kind "wav").

Tolerances: the transform FP64 to 1e-12 relative element-wise (rounding order
only), FP32 to 1e-5 relative L2; solver states after a fixed iteration count
FP64 1e-10, FP32 1e-4 relative L2, as for the other regularisers.
"""
import numpy as np
import pytest
import torch

from oracle import geometry as OG
from oracle import pdhg as OP
from oracle import wavelet as OW

from gpu_common import DT, desc_for, host, oracle_problem, rel, split_state, to_dev

pytestmark = pytest.mark.gpu

pat = pytest.importorskip("paper_1707_02245_amd.pat")

# (nx, ny, levels): square and oblong, bands below one workgroup, a 1 x 1
# last level, the largest level count the sides allow, and 128^2 (several
# workgroups per band at every level)
SHAPES = [(16, 16, 2), (32, 16, 3), (8, 8, 3), (24, 8, 3), (2, 2, 1), (64, 48, 4), (16, 32, 4),
          (128, 128, 3)]


def _check(got, ref, dt):
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    if dt == "f64":
        err = np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)
        assert err <= 1e-12, err
    else:
        assert rel(got, ref) <= 1e-5, rel(got, ref)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES, ids=[f"{a}x{b}J{c}" for a, b, c in SHAPES])
def test_transform_and_adjoint_match_the_oracle(shape, dt):
    nx, ny, J = shape
    rng = np.random.default_rng(nx * 1000 + ny * 10 + J)
    W = OW.dtwt_matrix(nx, ny, J)
    u = rng.standard_normal((ny, nx))
    print(f"wavelet {nx}x{ny} J={J} {dt}", flush=True)
    c = pat.wavelet_forward(to_dev(u, DT[dt]), J)
    _check(host(c), W @ u.ravel(), dt)
    cin = rng.standard_normal(4 * nx * ny)
    v = pat.wavelet_adjoint(to_dev(cin, DT[dt]), nx, ny, J)
    _check(host(v), W.T @ cin, dt)
    # with a caller's work buffer (stream-ordered, nothing allocated): the
    # same bits, twice in a row through the same buffer
    work = pat.wavelet_work(nx, ny, DT[dt])
    for _ in range(2):
        c2 = pat.wavelet_forward(to_dev(u, DT[dt]), J, work=work)
        v2 = pat.wavelet_adjoint(to_dev(cin, DT[dt]), nx, ny, J, work=work)
        assert np.array_equal(host(c2), host(c)) and np.array_equal(host(v2), host(v))


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("J", [3, 8])
def test_full_size_parseval_inverse_and_constant(J, dt):
    """256 x 256 (the image size of the TV and TGV workloads), 3 levels and
    the 8 the sides allow: ||W u|| = ||u||, W^T W u = u, and a constant image
    has no detail and lowpass coefficients c 2^J / 2 (each tree's lowpass
    doubles a constant per level; the frame factor halves it)."""
    n = 256
    rng = np.random.default_rng(J)
    u = rng.uniform(-1, 1, (n, n))
    ud = to_dev(u, DT[dt])
    c = pat.wavelet_forward(ud, J)
    back = pat.wavelet_adjoint(c, n, n, J)
    tol = 1e-12 if dt == "f64" else 2e-6
    assert abs(np.linalg.norm(host(c)) / np.linalg.norm(u) - 1.0) <= tol
    assert rel(host(back), u) <= tol * 10
    cc = host(pat.wavelet_forward(torch.full((n, n), 3.0, dtype=DT[dt], device="cuda"), J))
    ll = OW.band_offsets(n, n, J)[("LL", "aa")]
    assert np.abs(cc[:ll]).max() <= (1e-12 if dt == "f64" else 1e-5) * 3.0
    assert np.allclose(cc[ll:], 3.0 * 2 ** J / 2, rtol=1e-12 if dt == "f64" else 1e-6)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_large_levels_inverse_and_parseval(dt):
    """1024 x 1024, 3 levels: the synthesis takes its LDS-tiled kernel at
    levels 1 and 2 (256 tiles of 16 x 16 positions at level 2) and one thread
    per position at level 3. W^T W u = u and ||W u|| = ||u|| hold at any size,
    with W pinned to the oracle's matrix on the small shapes above."""
    n, J = 1024, 3
    rng = np.random.default_rng(7)
    u = rng.uniform(-1, 1, (n, n))
    print(f"wavelet {n}x{n} J={J} {dt}", flush=True)
    c = pat.wavelet_forward(to_dev(u, DT[dt]), J)
    back = pat.wavelet_adjoint(c, n, n, J)
    tol = 1e-12 if dt == "f64" else 2e-6
    assert abs(np.linalg.norm(host(c)) / np.linalg.norm(u) - 1.0) <= tol
    assert rel(host(back), u) <= tol * 10


def test_transform_rejects_bad_shapes():
    u = torch.zeros((12, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(Exception):
        pat.wavelet_forward(u, 3)   # 12 is not a multiple of 8
    with pytest.raises(Exception):
        pat.wavelet_forward(u, 0)


# ------------------------------------------------------------------ the solver

GEOMS = {
    # 48 x 32 on a 12-detector ring (oblong image: plain stored A^T)
    "rect48": dict(n=48, n_det=12, n_t=90, ny=32, y_max=-1 + 32 * 2 / 48),
    # 64^2 on a 32-detector ring (quarter-turn symmetric: the quarter A^T)
    "ring64": dict(n=64, n_det=32, n_t=128),
}


def _geoms(name, dt):
    kw = dict(GEOMS[name])
    d = desc_for(kw.pop("n"), kw.pop("n_det"), kw.pop("n_t"))
    d.update(kw)
    og = OG.make_geometry(d)
    g = pat.Geometry(dtype=DT[dt], **d)
    return og, g


def _data(og, seed):
    A = OG.forward_matrix(og)
    rng = np.random.default_rng(seed)
    u = np.zeros((og.ny, og.nx))
    u[og.ny // 4: og.ny // 2, og.nx // 3] = 1.0          # a thin vertical line
    u[og.ny // 2:, og.nx // 2:] += 0.5                    # and a block
    f = A @ u.ravel() + 0.01 * rng.standard_normal(og.n_bins)
    return A, f


def _gap_terms_agree(info, p, ref, dt):
    g_ref = OP.gap_terms(p, ref, 2.0)
    f64 = dt == "f64"
    print(f"  P {info['primal']:.6e}/{g_ref['P']:.6e} R {info['kty_l1']:.6e}/{g_ref['R']:.6e} "
          f"gap {info['gap']:.6e}/{g_ref['gap']:.6e}", flush=True)
    assert info["primal"] == pytest.approx(g_ref["P"], rel=1e-9 if f64 else 1e-4)
    assert abs(info["fstar"] - g_ref["Fstar"]) <= (1e-10 if f64 else 1e-5) * g_ref["P"]
    assert info["kty_l1"] == pytest.approx(g_ref["R"], rel=1e-8 if f64 else 1e-4)
    assert abs(info["gap"] - g_ref["gap"]) <= (1e-10 if f64 else 1e-5) * g_ref["P"]
    assert info["residual"] == pytest.approx(OP.residual(ref), rel=1e-8 if f64 else 1e-3)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_diag_and_block_step_sizes(dt):
    og, g = _geoms("rect48", dt)
    A = OG.forward_matrix(og)
    p = oracle_problem(A, np.zeros(og.n_bins), og.nx, "wav", 0.02, ny=og.ny, levels=3)
    ref = OP.precond_diag(p)
    pc = pat.Precond(g, pat.Reg("wav", 0.02, levels=3), "diag")
    tol = 1e-12 if dt == "f64" else 1e-5
    assert rel(host(pc.get("tau_u")), ref["tau_u"]) <= tol
    assert rel(host(pc.get("sigma_q")), ref["sigma_q"]) <= tol
    sr = host(pc.get("sigma_r"))
    assert sr.size == 4 * og.n_pix and np.all(sr == 1.0)
    if dt == "f64":
        refb = OP.precond_block(p)
        pb = pat.Precond(g, pat.Reg("wav", 0.02, levels=3), "block")
        assert host(pb.get("tau_u"))[0] == pytest.approx(refb["tau_u"][0], rel=1e-9)
        assert host(pb.get("sigma_q"))[0] == pytest.approx(refb["sigma_q"][0], rel=1e-9)
        assert host(pb.get("sigma_r"))[0] == pytest.approx(refb["sigma_r"][0], rel=1e-9)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("name,J", [("rect48", 3), ("ring64", 2), ("ring64", 6)])
def test_fixed_iterations_full_state(name, J, dt):
    """State after 60 iterations (u, ubar, q, r) and the gap terms against
    Algorithm 1 with W."""
    og, g = _geoms(name, dt)
    A, f = _data(og, 5)
    lam = 0.01
    p = oracle_problem(A, f, og.nx, "wav", lam, ny=og.ny, levels=J)
    ref = OP.pdhg_solve(p, OP.precond_diag(p), iters=60)
    reg = pat.Reg("wav", lam, levels=J)
    st = torch.zeros(g.state_elems("wav"), dtype=DT[dt], device="cuda")
    u, info, _ = pat.solve(g, to_dev(f, DT[dt]), reg, max_iter=60, gap_tol=0.0, gap_every=10,
                           graph_block=20, state_out=st)
    got = split_state(host(st), "wav", og.n_pix, og.n_bins)
    tol = 1e-10 if dt == "f64" else 1e-4
    print(f"wav {name} J={J} {dt}: rel u {rel(got['u'], ref['u']):.2e} r {rel(got['r'], ref['r']):.2e}",
          flush=True)
    assert info["iters"] == 60
    assert rel(host(u), ref["u"]) <= tol
    for key in ("u", "ubar", "q", "r"):
        assert rel(got[key], ref[key]) <= tol, key
    # the dual stays in the box [-lam, lam] and reaches it
    assert np.abs(got["r"]).max() <= lam * (1 + 1e-6)
    assert np.abs(got["r"]).max() >= 0.999 * lam
    _gap_terms_agree(info, p, ref, dt)


def test_block_steps_fixed_iterations():
    """The two-block scalar steps (L2 = ||W|| by power iteration, sigma2 for
    every coefficient) for 60 iterations against the oracle's."""
    og, g = _geoms("rect48", "f64")
    A, f = _data(og, 10)
    p = oracle_problem(A, f, og.nx, "wav", 0.01, ny=og.ny, levels=3)
    pcr = OP.precond_block(p)
    assert pcr["L2"] == pytest.approx(1.05, rel=1e-9)  # ||W|| = 1 times the safety factor
    ref = OP.pdhg_solve(p, pcr, iters=60)
    reg = pat.Reg("wav", 0.01, levels=3)
    pc = pat.Precond(g, reg, "block")
    st = torch.zeros(g.state_elems("wav"), dtype=torch.float64, device="cuda")
    _, info, _ = pat.solve(g, to_dev(f, torch.float64), reg, max_iter=60, gap_tol=0.0, gap_every=10,
                           graph_block=20, state_out=st, precond=pc)
    got = split_state(host(st), "wav", og.n_pix, og.n_bins)
    for key in ("u", "ubar", "q", "r"):
        assert rel(got[key], ref[key]) <= 1e-8, key


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_accelerated_fixed_iterations(dt):
    og, g = _geoms("rect48", dt)
    A, f = _data(og, 6)
    p = oracle_problem(A, f, og.nx, "wav", 0.01, ny=og.ny, levels=3)
    ref = OP.pdhg_solve(p, OP.precond_diag(p), iters=60, accel_gamma=0.5, accel_step_max=3.0)
    st = torch.zeros(g.state_elems("wav"), dtype=DT[dt], device="cuda")
    _, info, _ = pat.solve(g, to_dev(f, DT[dt]), pat.Reg("wav", 0.01, levels=3), max_iter=60, gap_tol=0.0,
                           gap_every=10, graph_block=20, state_out=st, accel_gamma=0.5, accel_step_max=3.0)
    got = split_state(host(st), "wav", og.n_pix, og.n_bins)
    tol = 1e-10 if dt == "f64" else 1e-4
    for key in ("u", "ubar", "q", "r"):
        assert rel(got[key], ref[key]) <= tol, key
    _gap_terms_agree(info, p, ref, dt)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_batch_with_tv_is_bitwise_single_solves(dt):
    """A wavelet and a TV instance on one geometry in one batch (shared
    forward and A^T passes, the wavelet steps per instance): each equals its
    own solve bit for bit."""
    og, g = _geoms("ring64", dt)
    A, f = _data(og, 7)
    fd = to_dev(f, DT[dt])
    problems = [(g, fd, pat.Reg("wav", 0.01, levels=3)), (g, fd, pat.Reg("tv", 0.01))]
    us, infos, _ = pat.solve_batched(problems, max_iter=200, gap_tol=1e-3, gap_every=10, graph_block=50)
    for (gg, ff, reg), u, info in zip(problems, us, infos):
        u1, i1, _ = pat.solve(gg, ff, reg, max_iter=200, gap_tol=1e-3, gap_every=10, graph_block=50)
        assert info["iters"] == i1["iters"]
        assert np.array_equal(host(u), host(u1)), reg.kind


def test_resume_is_bitwise():
    og, g = _geoms("rect48", "f32")
    A, f = _data(og, 8)
    fd = to_dev(f, torch.float32)
    reg = pat.Reg("wav", 0.01, levels=3)
    n_st = g.state_elems("wav")
    assert n_st == 2 * og.n_pix + og.n_bins + 4 * og.n_pix
    full, half, again = (torch.zeros(n_st, dtype=torch.float32, device="cuda") for _ in range(3))
    pat.solve(g, fd, reg, max_iter=100, gap_tol=0.0, gap_every=10, graph_block=50, state_out=full)
    pat.solve(g, fd, reg, max_iter=50, gap_tol=0.0, gap_every=10, graph_block=50, state_out=half)
    pat.solve(g, fd, reg, max_iter=50, gap_tol=0.0, gap_every=10, graph_block=50, state_in=half,
              state_out=again)
    assert np.array_equal(host(full), host(again))


def test_converges_to_the_gap_and_the_oracle_objective():
    """Run to rel. gap 1e-3: the same stopping iteration as the oracle (FP32
    within one check interval, its gap rounding near the threshold) and the
    same objective."""
    og, _ = _geoms("rect48", "f64")
    A, f = _data(og, 9)
    p = oracle_problem(A, f, og.nx, "wav", 0.01, ny=og.ny, levels=3)
    ref = OP.pdhg_solve(p, OP.precond_diag(p), tol=1e-3, max_iter=20000, gap_every=50)
    assert ref["history"][-1]["rel_gap"] <= 1e-3
    for dt in ("f64", "f32"):
        _, g = _geoms("rect48", dt)
        u, info, st = pat.solve(g, to_dev(f, DT[dt]), pat.Reg("wav", 0.01, levels=3), max_iter=20000,
                                gap_tol=1e-3, gap_every=50, graph_block=50)
        print(f"wav {dt}: iters {info['iters']} (oracle {ref['history'][-1]['n']}) "
              f"rel_gap {info['rel_gap']:.3e}", flush=True)
        assert st == 0 and info["converged"] == 1 and info["rel_gap"] <= 1e-3
        if dt == "f64":
            assert info["iters"] == ref["history"][-1]["n"]
        else:
            assert abs(info["iters"] - ref["history"][-1]["n"]) <= 50
        assert info["primal"] == pytest.approx(ref["history"][-1]["P"], rel=1e-4)
