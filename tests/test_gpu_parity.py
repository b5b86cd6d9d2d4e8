"""GPU parity of the HIP library (through the C ABI) against the FP64 oracle.

Tolerances: FP64 element-wise to 1e-12 relative per apply (rounding order
only); FP32 to 1e-5 relative L2 per apply and 1e-3 relative L2 on the image
after a fixed iteration count (the workload targets).
"""
import math

import numpy as np
import pytest
import torch

import phantoms
from oracle import geometry as OG
from oracle import pdhg as OP

from gpu_common import (DT, column_of_A, desc_for, host, oracle_problem, rel, split_state,
                        synth_data, to_dev)

pytestmark = pytest.mark.gpu

pat = pytest.importorskip("paper_1707_02245_amd.pat")

TOL_APPLY = {"f64": 1e-12, "f32": 1e-5}

CASES = {
    # name: (desc kwargs, note)
    "tv64": dict(n=64, n_det=32, n_t=128),                      # the 64^2 workload
    "ragged": dict(n=37, n_det=7, n_t=53, ny=29, y_max=-1 + 29 * 2 / 37),
    "arc90": dict(n=48, n_det=9, n_t=80, arc_span=math.pi / 2),
    "inside": dict(n=40, n_det=3, n_t=30, det_xy=[[0.1, -0.2], [-0.93, 0.9], [0.5, 0.05]],
                   dt=1.2 / 29),
    "tiny": dict(n=2, n_det=2, n_t=5),
    "onedet": dict(n=33, n_det=1, n_t=70),
}


def _desc(name):
    kw = dict(CASES[name])
    n = kw.pop("n")
    d = desc_for(n, kw.pop("n_det"), kw.pop("n_t"))
    if "ny" in kw:
        d["ny"] = kw.pop("ny")
    if "det_xy" in kw:
        d["det_xy"] = np.array(kw.pop("det_xy"))
        d["n_det"] = d["det_xy"].shape[0]
    d.update(kw)
    return d


def _geoms(name, dt):
    d = _desc(name)
    og = OG.make_geometry(d)
    gd = {k: v for k, v in d.items()}
    g = pat.Geometry(dtype=DT[dt], **gd)
    return d, og, g


@pytest.mark.parametrize("adj", ["tiled", "csr", "scatter"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("name", list(CASES))
def test_forward_adjoint_elementwise(name, dt, adj):
    d, og, g = _geoms(name, dt)
    g.set_adjoint(adj)
    A = OG.forward_matrix(og)
    rng = np.random.default_rng(11)
    u = rng.standard_normal(og.n_pix)
    y = rng.standard_normal(og.n_bins)
    print(f"case {name} {dt} {adj}: nx={og.nx} ny={og.ny} n_det={og.n_det} n_t={og.n_t}", flush=True)
    fu = host(g.forward(to_dev(u.reshape(og.ny, og.nx), DT[dt])))
    aty = host(g.adjoint(to_dev(y.reshape(og.n_det, og.n_t), DT[dt])))
    ef, ea = rel(fu, A @ u), rel(aty, A.T @ y)
    assert ef <= TOL_APPLY[dt] and ea <= TOL_APPLY[dt], (ef, ea)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("name", list(CASES))
def test_forward_paths(name, dt):
    """Radius-major and detector-major gather blocks give the same data bit
    for bit for every lane width; the LDS-tiled path gives the same operator
    (different summation order); all match the oracle."""
    d, og, g = _geoms(name, dt)
    A = OG.forward_matrix(og)
    u = np.random.default_rng(13).standard_normal((og.ny, og.nx))
    ud = to_dev(u, DT[dt])
    ref = A @ u.ravel()
    for lanes in (4, 5, 6):
        outs = []
        for path in (0, 1):
            g.set_launch(lanes, g.info["adj_tile"], g.info["adj_det_group"])
            g.set_forward_path(path)
            assert g.info["fwd_path"] == path
            outs.append(host(g.forward(ud)))
        assert np.array_equal(outs[0], outs[1]), lanes
        assert rel(outs[1], ref) <= TOL_APPLY[dt], lanes
    g.set_forward_path(2)
    assert g.info["fwd_path"] == 2 and g.info["fwd_pairs"] > 0
    assert rel(host(g.forward(ud)), ref) <= TOL_APPLY[dt]
    # path 3 (the stored A) exists on quarter-turn symmetric geometries only
    if g.info["sym_rot"] == 4:
        g.set_forward_path(3)
        assert rel(host(g.forward(ud)), ref) <= TOL_APPLY[dt]
    else:
        with pytest.raises(RuntimeError):
            g.set_forward_path(3)
    with pytest.raises(RuntimeError):
        g.set_forward_path(4)


@pytest.mark.parametrize("kind", ["tgv", "dtv"])
def test_tiled_forward_in_solver(kind):
    """The solver on the LDS-tiled forward (dual step, gap terms, row-sum
    step sizes) follows the gather path to rounding: 60 FP64 iterations,
    single and batched (two instances sharing the geometry)."""
    d = desc_for(80, 24, 120)
    f = np.random.default_rng(3).standard_normal((24, 120)) * 0.05
    theta = to_dev(np.random.default_rng(4).uniform(-1, 1, (80, 80)), torch.float64)
    reg = pat.Reg(kind, 0.02, 0.04, eta=0.3, theta=theta if kind == "dtv" else None)
    res = {}
    for path in (0, 2):
        g = pat.Geometry(dtype=torch.float64, **d)
        g.set_forward_path(path)
        fd = to_dev(f, torch.float64)
        u, info, _ = pat.solve(g, fd, reg, max_iter=60, gap_tol=0.0, gap_every=20, graph_block=20)
        us, infos, _ = pat.solve_batched([(g, fd, reg), (g, fd * 0.5, reg)], max_iter=60, gap_tol=0.0,
                                         gap_every=20, graph_block=20)
        res[path] = (host(u), info["rel_gap"], host(us[1]), infos[1]["rel_gap"])
    assert rel(res[2][0], res[0][0]) <= 1e-11
    assert abs(res[2][1] - res[0][1]) <= 1e-9 * abs(res[0][1])
    assert rel(res[2][2], res[0][2]) <= 1e-11
    assert abs(res[2][3] - res[0][3]) <= 1e-9 * abs(res[0][3])


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("name", ["tv64", "ragged"])
def test_tiled_workgroup_shapes(name, dt):
    """Every workgroup shape of the tiled adjoint (4/8/16 waves, 16/64 lanes
    per row) matches the oracle, with quarter-turn storage (tv64) and
    without (ragged)."""
    d, og, g = _geoms(name, dt)
    A = OG.forward_matrix(og)
    y = np.random.default_rng(12).standard_normal(og.n_bins)
    ref = A.T @ y
    yd = to_dev(y.reshape(og.n_det, og.n_t), DT[dt])
    g.set_adjoint("tiled")
    assert g.info["csr_rot"] == (4 if name == "tv64" else 1)
    for waves in (4, 8, 16):
        for lanes in (16, 64):
            g.set_tiled_launch(waves, lanes)
            e = rel(host(g.adjoint(yd)), ref)
            assert e <= TOL_APPLY[dt], (waves, lanes, e)
    with pytest.raises(RuntimeError):
        g.set_tiled_launch(2, 16)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_forward_padded_and_partials_entry_points(dt):
    """pat_forward_padded on the zero-bordered image equals pat_forward; with
    the full stored matrix (no quarter turns) the one partial image is the
    adjoint; the matrix-free mode has no partials."""
    d, og, g = _geoms("ragged", dt)
    u = to_dev(np.random.default_rng(6).standard_normal((og.ny, og.nx)), DT[dt])
    upad = torch.zeros((og.ny + 2, og.nx + 2), dtype=DT[dt], device="cuda")
    upad[1:-1, 1:-1] = u
    assert np.array_equal(host(g.forward_padded(upad)), host(g.forward(u)))
    y = to_dev(np.random.default_rng(7).standard_normal((og.n_det, og.n_t)), DT[dt])
    g.set_adjoint("tiled")
    assert g.info["csr_rot"] == 1
    assert np.array_equal(host(g.adjoint_partials(y))[0], host(g.adjoint(y)))
    g.set_adjoint("scatter")
    with pytest.raises(RuntimeError):
        g.adjoint_partials(y, torch.zeros((1, og.ny, og.nx), dtype=DT[dt], device="cuda"))


@pytest.mark.parametrize("launch", [(4, 16, 1), (5, 32, 3), (6, 64, 7)])
def test_launch_shapes_agree_with_oracle(launch):
    d, og, g = _geoms("ragged", "f32")
    g.set_launch(*launch)
    g.set_adjoint("scatter")
    A = OG.forward_matrix(og)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(og.n_pix)
    y = rng.standard_normal(og.n_bins)
    fu = host(g.forward(to_dev(u.reshape(og.ny, og.nx), torch.float32)))
    aty = host(g.adjoint(to_dev(y.reshape(og.n_det, og.n_t), torch.float32)))
    ef, ea = rel(fu, A @ u), rel(aty, A.T @ y)
    assert ef <= 1e-5 and ea <= 1e-5, (ef, ea)


@pytest.mark.parametrize("adj", ["tiled", "csr", "scatter"])
def test_adjoint_is_deterministic(adj):
    d = desc_for(96, 40, 150)
    g = pat.Geometry(dtype=torch.float32, **d)
    g.set_adjoint(adj)
    y = to_dev(np.random.default_rng(2).standard_normal((40, 150)), torch.float32)
    a = host(g.adjoint(y))
    b = host(g.adjoint(y))
    assert np.array_equal(a, b)


def test_csr_matches_oracle_matrix_structure():
    """The stored A^T has the oracle's sparsity (exact zeros dropped) and values."""
    d, og, g = _geoms("arc90", "f64")
    A = OG.forward_matrix(og)
    A.eliminate_zeros()
    assert g.info["csr_nnz"] == A.nnz


def _quarter_turn_symmetric(d):
    """A closed ring of 4m detectors about the centre of a square grid."""
    return (d["nx"] == d["ny"] and d["n_det"] % 4 == 0 and d.get("det_xy") is None
            and abs(d["arc_span"] - 2 * math.pi) < 1e-12 and d["det_cx"] == 0.0
            and d["det_cy"] == 0.0 and d["x_min"] == -d["x_max"] and d["y_min"] == -d["y_max"])


def _expected_tiles(A, nx, ny, n_det, n_t, esz, rot=1):
    """Tile side and largest window of the LDS-staged adjoint: per tile of
    side x side pixels and detector, the run of radii its non-zeros span; the
    first side (8, then 4) whose largest per-tile sum of runs over the stored
    detectors (the first n_det/rot) fits 16-bit offsets and, times rot slots,
    64 KB, else no tiles."""
    n_det //= rot
    At = A[:n_det * n_t].T.tocsr()
    At.eliminate_zeros()
    for side in (8, 4):
        tx, ty = -(-nx // side), -(-ny // side)
        wmax = 0
        for t in range(tx * ty):
            lo = np.full(n_det, n_t)
            hi = np.full(n_det, -1)
            for r in range(side * side):
                i, j = (t % tx) * side + r % side, (t // tx) * side + r // side
                if i < nx and j < ny:
                    cols = At.indices[At.indptr[j * nx + i]:At.indptr[j * nx + i + 1]]
                    np.minimum.at(lo, cols // n_t, cols % n_t)
                    np.maximum.at(hi, cols // n_t, cols % n_t)
            wmax = max(wmax, int(np.sum(np.where(hi >= 0, hi - lo + 1, 0))))
        if 1 <= wmax <= 65535 and wmax * esz * rot <= 65536:
            return side, wmax
    return 0, 0


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(64, 16, 3500), (64, 16, 8000), (37, 7, 53)])
def test_tile_choice_and_tiled_adjoint(shape, dt):
    """Long windows (fine time sampling): 8x8 tiles, 4x4 tiles or the plain
    CSR, as the LDS budget allows; the adjoint matches the oracle in each."""
    n, n_det, n_t = shape
    d = desc_for(n, n_det, n_t)
    og = OG.make_geometry(d)
    A = OG.forward_matrix(og)
    rot = 4 if _quarter_turn_symmetric(d) else 1
    side, wmax = _expected_tiles(A, n, n, n_det, n_t, 8 if dt == "f64" else 4, rot)
    print(f"tiles {shape} {dt}: expected side {side} window {wmax} rot {rot}", flush=True)
    g = pat.Geometry(dtype=DT[dt], **d)
    info = g.info
    assert (info["sym_rot"], info["csr_rot"]) == (rot, rot)
    assert (info["csr_tile_side"], info["csr_win_max"]) == (side, wmax)
    assert info["adj_mode"] == (2 if side else 1)
    y = np.random.default_rng(4).standard_normal(og.n_bins)
    aty = host(g.adjoint(to_dev(y.reshape(n_det, n_t), DT[dt])))
    assert rel(aty, A.T @ y) <= TOL_APPLY[dt]


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(64, 32, 128), (45, 12, 70)])
def test_quarter_turn_storage(shape, dt):
    """A ring of 4m detectors about a square grid: the stored A^T keeps the
    rows of the first m detectors only (exactly the oracle's non-zeros of
    those rows) and the quarter-turn adjoint (tiled and plain) matches the
    oracle's A^T and the fully stored matrix; a ring that is not symmetric
    (shifted centre) stores every detector."""
    n, n_det, n_t = shape
    d = desc_for(n, n_det, n_t)
    og = OG.make_geometry(d)
    A = OG.forward_matrix(og)
    A.eliminate_zeros()
    y = np.random.default_rng(9).standard_normal(og.n_bins)
    ref = A.T @ y
    print(f"quarter turns {shape} {dt}", flush=True)
    g = pat.Geometry(dtype=DT[dt], **d)
    info = g.info
    assert (info["sym_rot"], info["csr_rot"]) == (4, 4)
    assert info["csr_nnz"] == A[:(n_det // 4) * n_t].nnz
    yd = to_dev(y.reshape(n_det, n_t), DT[dt])
    out = {}
    for adj in ("tiled", "csr"):
        g.set_adjoint(adj)
        out[adj] = host(g.adjoint(yd))
        assert rel(out[adj], ref) <= TOL_APPLY[dt], adj
    # the partial images sum (in order) to the adjoint, bit for bit, in both
    # stored modes; partial r holds the data of detectors r n_det/4 ..
    for adj in ("tiled", "csr"):
        g.set_adjoint(adj)
        parts = g.adjoint_partials(yd)
        assert tuple(parts.shape) == (4, n, n)
        acc = torch.zeros_like(parts[0])
        for r in range(4):
            acc = acc + parts[r]
        assert np.array_equal(host(acc), out[adj]), adj
        q = n_det // 4
        for r in (0, 3):
            yr = np.zeros_like(y).reshape(n_det, n_t)
            yr[r * q:(r + 1) * q] = y.reshape(n_det, n_t)[r * q:(r + 1) * q]
            assert rel(host(parts[r]), A.T @ yr.ravel()) <= TOL_APPLY[dt], (adj, r)
    g.set_symmetry(False)
    assert (g.info["sym_rot"], g.info["csr_rot"], g.info["csr_nnz"]) == (4, 1, A.nnz)
    for adj in ("tiled", "csr"):
        g.set_adjoint(adj)
        full = host(g.adjoint(yd))
        assert rel(full, out[adj]) <= TOL_APPLY[dt], adj
    g.set_symmetry(True)
    assert g.info["csr_rot"] == 4
    g2 = pat.Geometry(dtype=DT[dt], **dict(d, det_cx=0.01))
    assert (g2.info["sym_rot"], g2.info["csr_rot"]) == (1, 1)


FULL = {
    "tgv256": (256, 256, 512, 2 * math.pi),
    "dtv512": (512, 128, 1024, math.pi / 2),
}


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("adj", ["tiled", "csr", "scatter"])
@pytest.mark.parametrize("name", list(FULL))
def test_full_size_sampled_rows_columns_and_dot(name, adj, dt):
    """Workload sizes: sampled rows of A and columns of A (= rows of A^T)
    from the oracle, plus the dot-product identity over the whole operator;
    with the quarter-turn storage also each partial image (the data of one
    quarter of the ring) on the sampled pixels."""
    n, n_det, n_t, span = FULL[name]
    d = desc_for(n, n_det, n_t, arc_span=span)
    og = OG.make_geometry(d)
    g = pat.Geometry(dtype=DT[dt], **d)
    g.set_adjoint(adj)
    tol = TOL_APPLY[dt]
    rng = np.random.default_rng(21)
    u = rng.standard_normal((n, n))
    y = rng.standard_normal((n_det, n_t))
    print(f"case {name} {dt} {adj}: forward/adjoint at {n}^2, {n_det}x{n_t}", flush=True)
    yd = to_dev(y, DT[dt])
    fu = host(g.forward(to_dev(u, DT[dt]))).ravel()
    aty = host(g.adjoint(yd)).ravel()
    bins = np.sort(rng.choice(og.n_bins, 96, replace=False))
    ref_rows = OG.forward_rows(og, bins) @ u.ravel()
    er = rel(fu[bins], ref_rows)
    assert er <= tol, er
    pix = np.sort(rng.choice(og.n_pix, 12, replace=False))
    cols = [column_of_A(og, j) for j in pix]
    ref_cols = np.array([c @ y.ravel() for c in cols])
    ec = rel(aty[pix], ref_cols)
    assert ec <= tol, ec
    lhs = float(fu @ y.ravel())
    rhs = float(u.ravel() @ aty)
    assert abs(lhs - rhs) <= tol * np.linalg.norm(fu) * np.linalg.norm(y)
    rot = g.info["csr_rot"]
    if adj != "scatter" and rot > 1:
        parts = host(g.adjoint_partials(yd)).reshape(rot, -1)
        qd = n_det // rot
        for r in range(rot):
            sl = slice(r * qd * n_t, (r + 1) * qd * n_t)
            ref_part = np.array([c[sl] @ y.ravel()[sl] for c in cols])
            ep = rel(parts[r][pix], ref_part)
            assert ep <= tol, (r, ep)


_TGV256 = {}


def _tgv256_oracle():
    """The oracle's A at 256^2 / 256 x 512 (built once: about a minute)."""
    if not _TGV256:
        d = desc_for(256, 256, 512)
        _TGV256["d"] = d
        _TGV256["A"] = OG.forward_matrix(OG.make_geometry(d))
    return _TGV256["d"], _TGV256["A"]


@pytest.mark.timeout(600)
def test_tgv256_f64_full_state_after_20_iterations():
    """The headline configuration in its own precision and size: FP64 TGV
    (alpha1 0.02, alpha0 0.04) at 256^2 with 256 detectors x 512 samples, the
    solver's default launch (quarter-turn tiled A^T, gather forward with the
    fused dual steps), 20 iterations from zero on vessel-phantom data, against
    the oracle's full state (u, ubar, q, r, v, vbar, s) and gap terms."""
    d, A = _tgv256_oracle()
    print("tgv256 f64: oracle matrix built", flush=True)
    # data from the reconstruction grid's own operator (the finer synthesis
    # grid would cost minutes of oracle time; parity does not need it)
    case = phantoms.make_case("vessel", 256, 100, 256, 512)
    fc = A @ case["u_gt"].ravel()
    f = fc + 0.10 * np.linalg.norm(fc) / math.sqrt(fc.size) * case["noise"].ravel()
    p = oracle_problem(A, f, 256, "tgv", 0.02, 0.04)
    ref = OP.pdhg_solve(p, OP.precond_diag(p), iters=20)
    g = pat.Geometry(dtype=torch.float64, **d)
    assert g.info["csr_rot"] == 4 and g.info["adj_mode"] == 2
    st = torch.zeros(g.state_elems("tgv"), dtype=torch.float64, device="cuda")
    u, info, status = pat.solve(g, to_dev(f, torch.float64), pat.Reg("tgv", 0.02, 0.04), max_iter=20,
                                gap_tol=0.0, gap_every=10, graph_block=10, state_out=st)
    assert info["iters"] == 20 and status == 0
    got = split_state(host(st), "tgv", p.N, A.shape[0])
    for key in ("u", "ubar", "q", "r", "v", "vbar", "s"):
        e = rel(got[key], ref[key])
        print(f"  {key}: rel {e:.2e}", flush=True)
        assert e <= 1e-10, (key, e)
    _assert_gap_terms(info, p, ref, "tgv", "f64")


# ------------------------------------------------------------------ step sizes

def _theta(n, ny=None, seed=3):
    ny = n if ny is None else ny
    return np.random.default_rng(seed).uniform(-1.5, 1.5, (ny, n))


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["tv", "tgv", "dtv", "tikhonov"])
def test_diag_preconditioner(kind, dt):
    d, og, g = _geoms("ragged", dt)
    A = OG.forward_matrix(og)
    th = _theta(og.nx, og.ny)
    p = oracle_problem(A, np.zeros(og.n_bins), og.nx, kind, 0.02, 0.04, 0.3, th, ny=og.ny)
    ref = OP.precond_diag(p)
    reg = pat.Reg(kind, 0.02, 0.04, 0.3, to_dev(th, DT[dt]) if kind == "dtv" else None)
    pc = pat.Precond(g, reg, "diag")
    # sigma_q = 1/(A 1): it carries the per-apply rounding of A (FP32 sums
    # of FP32 weights; positions and the cos/sin table are FP64)
    tol = 1e-12 if dt == "f64" else TOL_APPLY["f32"]
    errs = {"sigma_q": rel(host(pc.get("sigma_q")), ref["sigma_q"]),
            "tau_u": rel(host(pc.get("tau_u")), ref["tau_u"])}
    if kind != "tikhonov":
        errs["sigma_r"] = rel(host(pc.get("sigma_r")), ref["sigma_r"])
    if kind == "tgv":
        errs["sigma_s"] = rel(host(pc.get("sigma_s")), ref["sigma_s"])
        errs["tau_v"] = rel(host(pc.get("tau_v")), ref["tau_v"].ravel())
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("kind", ["tv", "tgv", "dtv"])
def test_block_preconditioner(kind):
    d, og, g = _geoms("arc90", "f64")
    A = OG.forward_matrix(og)
    th = _theta(og.nx)
    p = oracle_problem(A, np.zeros(og.n_bins), og.nx, kind, 0.02, 0.04, 0.3, th)
    ref = OP.precond_block(p)
    reg = pat.Reg(kind, 0.02, 0.04, 0.3, to_dev(th, torch.float64) if kind == "dtv" else None)
    pc = pat.Precond(g, reg, "block")
    assert host(pc.get("tau_u"))[0] == pytest.approx(ref["tau_u"][0], rel=1e-9)
    assert host(pc.get("sigma_q"))[0] == pytest.approx(ref["sigma_q"][0], rel=1e-9)
    assert host(pc.get("sigma_r"))[0] == pytest.approx(ref["sigma_r"][0], rel=1e-9)


# ------------------------------------------------------------------ PDHG iterations

def _reg_pair(kind, og, dt, lam=0.02):
    th = _theta(og.nx, og.ny)
    reg = pat.Reg(kind, lam, 2 * lam, 0.1, to_dev(th, DT[dt]) if kind == "dtv" else None)
    return reg, th


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["tv", "tgv", "dtv", "tikhonov"])
def test_fixed_iterations_full_state(kind, dt):
    """State after 60 iterations (u, ubar, q, r, v, vbar, s) against Alg. 1/2."""
    name = "arc90" if kind == "dtv" else "ragged"
    d, og, g = _geoms(name, dt)
    A = OG.forward_matrix(og)
    fam = {"tv": "disc", "tgv": "vessel", "dtv": "segment", "tikhonov": "disc"}[kind]
    rng = np.random.default_rng(4)
    f = A @ np.clip(rng.uniform(-0.2, 1, og.n_pix), 0, None) + 0.01 * rng.standard_normal(og.n_bins)
    reg, th = _reg_pair(kind, og, dt)
    p = oracle_problem(A, f, og.nx, kind, reg.lam, reg.alpha0, reg.eta, th, ny=og.ny)
    ref = OP.pdhg_solve(p, OP.precond_diag(p), iters=60)
    st = torch.zeros(g.state_elems(kind), dtype=DT[dt], device="cuda")
    u, info, status = pat.solve(g, to_dev(f, DT[dt]), reg, max_iter=60, gap_tol=0.0,
                               gap_every=10, graph_block=20, state_out=st)
    got = split_state(host(st), kind, og.n_pix, og.n_bins)
    tol = 1e-10 if dt == "f64" else 1e-4
    print(f"{kind} {dt}: rel u {rel(got['u'], ref['u']):.2e}", flush=True)
    assert info["iters"] == 60
    eu = rel(host(u), ref["u"])
    assert eu <= tol, eu
    for key in ("u", "ubar", "q", "r", "v", "vbar", "s"):
        if key in got and key in ref:
            e = rel(got[key], ref[key])
            assert e <= tol, (key, e)
    _assert_gap_terms(info, p, ref, kind, dt)


def _assert_gap_terms(info, p, ref, kind, dt):
    """P, F*, ||K^T y||_1 (LS-T: ||A^T q||^2), the gap and the residual of
    Sec. 3.3.3 reported by the library, each against the oracle's state."""
    g_ref = OP.gap_terms(p, ref, 2.0)
    res_ref = OP.residual(ref)
    f64 = dt == "f64"
    print(f"  P {info['primal']:.6e}/{g_ref['P']:.6e} F* {info['fstar']:.6e}/{g_ref['Fstar']:.6e} "
          f"R {info['kty_l1']:.6e}/{g_ref['R']:.6e} res {info['residual']:.6e}/{res_ref:.6e}", flush=True)
    assert info["primal"] == pytest.approx(g_ref["P"], rel=1e-9 if f64 else 1e-4)
    # F* = 1/2||q||^2 + <q, f> is a difference of O(P) terms: compare on the scale of P
    assert abs(info["fstar"] - g_ref["Fstar"]) <= (1e-10 if f64 else 1e-5) * g_ref["P"]
    # the library reports ||A^T q||^2 for LS-T (the oracle's R is that over 2 alpha)
    kty = info["kty_l1"] / (2.0 * p.lam) if kind == "tikhonov" else info["kty_l1"]
    assert kty == pytest.approx(g_ref["R"], rel=1e-8 if f64 else 1e-4)
    # near convergence the gap is a small difference of O(P) terms: compare on the scale of P
    assert abs(info["gap"] - g_ref["gap"]) <= (1e-10 if f64 else 1e-5) * g_ref["P"]
    # FP32: the change of u over one iteration is a difference of nearly
    # equal FP32 values (measured 6e-5 relative on the LS-T state)
    assert info["residual"] == pytest.approx(res_ref, rel=1e-8 if f64 else 1e-3)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("kind", ["tv", "tgv", "dtv", "tikhonov"])
def test_accelerated_fixed_iterations_full_state(kind, dt):
    """Accelerated PDHGM (step multipliers and theta_n of the schedule, frozen
    at a dual-step factor of 3 after four updates) for 60 iterations across
    three graph blocks: full state and gap terms against the oracle."""
    name = "arc90" if kind == "dtv" else "ragged"
    d, og, g = _geoms(name, dt)
    A = OG.forward_matrix(og)
    rng = np.random.default_rng(14)
    f = A @ np.clip(rng.uniform(-0.2, 1, og.n_pix), 0, None) + 0.01 * rng.standard_normal(og.n_bins)
    reg, th = _reg_pair(kind, og, dt)
    p = oracle_problem(A, f, og.nx, kind, reg.lam, reg.alpha0, reg.eta, th, ny=og.ny)
    ref = OP.pdhg_solve(p, OP.precond_diag(p), iters=60, accel_gamma=0.5, accel_step_max=3.0)
    st = torch.zeros(g.state_elems(kind), dtype=DT[dt], device="cuda")
    u, info, status = pat.solve(g, to_dev(f, DT[dt]), reg, max_iter=60, gap_tol=0.0, gap_every=10,
                                graph_block=20, state_out=st, accel_gamma=0.5, accel_step_max=3.0)
    got = split_state(host(st), kind, og.n_pix, og.n_bins)
    tol = 1e-10 if dt == "f64" else 1e-4
    print(f"accelerated {kind} {dt}: rel u {rel(got['u'], ref['u']):.2e}", flush=True)
    assert info["iters"] == 60
    for key in ("u", "ubar", "q", "r", "v", "vbar", "s"):
        if key in got and key in ref:
            e = rel(got[key], ref[key])
            assert e <= tol, (key, e)
    _assert_gap_terms(info, p, ref, kind, dt)


def test_accelerated_converges_like_the_oracle():
    """Accelerated solve to a gap tolerance (gap every 50): the same stopping
    iteration and objective as the oracle's accelerated run."""
    d = desc_for(48, 24, 96)
    og = OG.make_geometry(d)
    A = OG.forward_matrix(og)
    f, _ = synth_data(d, "disc", 5)
    p = oracle_problem(A, f, 48, "tv", 0.01)
    ref = OP.pdhg_solve(p, OP.precond_diag(p), tol=1e-3, max_iter=20000, gap_every=50,
                        accel_gamma=1.0, accel_step_max=4.0)
    g = pat.Geometry(dtype=torch.float64, **d)
    u, info, st = pat.solve(g, to_dev(f, torch.float64), pat.Reg("tv", 0.01), max_iter=20000, gap_tol=1e-3,
                            gap_every=50, graph_block=50, accel_gamma=1.0, accel_step_max=4.0)
    print(f"accelerated: iters {info['iters']} (oracle {ref['history'][-1]['n']})", flush=True)
    assert st == 0 and info["iters"] == ref["history"][-1]["n"]
    assert info["primal"] == pytest.approx(ref["history"][-1]["P"], rel=1e-9)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_accelerated_and_plain_in_one_batch(dt):
    """A batch mixing accelerated and plain instances (two sharing a
    geometry): every instance equals its single solve bit for bit."""
    d, og, g = _geoms("ragged", dt)
    A = OG.forward_matrix(og)
    rng = np.random.default_rng(31)
    problems, accel = [], []
    for i, kind in enumerate(["tv", "tgv", "tv"]):
        f = A @ rng.uniform(0, 1, og.n_pix)
        problems.append((g, to_dev(f, DT[dt]), pat.Reg(kind, 0.02, 0.04)))
        accel.append((0.5 * i, 3.0) if i else (0.0, 1.0))
    us, infos, st = pat.solve_batched(problems, max_iter=120, gap_tol=0.0, gap_every=20, graph_block=40,
                                      accel=accel)
    for (gg, f, reg), (ag, am), ub, ib in zip(problems, accel, us, infos):
        u1, i1, _ = pat.solve(gg, f, reg, max_iter=120, gap_tol=0.0, gap_every=20, graph_block=40,
                              accel_gamma=ag, accel_step_max=am)
        assert torch.equal(ub, u1), (reg.kind, ag)
        assert ib["rel_gap"] == i1["rel_gap"]


@pytest.mark.parametrize("adj", ["tiled", "csr", "scatter"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_tv64_workload_200_iterations(dt, adj):
    """The 64^2 TV workload: lambda 0.05, DIAG, 200 iterations from zero, on
    disc-phantom data synthesised on the 128^2 grid with 5% noise (each
    adjoint path of the solver)."""
    d = desc_for(64, 32, 128)
    og = OG.make_geometry(d)
    A = OG.forward_matrix(og)
    g = pat.Geometry(dtype=DT[dt], **d)
    g.set_adjoint(adj)
    for seed in (0, 1):
        f, _ = synth_data(d, "disc", seed)
        p = oracle_problem(A, f, 64, "tv", 0.05)
        ref = OP.pdhg_solve(p, OP.precond_diag(p), iters=200)
        u, info, _ = pat.solve(g, to_dev(f, DT[dt]), pat.Reg("tv", 0.05), max_iter=200,
                               gap_tol=0.0, gap_every=50, graph_block=50)
        e = rel(host(u), ref["u"])
        print(f"tv64 {dt} {adj} seed {seed}: rel L2 image {e:.3e}", flush=True)
        assert e <= (1e-10 if dt == "f64" else 1e-3)


def test_resume_is_bitwise():
    d, og, g = _geoms("ragged", "f32")
    A = OG.forward_matrix(og)
    f = A @ np.random.default_rng(8).uniform(0, 1, og.n_pix)
    reg = pat.Reg("tgv", 0.01, 0.02)
    fd = to_dev(f, torch.float32)
    n_st = g.state_elems("tgv")
    full = torch.zeros(n_st, dtype=torch.float32, device="cuda")
    half = torch.zeros(n_st, dtype=torch.float32, device="cuda")
    again = torch.zeros(n_st, dtype=torch.float32, device="cuda")
    pat.solve(g, fd, reg, max_iter=100, gap_tol=0.0, gap_every=10, graph_block=50, state_out=full)
    pat.solve(g, fd, reg, max_iter=50, gap_tol=0.0, gap_every=10, graph_block=50, state_out=half)
    pat.solve(g, fd, reg, max_iter=50, gap_tol=0.0, gap_every=10, graph_block=50,
              state_in=half, state_out=again)
    assert np.array_equal(host(full), host(again))


def test_graph_and_direct_launches_agree():
    d, og, g = _geoms("arc90", "f32")
    A = OG.forward_matrix(og)
    f = to_dev(A @ np.random.default_rng(9).uniform(0, 1, og.n_pix), torch.float32)
    reg = pat.Reg("tv", 0.01)
    a, ia, _ = pat.solve(g, f, reg, max_iter=80, gap_tol=0.0, gap_every=10, graph_block=40)
    b, ib, _ = pat.solve(g, f, reg, max_iter=80, gap_tol=0.0, gap_every=10, graph_block=0)
    assert np.array_equal(host(a), host(b))
    assert ia["gap"] == ib["gap"]


def test_warm_start_and_fallback():
    d, og, g = _geoms("tv64", "f64")
    A = OG.forward_matrix(og)
    f, _ = synth_data(d, "disc", 3)
    p = oracle_problem(A, f, 64, "tv", 0.05)
    pc = OP.precond_diag(p)
    fd = to_dev(f, torch.float64)
    reg = pat.Reg("tv", 0.05)
    good = OP.pdhg_solve(p, pc, iters=100)["u"]
    ref = OP.pdhg_solve(p, pc, iters=40, u0=good)
    u, info, _ = pat.solve(g, fd, reg, max_iter=40, gap_tol=0.0, gap_every=10, graph_block=20,
                           u0=to_dev(good.reshape(64, 64), torch.float64))
    assert info["fallback"] == 0 and rel(host(u), ref["u"]) <= 1e-10
    zero = OP.pdhg_solve(p, pc, iters=40)["u"]
    for bad in (np.full((64, 64), np.nan), np.full((64, 64), 1e3)):
        assert OP.warm_start_rejected(p, bad.ravel())
        u, info, _ = pat.solve(g, fd, reg, max_iter=40, gap_tol=0.0, gap_every=10,
                               graph_block=20, u0=to_dev(bad, torch.float64))
        assert info["fallback"] == 1 and rel(host(u), zero) <= 1e-10


def test_dual_warm_start_and_fallback():
    """A start (u0, q0, r0) runs the oracle's iteration from the same state
    (ubar0 = u0); a non-finite dual start falls back to zero."""
    d, og, g = _geoms("tv64", "f64")
    A = OG.forward_matrix(og)
    f, _ = synth_data(d, "disc", 3)
    p = oracle_problem(A, f, 64, "tv", 0.05)
    pc = OP.precond_diag(p)
    fd = to_dev(f, torch.float64)
    reg = pat.Reg("tv", 0.05)
    good = OP.pdhg_solve(p, pc, iters=100)
    st = OP.init_state(p, good["u"])
    st["q"], st["r"] = good["q"].copy(), good["r"].copy()
    ref = OP.pdhg_solve(p, pc, iters=40, state=st)
    y0 = np.concatenate([good["q"], good["r"].ravel()])
    n_state = g.state_elems("tv")
    so = torch.empty(n_state, dtype=torch.float64, device="cuda")
    u, info, _ = pat.solve(g, fd, reg, max_iter=40, gap_tol=0.0, gap_every=10, graph_block=20,
                           u0=to_dev(good["u"].reshape(64, 64), torch.float64),
                           y0=to_dev(y0, torch.float64), state_out=so)
    assert info["fallback"] == 0 and rel(host(u), ref["u"]) <= 1e-10
    got = split_state(host(so), "tv", 64 * 64, A.shape[0])
    assert rel(got["q"], ref["q"]) <= 1e-10 and rel(got["r"], ref["r"]) <= 1e-10
    zero = OP.pdhg_solve(p, pc, iters=40)["u"]
    bad = y0.copy()
    bad[7] = np.nan
    u, info, _ = pat.solve(g, fd, reg, max_iter=40, gap_tol=0.0, gap_every=10, graph_block=20,
                           u0=to_dev(good["u"].reshape(64, 64), torch.float64),
                           y0=to_dev(bad, torch.float64))
    assert info["fallback"] == 1 and rel(host(u), zero) <= 1e-10
    with pytest.raises(pat.L.PatError):
        pat.solve(g, fd, pat.Reg("tgv", 0.05, 0.1), max_iter=10,
                  u0=to_dev(good["u"].reshape(64, 64), torch.float64), y0=to_dev(y0, torch.float64))


def test_converges_to_gap_and_matches_oracle_objective():
    """Run to a gap tolerance: same stopping iteration as the oracle (up to one
    check interval, the FP32 gap rounding near the threshold) and the same
    objective."""
    d = desc_for(48, 24, 96)
    og = OG.make_geometry(d)
    A = OG.forward_matrix(og)
    f, _ = synth_data(d, "disc", 5)
    p = oracle_problem(A, f, 48, "tv", 0.01)
    ref = OP.pdhg_solve(p, OP.precond_diag(p), tol=1e-3, max_iter=20000, gap_every=50)
    assert ref["history"][-1]["rel_gap"] <= 1e-3
    for dt in ("f64", "f32"):
        g = pat.Geometry(dtype=DT[dt], **d)
        u, info, st = pat.solve(g, to_dev(f, DT[dt]), pat.Reg("tv", 0.01), max_iter=20000,
                                gap_tol=1e-3, gap_every=50, graph_block=50)
        print(f"{dt}: iters {info['iters']} (oracle {ref['history'][-1]['n']}) "
              f"rel_gap {info['rel_gap']:.3e}", flush=True)
        assert st == 0 and info["converged"] == 1 and info["rel_gap"] <= 1e-3
        if dt == "f64":
            assert info["iters"] == ref["history"][-1]["n"]
        else:
            assert abs(info["iters"] - ref["history"][-1]["n"]) <= 50
        assert info["primal"] == pytest.approx(ref["history"][-1]["P"], rel=1e-4)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_batched_matches_single_solves(dt):
    """Mixed sizes and regularisers in one batch; two instances share a
    geometry (one pass over its stored A^T serves both)."""
    problems, singles = [], []
    specs = [("ragged", "tv", 0.01), ("arc90", "tgv", 0.01), ("tv64", "dtv", 0.02),
             ("ragged", "tgv", 0.005)]
    shared = None
    for name, kind, lam in specs:
        if name == "ragged" and shared is not None:
            d, og, g = shared
        else:
            d, og, g = _geoms(name, dt)
            if name == "ragged":
                shared = (d, og, g)
        A = OG.forward_matrix(og)
        f = to_dev(A @ np.random.default_rng(len(problems)).uniform(0, 1, og.n_pix), DT[dt])
        reg, _ = _reg_pair(kind, og, dt, lam)
        problems.append((g, f, reg))
    us, infos, st = pat.solve_batched(problems, max_iter=300, gap_tol=1e-3, gap_every=10,
                                      graph_block=50)
    for (g, f, reg), u, info in zip(problems, us, infos):
        u1, i1, _ = pat.solve(g, f, reg, max_iter=300, gap_tol=1e-3, gap_every=10, graph_block=50)
        assert info["iters"] == i1["iters"]
        assert np.array_equal(host(u), host(u1))


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_batched_shared_geometry_four_right_hand_sides(dt):
    """Four instances on one geometry: one tiled pass over A^T serves all four
    (in FP64 their staged windows need more than 64 KB of LDS); each result is
    bitwise the single-instance solve, which matches the oracle."""
    d = desc_for(128, 128, 256)
    og = OG.make_geometry(d)
    A = OG.forward_matrix(og)
    g = pat.Geometry(dtype=DT[dt], **d)
    info = g.info
    esz = 8 if dt == "f64" else 4
    print(f"tiles {info['csr_tile_side']} window {info['csr_win_max']} -> "
          f"{4 * info['csr_win_max'] * esz} B of LDS for 4 right-hand sides", flush=True)
    assert info["adj_mode"] == 2
    rng = np.random.default_rng(12)
    fs = [A @ rng.uniform(0, 1, og.n_pix) for _ in range(4)]
    reg = pat.Reg("tv", 0.01)
    problems = [(g, to_dev(f, DT[dt]), reg) for f in fs]
    us, infos, st = pat.solve_batched(problems, max_iter=60, gap_tol=0.0, gap_every=20, graph_block=20)
    for (g_, f, reg_), u, info in zip(problems, us, infos):
        u1, i1, _ = pat.solve(g, f, reg, max_iter=60, gap_tol=0.0, gap_every=20, graph_block=20)
        assert info["iters"] == i1["iters"] == 60
        assert np.array_equal(host(u), host(u1))
        assert info["rel_gap"] == i1["rel_gap"]
    p = oracle_problem(A, fs[3], 128, "tv", 0.01)
    ref = OP.pdhg_solve(p, OP.precond_diag(p), iters=60)
    assert rel(host(us[3]), ref["u"]) <= (1e-10 if dt == "f64" else 1e-3)


def test_batched_on_four_pixel_tiles():
    """A geometry whose windows only fit 4x4 tiles (fine time sampling), two
    instances sharing it: the multi-right-hand-side tiled pass equals the
    single solves bitwise and the oracle."""
    d = desc_for(64, 16, 3500)
    og = OG.make_geometry(d)
    A = OG.forward_matrix(og)
    g = pat.Geometry(dtype=torch.float64, **d)
    assert (g.info["adj_mode"], g.info["csr_tile_side"]) == (2, 4)
    rng = np.random.default_rng(14)
    fs = [A @ rng.uniform(0, 1, og.n_pix) for _ in range(2)]
    reg = pat.Reg("tv", 0.01)
    problems = [(g, to_dev(f, torch.float64), reg) for f in fs]
    us, infos, st = pat.solve_batched(problems, max_iter=40, gap_tol=0.0, gap_every=20, graph_block=20)
    for (g_, f, reg_), u in zip(problems, us):
        u1, _, _ = pat.solve(g, f, reg, max_iter=40, gap_tol=0.0, gap_every=20, graph_block=20)
        assert np.array_equal(host(u), host(u1))
    p = oracle_problem(A, fs[1], 64, "tv", 0.01)
    ref = OP.pdhg_solve(p, OP.precond_diag(p), iters=40)
    assert rel(host(us[1]), ref["u"]) <= 1e-10



@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_batched_bitwise_with_long_rows(dt):
    """A geometry without quarter-turn storage (one slot, rows of about 110
    entries, several per lane) batched with a quarter-turn geometry (four
    slots): the shared tiled launch then carries four slots for both, and the
    long-row instance still equals its single solve bitwise, because each
    slot's summation order does not depend on how many slots a launch
    carries."""
    d_long = desc_for(36, 18, 120)
    og = OG.make_geometry(d_long)
    A = OG.forward_matrix(og)
    g_long = pat.Geometry(dtype=DT[dt], **d_long)
    d4, og4, g4 = _geoms("tv64", dt)
    assert g_long.info["csr_rot"] == 1 and g4.info["csr_rot"] == 4
    assert g_long.info["adj_mode"] == 2 and g4.info["adj_mode"] == 2
    rng = np.random.default_rng(15)
    fl = A @ rng.uniform(0, 1, og.n_pix)
    f_long = to_dev(fl, DT[dt])
    f4 = to_dev(OG.forward_matrix(og4) @ rng.uniform(0, 1, og4.n_pix), DT[dt])
    reg = pat.Reg("tv", 0.01)
    problems = [(g4, f4, reg), (g_long, f_long, reg)]
    us, infos, st = pat.solve_batched(problems, max_iter=40, gap_tol=0.0, gap_every=20, graph_block=20)
    for (g, f, reg_), u in zip(problems, us):
        u1, _, _ = pat.solve(g, f, reg, max_iter=40, gap_tol=0.0, gap_every=20, graph_block=20)
        assert np.array_equal(host(u), host(u1))
    p = oracle_problem(A, fl, 36, "tv", 0.01)
    ref = OP.pdhg_solve(p, OP.precond_diag(p), iters=40)
    assert rel(host(us[1]), ref["u"]) <= (1e-10 if dt == "f64" else 1e-3)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_batched_three_on_one_geometry(dt):
    """Three instances on one geometry: each forward block serves all three
    (one position and cell per sample, taps from the three images), and each
    result is bitwise the single-instance solve, which matches the oracle."""
    d, og, g = _geoms("tv64", dt)
    A = OG.forward_matrix(og)
    rng = np.random.default_rng(16)
    fs = [A @ rng.uniform(0, 1, og.n_pix) for _ in range(3)]
    regs = [pat.Reg("tv", 0.01), pat.Reg("tgv", 0.01, 0.02), pat.Reg("tv", 0.02)]
    problems = [(g, to_dev(f, DT[dt]), r) for f, r in zip(fs, regs)]
    us, infos, st = pat.solve_batched(problems, max_iter=60, gap_tol=0.0, gap_every=20, graph_block=20)
    for (g_, f, r), u, info in zip(problems, us, infos):
        u1, i1, _ = pat.solve(g, f, r, max_iter=60, gap_tol=0.0, gap_every=20, graph_block=20)
        assert np.array_equal(host(u), host(u1))
        # the gap terms come from the shared forward block too
        assert info["rel_gap"] == i1["rel_gap"]
    p = oracle_problem(A, fs[0], 64, "tv", 0.01)
    ref = OP.pdhg_solve(p, OP.precond_diag(p), iters=60)
    assert rel(host(us[0]), ref["u"]) <= (1e-10 if dt == "f64" else 1e-3)

def test_autotune_and_cache(tmp_path):
    d, og, g = _geoms("arc90", "f32")
    path = str(tmp_path / "tune.txt")
    r1 = g.autotune(path, reps=3)
    assert r1["from_cache"] == 0 and r1["fwd_lanes_log2"] in (4, 5, 6)
    assert open(path).read().count("\n") == 1
    g2 = pat.Geometry(dtype=torch.float32, **d)
    r2 = g2.autotune(path, reps=3)
    assert r2["from_cache"] == 1
    assert (r2["fwd_lanes_log2"], r2["adj_mode"], r2["adj_tile"], r2["adj_det_group"]) == \
        (r1["fwd_lanes_log2"], r1["adj_mode"], r1["adj_tile"], r1["adj_det_group"])
    A = OG.forward_matrix(og)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(og.n_pix)
    y = rng.standard_normal(og.n_bins)
    fu = host(g2.forward(to_dev(u.reshape(og.ny, og.nx), torch.float32)))
    aty = host(g2.adjoint(to_dev(y.reshape(og.n_det, og.n_t), torch.float32)))
    ef, ea = rel(fu, A @ u), rel(aty, A.T @ y)
    assert ef <= 1e-5 and ea <= 1e-5, (ef, ea)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_batched_64_lane_rows_beside_short_rows_against_oracle(dt):
    """A geometry whose stored rows average more than 512 entries (many
    detectors on a half arc, stored in full) makes a batched launch use 64
    lanes per row for every geometry in it; batched beside two short-row
    geometries (one quarter-turn symmetric) and mixed regularisers, every
    instance is compared with the oracle's iterates."""
    d_long = desc_for(24, 168, 48, arc_span=math.pi)
    d_mid = desc_for(40, 12, 70)
    d_rag = _desc("ragged")
    rng = np.random.default_rng(41)
    cases = []
    for d, kind in ((d_long, "tv"), (d_mid, "tgv"), (d_rag, "dtv")):
        og = OG.make_geometry(d)
        A = OG.forward_matrix(og)
        g = pat.Geometry(dtype=DT[dt], **d)
        f = A @ np.clip(rng.uniform(-0.2, 1, og.n_pix), 0, None)
        reg, th = _reg_pair(kind, og, dt)
        cases.append((g, og, A, f, reg, th, kind))
    g_long = cases[0][0]
    mean_row = g_long.info["csr_nnz"] / (24 * 24)
    print(f"long rows: mean {mean_row:.0f} entries, rot {g_long.info['csr_rot']}", flush=True)
    assert mean_row >= 512 and g_long.info["csr_rot"] == 1 and cases[1][0].info["csr_rot"] == 4
    problems = [(c[0], to_dev(c[3], DT[dt]), c[4]) for c in cases]
    us, infos, st = pat.solve_batched(problems, max_iter=60, gap_tol=0.0, gap_every=20, graph_block=20)
    for (g, og, A, f, reg, th, kind), u in zip(cases, us):
        p = oracle_problem(A, f, og.nx, kind, reg.lam, reg.alpha0, reg.eta, th, ny=og.ny)
        ref = OP.pdhg_solve(p, OP.precond_diag(p), iters=60)
        e = rel(host(u), ref["u"])
        print(f"  {kind} {og.nx}x{og.ny}: rel {e:.2e}", flush=True)
        assert e <= (1e-10 if dt == "f64" else 1e-3), (kind, e)
