"""Failure statuses of the C ABI (include/pat.h): invalid arguments are
rejected before any device work with outputs untouched, a non-finite gap
stops the solve with PAT_ERR_NUMERIC and outputs untouched, and the iteration
cap returns the PAT_NOT_CONVERGED warning with valid outputs and a filled
pat_solve_info."""
import ctypes as C
import math

import numpy as np
import pytest
import torch

from gpu_common import desc_for, to_dev

pytestmark = pytest.mark.gpu

pat = pytest.importorskip("paper_1707_02245_amd.pat")
L = pat.L

SENTINEL = 7.25


@pytest.fixture(scope="module")
def setup():
    d = desc_for(24, 8, 48)
    g = pat.Geometry(dtype=torch.float64, **d)
    rng = np.random.default_rng(3)
    u = torch.tensor(rng.uniform(0, 1, (24, 24)), dtype=torch.float64, device="cuda")
    f = g.forward(u)
    theta = torch.zeros(24 * 24, dtype=torch.float64, device="cuda")
    return g, f, theta


def _raw_solve(g, f, reg, opts, out):
    info = L.SolveInfo()
    info.iters = -1
    st = L.load().pat_pdhg_solve(g.handle, C.c_void_p(f.data_ptr()), C.byref(reg.c_struct()),
                                 C.byref(opts), C.c_void_p(out.data_ptr()), C.byref(info),
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st, info


def _opts(**kw):
    o = pat._opts(200, 1e-4, 50, 50, 1.0, 2.0, None, None, None, None)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


BAD = {
    "lambda<0": (dict(kind="tv", lam=-0.1), {}),
    "lambda nan": (dict(kind="tv", lam=math.nan), {}),
    "alpha0<0": (dict(kind="tgv", lam=0.02, alpha0=-1.0), {}),
    "eta=0": (dict(kind="dtv", lam=0.02, eta=0.0, theta=True), {}),
    "eta>1": (dict(kind="dtv", lam=0.02, eta=1.5, theta=True), {}),
    "dtv without theta": (dict(kind="dtv", lam=0.02, eta=0.1), {}),
    "tikhonov alpha 0": (dict(kind="tikhonov", lam=0.0), {}),
    "max_iter=0": (dict(kind="tv", lam=0.02), dict(max_iter=0)),
    "max_iter<0": (dict(kind="tv", lam=0.02), dict(max_iter=-5)),
    "gap_every=0": (dict(kind="tv", lam=0.02), dict(gap_every=0)),
    "graph_block<0": (dict(kind="tv", lam=0.02), dict(graph_block=-1)),
    "gap_box=0": (dict(kind="tv", lam=0.02), dict(gap_box=0.0)),
    "gap_box<0": (dict(kind="tv", lam=0.02), dict(gap_box=-2.0)),
    "gap_tol nan": (dict(kind="tv", lam=0.02), dict(gap_tol=math.nan)),
    "theta>1": (dict(kind="tv", lam=0.02), dict(theta=1.5)),
    "accel_gamma<0": (dict(kind="tv", lam=0.02), dict(accel_gamma=-1.0, accel_step_max=4.0)),
    "accel_gamma inf": (dict(kind="tv", lam=0.02), dict(accel_gamma=math.inf, accel_step_max=4.0)),
    "accel_step_max<1": (dict(kind="tv", lam=0.02), dict(accel_gamma=1.0, accel_step_max=0.5)),
    "accel with theta<1": (dict(kind="tv", lam=0.02), dict(accel_gamma=1.0, accel_step_max=4.0, theta=0.5)),
}


@pytest.mark.parametrize("case", list(BAD))
def test_invalid_arguments_leave_outputs_untouched(setup, case):
    g, f, theta = setup
    rk, ok = BAD[case]
    rk = dict(rk)
    use_theta = rk.pop("theta", False)
    reg = pat.Reg(rk.pop("kind"), rk.pop("lam"), rk.pop("alpha0", 0.0), rk.pop("eta", 1.0),
                  theta if use_theta else None)
    out = torch.full((24, 24), SENTINEL, dtype=torch.float64, device="cuda")
    st, info = _raw_solve(g, f, reg, _opts(**ok), out)
    print(f"{case}: status {st} ({L.status_name(st)}): {L.load().pat_last_error().decode()}", flush=True)
    assert st == L.PAT_ERR_INVALID_ARG
    assert L.load().pat_last_error().decode() != ""
    assert torch.all(out == SENTINEL)
    assert info.iters == -1  # info untouched as well


def test_batched_rejects_mixed_element_types(setup):
    g, f, _ = setup
    g32 = pat.Geometry(dtype=torch.float32, **desc_for(24, 8, 48))
    f32 = f.float()
    with pytest.raises(L.PatError) as e:
        pat.solve_batched([(g, f, pat.Reg("tv", 0.02)), (g32, f32, pat.Reg("tv", 0.02))], max_iter=10)
    assert e.value.status == L.PAT_ERR_INVALID_ARG


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("bad", [math.nan, math.inf])
def test_non_finite_data_is_a_numeric_error(setup, dt, bad):
    g0, f0, _ = setup
    g = g0 if dt == torch.float64 else pat.Geometry(dtype=dt, **desc_for(24, 8, 48))
    f = f0.to(dt).clone()
    f.view(-1)[17] = bad
    out = torch.full((24, 24), SENTINEL, dtype=dt, device="cuda")
    state = torch.full((g.state_elems("tv"),), SENTINEL, dtype=dt, device="cuda")
    st_, info = _raw_solve(g, f, pat.Reg("tv", 0.02),
                           _opts(d_state_out=state.data_ptr(), max_iter=100), out)
    print(f"f[17] = {bad} ({dt}): status {st_}, {L.load().pat_last_error().decode()}", flush=True)
    assert st_ == L.PAT_ERR_NUMERIC
    assert torch.all(out == SENTINEL) and torch.all(state == SENTINEL)


def test_cap_returns_not_converged_with_valid_outputs(setup):
    g, f, _ = setup
    out = torch.full((24, 24), SENTINEL, dtype=torch.float64, device="cuda")
    st, info = _raw_solve(g, f, pat.Reg("tv", 0.02), _opts(max_iter=30, gap_tol=1e-13, gap_every=10,
                                                            graph_block=10), out)
    assert st == L.PAT_NOT_CONVERGED
    assert info.iters == 30 and info.converged == 0
    assert math.isfinite(info.rel_gap) and info.rel_gap > 1e-13
    assert math.isfinite(info.primal) and info.primal > 0
    assert bool(torch.all(torch.isfinite(out))) and not torch.any(out == SENTINEL)
    # the same call through the binding returns the warning, not an exception
    u, info2, st2 = pat.solve(g, f, pat.Reg("tv", 0.02), max_iter=30, gap_tol=1e-13, gap_every=10,
                              graph_block=10)
    assert st2 == L.PAT_NOT_CONVERGED and info2["iters"] == 30
    assert torch.equal(u, out)
