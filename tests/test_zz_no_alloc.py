"""pat_adjoint_noalloc (through the C ABI) against pat_adjoint: the same
kernels, so the same bits, on two calls in a row (the second on a smaller
geometry) in every adjoint mode, plus the size limit of its fixed scratch."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_common import desc_for, to_dev

pytestmark = pytest.mark.gpu

pat = pytest.importorskip("paper_1707_02245_amd.pat")
L = pat.L


def _noalloc(g, f, out):
    st = L.load().pat_adjoint_noalloc(g.handle, C.c_void_p(f.data_ptr()), C.c_void_p(out.data_ptr()),
                                      C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("mode", ["tiled", "csr", "scatter"])
def test_noalloc_adjoint_equals_adjoint(mode, dt):
    big = desc_for(64, 32, 128)           # quarter-turn ring: 4 partial images
    small = desc_for(40, 12, 70)          # smaller geometry, also 4 slots
    rng = np.random.default_rng(11)
    for d in (big, small):
        g = pat.Geometry(dtype=dt, **d)
        g.set_adjoint(mode)
        if mode == "scatter":
            g.set_launch(6, 32, 4)        # several detector groups: partial images
        f = to_dev(rng.standard_normal((d["n_det"], d["n_t"])), dt)
        want = g.adjoint(f)
        got = torch.full_like(want, 123.0)
        print(f"noalloc {mode} {dt} {d['nx']}^2 {d['n_det']}x{d['n_t']} rot {g.info['csr_rot']}", flush=True)
        st = _noalloc(g, f, got)
        assert st == L.PAT_OK, L.load().pat_last_error().decode()
        torch.cuda.synchronize()
        assert torch.equal(got, want)


def test_noalloc_rejects_scratch_beyond_its_array():
    # matrix-free scatter with one detector per group: 64 partial images of
    # 256^2 doubles = 32 MiB > 16 MiB
    g = pat.Geometry(dtype=torch.float64, **desc_for(256, 64, 64))
    g.set_adjoint("scatter")
    g.set_launch(6, 32, 1)
    f = g.data(1.0)
    out = torch.full((256, 256), 5.0, dtype=torch.float64, device="cuda")
    st = _noalloc(g, f, out)
    torch.cuda.synchronize()
    assert st == L.PAT_ERR_INVALID_ARG
    assert "16777216" in L.load().pat_last_error().decode()
    assert torch.all(out == 5.0)
    # the allocating entry point still serves it, and a small call after the
    # rejected one works
    g.set_launch(6, 32, 16)
    want = g.adjoint(f)
    got = torch.empty_like(want)
    assert _noalloc(g, f, got) == L.PAT_OK
    torch.cuda.synchronize()
    assert torch.equal(got, want)
