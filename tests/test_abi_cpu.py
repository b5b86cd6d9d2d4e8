"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/pat.h declares, and rejects invalid arguments before
any device work."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1707_02245_amd import _lib as L
    return L, L.load()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "pat.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pat_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L, lib = _lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L._SIGS), "binding and header disagree"


def test_status_strings():
    L, lib = _lib()
    assert lib.pat_status_string(0) == b"PAT_OK"
    assert lib.pat_status_string(-1) == b"PAT_ERR_INVALID_ARG"
    assert lib.pat_status_string(1) == b"PAT_NOT_CONVERGED"


BAD = [
    dict(nx=1), dict(ny=1), dict(n_det=0), dict(n_t=1), dict(dt=0.0), dict(dt=-1.0),
    dict(c=0.0), dict(samples_per_pixel=0.0), dict(t0=-0.1), dict(x_max=float("nan")),
    dict(y_max=0.5), dict(arc_span=0.0), dict(arc_span=7.0), dict(det_radius=float("inf")),
]


@pytest.mark.parametrize("bad", BAD, ids=[",".join(b) for b in BAD])
def test_geometry_validation(bad):
    L, lib = _lib()
    from paper_1707_02245_amd.pat import make_desc
    kw = dict(nx=16, n_det=4, n_t=10, dt=0.2)
    kw.update(bad)
    d, keep = make_desc(**kw)
    h = C.c_void_p()
    st = lib.pat_geometry_create(C.byref(d), 0, None, C.byref(h))
    assert st == L.PAT_ERR_INVALID_ARG
    assert b"invalid argument" in lib.pat_last_error()
    assert h.value is None


def test_null_handles_rejected():
    L, lib = _lib()
    info = L.SolveInfo()
    reg = L.Regulariser()
    opts = L.SolveOpts()
    assert lib.pat_forward(None, None, None, None) == L.PAT_ERR_INVALID_ARG
    assert lib.pat_adjoint(None, None, None, None) == L.PAT_ERR_INVALID_ARG
    assert lib.pat_pdhg_solve(None, None, C.byref(reg), C.byref(opts), None, C.byref(info),
                              None) == L.PAT_ERR_INVALID_ARG
    assert lib.pat_precond(None, C.byref(reg), 0, None, None) == L.PAT_ERR_INVALID_ARG
    n = C.c_int64()
    assert lib.pat_state_elems(None, 0, C.byref(n)) == L.PAT_ERR_INVALID_ARG
    assert lib.pat_pdhg_solve_batched(0, None, None, None, None, None, None,
                                      None) == L.PAT_ERR_INVALID_ARG
    assert lib.pat_geometry_destroy(None) == L.PAT_OK


def test_wavelet_transform_validation():
    """pat_wavelet_forward / _adjoint reject bad shapes, levels, dtypes and
    NULL pointers before any device work."""
    L, lib = _lib()
    x = C.c_void_p(256)  # never dereferenced: every case fails validation first
    bad = [(1, 12, 8, 3, x, x), (1, 8, 8, 0, x, x), (1, 512, 512, 9, x, x), (1, 0, 8, 1, x, x),
           (2, 8, 8, 1, x, x), (1, 8, 8, 1, None, x), (1, 8, 8, 1, x, None), (0, 8, 6, 2, x, x)]
    for args in bad:
        for fn in (lib.pat_wavelet_forward, lib.pat_wavelet_adjoint):
            assert fn(*args, x, None) == L.PAT_ERR_INVALID_ARG, args
            assert b"invalid argument" in lib.pat_last_error()
    assert lib.pat_wavelet_work_elems(8, 8) == 64 + 16
    assert lib.pat_wavelet_work_elems(6, 2) == 12 + 3
    assert lib.pat_wavelet_work_elems(0, 8) == 0


STRUCTS = {
    "pat_geometry_desc": "GeometryDesc", "pat_geometry_info": "GeometryInfo",
    "pat_autotune_result": "AutotuneResult", "pat_regulariser": "Regulariser",
    "pat_solve_opts": "SolveOpts", "pat_solve_info": "SolveInfo", "pat_train_opts": "TrainOpts",
}


C_NAME = {"lam": "lambda"}  # ctypes names that are Python keywords


def test_struct_layouts_match_the_binding(tmp_path):
    """sizeof and every field offset of the C structs (compiled from the
    header by the host C compiler) equal the ctypes mirrors."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    from paper_1707_02245_amd import _lib as L
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pat.h"', 'int main(void) {']
    for cname, pyname in STRUCTS.items():
        st = getattr(L, pyname)
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in st._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {C_NAME.get(fname, fname)}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            a, b, c = ln.split()
            got[(a, b)] = int(c)
    for cname, pyname in STRUCTS.items():
        st = getattr(L, pyname)
        assert got[(cname, "size")] == C.sizeof(st), cname
        for fname, _ in st._fields_:
            assert got[(cname, fname)] == getattr(st, fname).offset, (cname, fname)
