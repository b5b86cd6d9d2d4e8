"""ctypes declarations of the C ABI in include/pat.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# PAT_LIB selects another build of the same library (e.g. the host-sanitized one)
LIB_PATH = os.environ.get("PAT_LIB") or os.path.join(_HERE, "libpat.so")

PAT_OK = 0
PAT_NOT_CONVERGED = 1
PAT_ERR_INVALID_ARG = -1
PAT_ERR_OOM = -2
PAT_ERR_DEVICE = -3
PAT_ERR_NUMERIC = -4
PAT_ERR_UNSUPPORTED = -5

PAT_F32, PAT_F64 = 0, 1
PAT_REG_TV, PAT_REG_TGV, PAT_REG_DTV, PAT_REG_TIKHONOV, PAT_REG_WAVELET = 0, 1, 2, 3, 4
PAT_PRECOND_DIAG, PAT_PRECOND_BLOCK = 0, 1


class GeometryDesc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("x_min", C.c_double), ("x_max", C.c_double),
        ("y_min", C.c_double), ("y_max", C.c_double),
        ("n_det", C.c_int32),
        ("det_cx", C.c_double), ("det_cy", C.c_double), ("det_radius", C.c_double),
        ("arc_center", C.c_double), ("arc_span", C.c_double),
        ("det_xy", C.POINTER(C.c_double)),
        ("n_t", C.c_int32),
        ("t0", C.c_double), ("dt", C.c_double), ("c", C.c_double),
        ("samples_per_pixel", C.c_double),
    ]


class GeometryInfo(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("n_det", C.c_int32), ("n_t", C.c_int32),
        ("n_pix", C.c_int64), ("n_bins", C.c_int64),
        ("n_samples", C.c_int64), ("n_window", C.c_int64),
        ("dtype", C.c_int32),
        ("fwd_lanes_log2", C.c_int32), ("adj_tile", C.c_int32), ("adj_det_group", C.c_int32),
        ("adj_mode", C.c_int32), ("csr_nnz", C.c_int64), ("csr_tile_side", C.c_int32),
        ("csr_win_max", C.c_int32), ("csr_rot", C.c_int32), ("sym_rot", C.c_int32),
        ("csr_waves", C.c_int32), ("csr_lanes", C.c_int32), ("fwd_path", C.c_int32),
        ("fwd_pairs", C.c_int64),
        ("fwd_sym", C.c_int32),
        ("fwd_entries", C.c_int64),
    ]


class AutotuneResult(C.Structure):
    _fields_ = [
        ("fwd_lanes_log2", C.c_int32), ("adj_mode", C.c_int32), ("adj_tile", C.c_int32),
        ("adj_det_group", C.c_int32), ("forward_ms", C.c_double), ("adjoint_ms", C.c_double),
        ("from_cache", C.c_int32),
    ]


class Regulariser(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("lam", C.c_double), ("tgv_alpha0", C.c_double),
        ("dtv_eta", C.c_double), ("d_dtv_theta", C.c_void_p), ("wav_levels", C.c_int32),
    ]


class SolveOpts(C.Structure):
    _fields_ = [
        ("max_iter", C.c_int32), ("gap_tol", C.c_double), ("gap_every", C.c_int32),
        ("graph_block", C.c_int32), ("theta", C.c_double), ("gap_box", C.c_double),
        ("d_u0", C.c_void_p), ("d_y0", C.c_void_p), ("d_state_in", C.c_void_p), ("d_state_out", C.c_void_p),
        ("precond", C.c_void_p), ("accel_gamma", C.c_double), ("accel_step_max", C.c_double),
    ]


class SolveInfo(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("converged", C.c_int32), ("fallback", C.c_int32),
        ("rel_gap", C.c_double), ("gap", C.c_double), ("primal", C.c_double),
        ("fstar", C.c_double), ("kty_l1", C.c_double), ("residual", C.c_double),
        ("seconds", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double), ("seed", C.c_uint64)]


_SIGS = {
    "pat_geometry_create": ([C.POINTER(GeometryDesc), C.c_int, C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "pat_geometry_destroy": ([C.c_void_p], C.c_int),
    "pat_geometry_get_info": ([C.c_void_p, C.POINTER(GeometryInfo)], C.c_int),
    "pat_geometry_set_launch": ([C.c_void_p, C.c_int32, C.c_int32, C.c_int32], C.c_int),
    "pat_geometry_set_adjoint": ([C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "pat_geometry_set_symmetry": ([C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "pat_geometry_set_forward_symmetry": ([C.c_void_p, C.c_int32], C.c_int),
    "pat_geometry_set_tiled_launch": ([C.c_void_p, C.c_int32, C.c_int32], C.c_int),
    "pat_geometry_set_forward_path": ([C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "pat_geometry_autotune": ([C.c_void_p, C.c_char_p, C.c_int32, C.c_void_p,
                               C.POINTER(AutotuneResult)], C.c_int),
    "pat_forward": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "pat_adjoint": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "pat_adjoint_noalloc": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "pat_forward_padded": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "pat_adjoint_partials": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "pat_precond": ([C.c_void_p, C.POINTER(Regulariser), C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "pat_precond_get": ([C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p], C.c_int),
    "pat_precond_destroy": ([C.c_void_p], C.c_int),
    "pat_state_elems": ([C.c_void_p, C.c_int32, C.POINTER(C.c_int64)], C.c_int),
    "pat_pdhg_solve": ([C.c_void_p, C.c_void_p, C.POINTER(Regulariser), C.POINTER(SolveOpts),
                        C.c_void_p, C.POINTER(SolveInfo), C.c_void_p], C.c_int),
    "pat_pdhg_solve_batched": ([C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                C.POINTER(Regulariser), C.POINTER(SolveOpts), C.POINTER(C.c_void_p),
                                C.POINTER(SolveInfo), C.c_void_p], C.c_int),
    "pat_pdhg_kernel_times": ([C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                               C.POINTER(Regulariser), C.POINTER(SolveOpts), C.c_int32,
                               C.POINTER(C.c_double), C.c_void_p], C.c_int),
    "pat_warmstart_create": ([C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.POINTER(C.c_void_p)], C.c_int),
    "pat_warmstart_destroy": ([C.c_void_p], C.c_int),
    "pat_warmstart_set_gemm_tiles": ([C.c_int32], C.c_int),
    "pat_warmstart_num_params": ([C.c_void_p, C.POINTER(C.c_int64)], C.c_int),
    "pat_warmstart_get_params": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "pat_warmstart_set_params": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "pat_warmstart_forward": ([C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                               C.c_void_p], C.c_int),
    "pat_warmstart_grad": ([C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                            C.c_void_p, C.POINTER(C.c_double), C.c_void_p], C.c_int),
    "pat_warmstart_train": ([C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                             C.POINTER(TrainOpts), C.POINTER(C.c_double), C.c_void_p], C.c_int),
    "pat_warmstart_save": ([C.c_void_p, C.c_char_p], C.c_int),
    "pat_warmstart_load": ([C.c_void_p, C.c_char_p], C.c_int),
    "pat_warmstart_normalize": ([C.c_void_p, C.POINTER(Regulariser), C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p], C.c_int),
    "pat_warmstart_infer": ([C.c_void_p, C.c_void_p, C.POINTER(Regulariser), C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_void_p], C.c_int),
    "pat_calib_create": ([C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_void_p,
                          C.POINTER(C.c_void_p)], C.c_int),
    "pat_calib_destroy": ([C.c_void_p], C.c_int),
    "pat_pressure_forward": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "pat_preprocess": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "pat_psnr": ([C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                  C.c_void_p], C.c_int),
    "pat_wavelet_work_elems": ([C.c_int32, C.c_int32], C.c_int64),
    "pat_wavelet_forward": ([C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_void_p], C.c_int),
    "pat_wavelet_adjoint": ([C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_void_p], C.c_int),
    "pat_status_string": ([C.c_int], C.c_char_p),
    "pat_last_error": ([], C.c_char_p),
}

_lib = None


def load() -> C.CDLL:
    """Load libpat.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1707_02245_amd.build` "
            "(there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class PatError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_name(status)}: {message}")
        self.status = status


def status_name(s: int) -> str:
    return load().pat_status_string(s).decode()


def check(status: int) -> int:
    """Raise PatError for error statuses (< 0); return warnings (>= 0)."""
    if status < 0:
        raise PatError(status, load().pat_last_error().decode())
    return status
