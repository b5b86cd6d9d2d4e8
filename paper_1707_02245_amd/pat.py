"""Python binding of libpat (same names as the C ABI; marshalling only).

Every step of the computation runs in the HIP kernels behind include/pat.h.
PyTorch tensors serve only as device memory and as the source of the current
HIP stream.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import torch

from . import _lib as L

_DT = {torch.float32: L.PAT_F32, torch.float64: L.PAT_F64}
_KIND = {"tv": L.PAT_REG_TV, "tgv": L.PAT_REG_TGV, "dtv": L.PAT_REG_DTV,
         "tikhonov": L.PAT_REG_TIKHONOV, "lst": L.PAT_REG_TIKHONOV, "wav": L.PAT_REG_WAVELET}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, dtype, numel, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{name}: expected contiguous {dtype} with {numel} elements, "
                         f"got {t.dtype} {tuple(t.shape)}")


def make_desc(nx, ny=None, x_min=-1.0, x_max=1.0, y_min=None, y_max=None, n_det=1,
              det_cx=0.0, det_cy=0.0, det_radius=1.2, arc_center=0.0, arc_span=2 * math.pi,
              det_xy=None, n_t=2, t0=0.0, dt=1.0, c=1.0, samples_per_pixel=1.0):
    """pat_geometry_desc from keyword arguments (det_xy: host float64 [n_det][2])."""
    ny = nx if ny is None else ny
    y_min = x_min if y_min is None else y_min
    y_max = x_max if y_max is None else y_max
    d = L.GeometryDesc()
    d.nx, d.ny = nx, ny
    d.x_min, d.x_max, d.y_min, d.y_max = x_min, x_max, y_min, y_max
    d.n_det = n_det
    d.det_cx, d.det_cy, d.det_radius = det_cx, det_cy, det_radius
    d.arc_center, d.arc_span = arc_center, arc_span
    keep = None
    if det_xy is not None:
        import numpy as np
        keep = np.ascontiguousarray(np.asarray(det_xy, dtype=np.float64).reshape(-1, 2))
        d.n_det = keep.shape[0]
        d.det_xy = keep.ctypes.data_as(C.POINTER(C.c_double))
    d.n_t, d.t0, d.dt, d.c = n_t, t0, dt, c
    d.samples_per_pixel = samples_per_pixel
    return d, keep


class Geometry:
    """pat_geometry handle: acquisition geometry plus device tables."""

    def __init__(self, dtype=torch.float32, **desc):
        lib = L.load()
        self.dtype = dtype
        d, keep = make_desc(**desc)
        self._desc = d
        h = C.c_void_p()
        L.check(lib.pat_geometry_create(C.byref(d), _DT[dtype], _stream(), C.byref(h)))
        del keep
        self._h = h
        info = L.GeometryInfo()
        L.check(lib.pat_geometry_get_info(h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in info._fields_}
        self.nx, self.ny = info.nx, info.ny
        self.n_det, self.n_t = info.n_det, info.n_t

    @property
    def handle(self):
        return self._h

    def refresh_info(self):
        info = L.GeometryInfo()
        L.check(L.load().pat_geometry_get_info(self._h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in info._fields_}
        return self.info

    def set_launch(self, lanes_log2, tile, det_group):
        L.check(L.load().pat_geometry_set_launch(self._h, lanes_log2, tile, det_group))
        return self.refresh_info()

    def set_adjoint(self, mode):
        """mode: "scatter" (matrix-free), "csr" (stored A^T) or "tiled" (stored
        A^T with LDS-staged input windows)."""
        m = {"scatter": 0, "csr": 1, "tiled": 2}[mode]
        L.check(L.load().pat_geometry_set_adjoint(self._h, m, _stream()))
        return self.refresh_info()

    def set_forward_path(self, path):
        """Forward path: 0/1 gather (radius-/detector-major blocks), 2 LDS tiles,
        3 the stored A by pixel tiles (quarter-turn symmetric geometries)."""
        L.check(L.load().pat_geometry_set_forward_path(self._h, path, _stream()))
        return self.refresh_info()

    def set_tiled_launch(self, waves, row_lanes):
        """Workgroup shape of the tiled adjoint: waves per workgroup (4, 8, 16)
        and lanes per matrix row (16, 64)."""
        L.check(L.load().pat_geometry_set_tiled_launch(self._h, waves, row_lanes))
        return self.refresh_info()

    def set_forward_symmetry(self, enable):
        """Let the forward use the quarter-turn symmetry of the geometry (the
        bins of the first quarter of the detectors on the image and its three
        turned copies) or evaluate every detector directly."""
        L.check(L.load().pat_geometry_set_forward_symmetry(self._h, 1 if enable else 0))
        return self.refresh_info()

    def set_symmetry(self, enable):
        """Let the stored A^T use the quarter-turn symmetry of the geometry
        (rows of a quarter of the detectors only) or store every detector."""
        L.check(L.load().pat_geometry_set_symmetry(self._h, 1 if enable else 0, _stream()))
        return self.refresh_info()

    def autotune(self, cache_path=None, reps=10):
        """pat_geometry_autotune: time the launch candidates (or read the cache)."""
        res = L.AutotuneResult()
        path = cache_path.encode() if cache_path else None
        L.check(L.load().pat_geometry_autotune(self._h, path, reps, _stream(), C.byref(res)))
        self.refresh_info()
        return {k: getattr(res, k) for k, _ in res._fields_}

    def close(self):
        if getattr(self, "_h", None):
            L.load().pat_geometry_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def image(self, fill=0.0):
        return torch.full((self.ny, self.nx), fill, dtype=self.dtype, device="cuda")

    def data(self, fill=0.0):
        return torch.full((self.n_det, self.n_t), fill, dtype=self.dtype, device="cuda")

    def forward(self, u, out=None):
        """f = A u (pat_forward)."""
        _need(u, self.dtype, self.nx * self.ny, "u")
        out = self.data() if out is None else out
        _need(out, self.dtype, self.n_det * self.n_t, "out")
        L.check(L.load().pat_forward(self._h, _ptr(u), _ptr(out), _stream()))
        return out

    def adjoint(self, f, out=None):
        """u = A^T f (pat_adjoint)."""
        _need(f, self.dtype, self.n_det * self.n_t, "f")
        out = self.image() if out is None else out
        _need(out, self.dtype, self.nx * self.ny, "out")
        L.check(L.load().pat_adjoint(self._h, _ptr(f), _ptr(out), _stream()))
        return out

    def forward_padded(self, upad, out=None):
        """f = A u from the zero-bordered image [ny+2][nx+2] (pat_forward_padded)."""
        _need(upad, self.dtype, (self.nx + 2) * (self.ny + 2), "upad")
        out = self.data() if out is None else out
        _need(out, self.dtype, self.n_det * self.n_t, "out")
        L.check(L.load().pat_forward_padded(self._h, _ptr(upad), _ptr(out), _stream()))
        return out

    def adjoint_partials(self, f, out=None):
        """The csr_rot partial images of A^T f (pat_adjoint_partials)."""
        _need(f, self.dtype, self.n_det * self.n_t, "f")
        rot = self.info["csr_rot"]
        if out is None:
            out = torch.zeros((rot, self.ny, self.nx), dtype=self.dtype, device="cuda")
        _need(out, self.dtype, rot * self.nx * self.ny, "out")
        L.check(L.load().pat_adjoint_partials(self._h, _ptr(f), _ptr(out), _stream()))
        return out

    def state_elems(self, kind):
        n = C.c_int64()
        L.check(L.load().pat_state_elems(self._h, _KIND[kind], C.byref(n)))
        return n.value


@dataclass
class Reg:
    """Regulariser: kind in tv | tgv | dtv | tikhonov | wav (levels: the
    wavelet transform's decomposition levels)."""
    kind: str
    lam: float
    alpha0: float = 0.0
    eta: float = 1.0
    theta: torch.Tensor | None = None
    levels: int = 3

    def c_struct(self):
        r = L.Regulariser()
        r.kind = _KIND[self.kind]
        r.lam, r.tgv_alpha0, r.dtv_eta = self.lam, self.alpha0, self.eta
        r.d_dtv_theta = self.theta.data_ptr() if self.theta is not None else None
        r.wav_levels = self.levels
        return r


class Precond:
    """pat_precond_h: step sizes of one (geometry, regulariser) pair."""

    def __init__(self, geom: Geometry, reg: Reg, kind="diag"):
        self.geom = geom
        self.reg = reg
        r = reg.c_struct()
        h = C.c_void_p()
        k = L.PAT_PRECOND_DIAG if kind == "diag" else L.PAT_PRECOND_BLOCK
        L.check(L.load().pat_precond(geom.handle, C.byref(r), k, _stream(), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def get(self, which):
        """which: sigma_q | sigma_r | sigma_s | tau_u | tau_v."""
        idx = ["sigma_q", "sigma_r", "sigma_s", "tau_u", "tau_v"].index(which)
        g = self.geom
        n = {0: g.n_det * g.n_t, 4: 2 * g.nx * g.ny}.get(idx, g.nx * g.ny)
        if idx == 1 and self.reg.kind == "wav":
            n = 4 * g.nx * g.ny
        out = torch.empty(n, dtype=g.dtype, device="cuda")
        L.check(L.load().pat_precond_get(self._h, idx, _ptr(out), _stream()))
        return out

    def close(self):
        if getattr(self, "_h", None):
            L.load().pat_precond_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _opts(max_iter, gap_tol, gap_every, graph_block, theta, gap_box, u0, state_in,
          state_out, precond, y0=None, accel_gamma=0.0, accel_step_max=1.0):
    o = L.SolveOpts()
    o.accel_gamma, o.accel_step_max = accel_gamma, accel_step_max
    o.max_iter, o.gap_tol, o.gap_every, o.graph_block = max_iter, gap_tol, gap_every, graph_block
    o.theta, o.gap_box = theta, gap_box
    o.d_u0 = u0.data_ptr() if u0 is not None else None
    o.d_y0 = y0.data_ptr() if y0 is not None else None
    o.d_state_in = state_in.data_ptr() if state_in is not None else None
    o.d_state_out = state_out.data_ptr() if state_out is not None else None
    o.precond = precond.handle.value if precond is not None else None
    return o


def solve(geom: Geometry, f, reg: Reg, max_iter=2000, gap_tol=1e-4, gap_every=50,
          graph_block=50, theta=1.0, gap_box=2.0, u0=None, state_in=None, state_out=None,
          precond: Precond | None = None, out=None, y0=None, accel_gamma=0.0, accel_step_max=1.0):
    """pat_pdhg_solve. Returns (u, info dict, status). accel_gamma > 0 runs
    the accelerated schedule (pat_solve_opts.accel_gamma, accel_step_max)."""
    _need(f, geom.dtype, geom.n_det * geom.n_t, "f")
    out = geom.image() if out is None else out
    n_state = None
    for name, t in (("u0", u0),):
        if t is not None:
            _need(t, geom.dtype, geom.nx * geom.ny, name)
    if y0 is not None:
        _need(y0, geom.dtype, geom.n_det * geom.n_t + 2 * geom.nx * geom.ny, "y0")
    if state_in is not None or state_out is not None:
        n_state = geom.state_elems(reg.kind)
    if state_in is not None:
        _need(state_in, geom.dtype, n_state, "state_in")
    if state_out is not None:
        _need(state_out, geom.dtype, n_state, "state_out")
    if reg.theta is not None:
        _need(reg.theta, geom.dtype, geom.nx * geom.ny, "theta")
    r = reg.c_struct()
    o = _opts(max_iter, gap_tol, gap_every, graph_block, theta, gap_box, u0, state_in,
              state_out, precond, y0, accel_gamma, accel_step_max)
    info = L.SolveInfo()
    st = L.check(L.load().pat_pdhg_solve(geom.handle, _ptr(f), C.byref(r), C.byref(o),
                                         _ptr(out), C.byref(info), _stream()))
    return out, info.as_dict(), st


def solve_batched(problems, max_iter=2000, gap_tol=1e-4, gap_every=50, graph_block=50,
                  theta=1.0, gap_box=2.0, states_out=None, accel=None, states_in=None):
    """pat_pdhg_solve_batched over a list of (geom, f, reg[, precond]) tuples;
    states_out / states_in: optional lists of state buffers (or None
    entries) to export / resume from; accel: optional list of
    (accel_gamma, accel_step_max) per instance.
    Returns (list of u, list of info dicts, status)."""
    n = len(problems)
    geoms = (C.c_void_p * n)()
    fs = (C.c_void_p * n)()
    outs = (C.c_void_p * n)()
    regs = (L.Regulariser * n)()
    opts = (L.SolveOpts * n)()
    infos = (L.SolveInfo * n)()
    us = []
    for i, p in enumerate(problems):
        g, f, reg = p[0], p[1], p[2]
        pc = p[3] if len(p) > 3 else None
        _need(f, g.dtype, g.n_det * g.n_t, f"f[{i}]")
        u = g.image()
        us.append(u)
        geoms[i] = g.handle.value
        fs[i] = f.data_ptr()
        outs[i] = u.data_ptr()
        regs[i] = reg.c_struct()
        so = states_out[i] if states_out is not None else None
        if so is not None:
            _need(so, g.dtype, g.state_elems(reg.kind), f"states_out[{i}]")
        si = states_in[i] if states_in is not None else None
        if si is not None:
            _need(si, g.dtype, g.state_elems(reg.kind), f"states_in[{i}]")
        ag, am = accel[i] if accel is not None else (0.0, 1.0)
        opts[i] = _opts(max_iter, gap_tol, gap_every, graph_block, theta, gap_box, None, si,
                        so, pc, None, ag, am)
    st = L.check(L.load().pat_pdhg_solve_batched(n, geoms, fs, regs, opts, outs, infos, _stream()))
    return us, [infos[i].as_dict() for i in range(n)], st


def kernel_times(problems, reps=20, gap_every=50, graph_block=50):
    """pat_pdhg_kernel_times over a list of (geom, f, reg[, precond]) tuples:
    average ms per launch of the solver's forward launch (with both dual
    steps), the regulariser dual step alone, A^T and the primal step."""
    n = len(problems)
    geoms = (C.c_void_p * n)()
    fs = (C.c_void_p * n)()
    regs = (L.Regulariser * n)()
    opts = (L.SolveOpts * n)()
    for i, p in enumerate(problems):
        g, f, reg = p[0], p[1], p[2]
        pc = p[3] if len(p) > 3 else None
        _need(f, g.dtype, g.n_det * g.n_t, f"f[{i}]")
        geoms[i] = g.handle.value
        fs[i] = f.data_ptr()
        regs[i] = reg.c_struct()
        opts[i] = _opts(1, 0.0, gap_every, graph_block, 1.0, 2.0, None, None, None, pc)
    ms = (C.c_double * 4)()
    L.check(L.load().pat_pdhg_kernel_times(n, geoms, fs, regs, opts, reps, ms, _stream()))
    return dict(forward_dual_ms=ms[0], reg_dual_ms=ms[1], adjoint_ms=ms[2], primal_ms=ms[3])


def wavelet_work(nx, ny, dtype):
    """A work buffer for the wavelet transform calls (pat_wavelet_work_elems)."""
    return torch.empty(L.load().pat_wavelet_work_elems(nx, ny), dtype=dtype, device="cuda")


def wavelet_forward(u, levels, out=None, work=None):
    """c = W u (pat_wavelet_forward): u a CUDA float tensor [ny][nx]; c [4 nx ny].
    work: optional buffer from wavelet_work (else the call allocates and waits)."""
    ny, nx = u.shape
    _need(u, u.dtype, nx * ny, "u")
    c = torch.empty(4 * nx * ny, dtype=u.dtype, device=u.device) if out is None else out
    _need(c, u.dtype, 4 * nx * ny, "out")
    if work is not None:
        _need(work, u.dtype, L.load().pat_wavelet_work_elems(nx, ny), "work")
    L.check(L.load().pat_wavelet_forward(_DT[u.dtype], nx, ny, levels, _ptr(u), _ptr(c), _ptr(work),
                                         _stream()))
    return c


def wavelet_adjoint(c, nx, ny, levels, out=None, work=None):
    """u = W^T c (pat_wavelet_adjoint): c a CUDA float tensor [4 nx ny]; u [ny][nx]."""
    _need(c, c.dtype, 4 * nx * ny, "c")
    u = torch.empty((ny, nx), dtype=c.dtype, device=c.device) if out is None else out
    _need(u, c.dtype, nx * ny, "out")
    if work is not None:
        _need(work, c.dtype, L.load().pat_wavelet_work_elems(nx, ny), "work")
    L.check(L.load().pat_wavelet_adjoint(_DT[c.dtype], nx, ny, levels, _ptr(c), _ptr(u), _ptr(work),
                                         _stream()))
    return u


def psnr(u, u_gt):
    """pat_psnr: (printed, standard) PSNR of u against u_gt (Sec. 5.4)."""
    if u.dtype != u_gt.dtype or u.numel() != u_gt.numel():
        raise ValueError("u and u_gt need one dtype and size")
    _need(u, u.dtype, u.numel(), "u")
    _need(u_gt, u.dtype, u.numel(), "u_gt")
    a, b = C.c_double(), C.c_double()
    L.check(L.load().pat_psnr(_DT[u.dtype], u.numel(), _ptr(u), _ptr(u_gt), C.byref(a), C.byref(b), _stream()))
    return a.value, b.value


class Calibration:
    """pat_calib: calibrated pressure model and preprocessing (Sec. 4.1, 4.2)."""

    def __init__(self, geom: Geometry, pcal, xp, yp, eps):
        _need(pcal, geom.dtype, geom.n_det * geom.n_t, "pcal")
        self.geom = geom
        h = C.c_void_p()
        L.check(L.load().pat_calib_create(geom.handle, _ptr(pcal), float(xp), float(yp), float(eps), _stream(),
                                          C.byref(h)))
        self._h = h

    def pressure(self, u, out=None):
        """Measured pressure of image u (pat_pressure_forward)."""
        g = self.geom
        _need(u, g.dtype, g.nx * g.ny, "u")
        out = g.data() if out is None else out
        _need(out, g.dtype, g.n_det * g.n_t, "out")
        L.check(L.load().pat_pressure_forward(self._h, _ptr(u), _ptr(out), _stream()))
        return out

    def preprocess(self, p, out=None):
        """Data for the reconstruction from measured pressure (pat_preprocess)."""
        g = self.geom
        _need(p, g.dtype, g.n_det * g.n_t, "p")
        out = g.data() if out is None else out
        _need(out, g.dtype, g.n_det * g.n_t, "out")
        L.check(L.load().pat_preprocess(self._h, _ptr(p), _ptr(out), _stream()))
        return out

    def close(self):
        if getattr(self, "_h", None):
            L.load().pat_calib_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
