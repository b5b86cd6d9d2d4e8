"""Geometry and the discrete circular-mean operator A, in float64.

Test infrastructure only (see the package docstring).

The paper models the data as integrals of the image over circles centred at
point detectors (Sec. 4.1, eq. K_def) and works with a matrix K computed once,
its transpose serving as adjoint (Sec. 3.3.1). The discretisation used here is
the circular *mean* over equispaced arc samples with bilinear interpolation:

    A[(d,k), j] = (1/M_k) * sum_m  hat((X_dkm - x_j)/h) * hat((Y_dkm - y_j)/h)

    (X, Y)_dkm = p_d + r_k (cos phi_km, sin phi_km),  phi_km = 2 pi (m + 1/2) / M_k
    r_k = c (t0 + k dt),  M_k = max(1, 4 ceil(2 pi r_k s / (4 h))),  hat(t) = max(0, 1 - |t|)

with pixel centres x_j on a cell-centred grid of pitch h and zero outside it.
Bins are ordered b = d * n_t + k, pixels j = iy * nx + ix (row = y).

The paper leaves the number of samples per circle open. M_k is the arc length
in samples rounded up to a multiple of four, so every circle's sample set is
unchanged by a quarter turn about its centre; a square grid centred in a ring
of 4m evenly spaced detectors then gives an operator that commutes with the
quarter turn (rotating the image shifts the data by m detectors).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass(frozen=True)
class Geometry:
    nx: int
    ny: int
    x_min: float
    x_max: float
    y_min: float
    y_max: float
    det_xy: np.ndarray      # (n_det, 2)
    radii: np.ndarray       # (n_t,) r_k = c (t0 + k dt)
    samples_per_pixel: float

    @property
    def h(self) -> float:
        return (self.x_max - self.x_min) / self.nx

    @property
    def n_det(self) -> int:
        return self.det_xy.shape[0]

    @property
    def n_t(self) -> int:
        return self.radii.shape[0]

    @property
    def n_bins(self) -> int:
        return self.n_det * self.n_t

    @property
    def n_pix(self) -> int:
        return self.nx * self.ny

    def n_samples(self) -> np.ndarray:
        """M_k = max(1, 4 ceil(2 pi r_k s / (4 h))) for every radius."""
        m = 4.0 * np.ceil(2.0 * math.pi * self.radii * self.samples_per_pixel / (4.0 * self.h))
        return np.maximum(1, m).astype(np.int64)

    def pixel_x(self) -> np.ndarray:
        return self.x_min + (np.arange(self.nx) + 0.5) * self.h

    def pixel_y(self) -> np.ndarray:
        return self.y_min + (np.arange(self.ny) + 0.5) * self.h


def detector_positions(n_det, cx, cy, radius, arc_center, arc_span) -> np.ndarray:
    """Point detectors on a circle arc.

    A closed circle (span 2 pi) spaces n_det detectors 2 pi / n_det apart from
    the centre angle; a shorter arc spaces them evenly with both ends included.
    """
    if abs(arc_span - 2.0 * math.pi) < 1e-12:
        ang = arc_center + 2.0 * math.pi * np.arange(n_det) / n_det
    elif n_det == 1:
        ang = np.array([arc_center])
    else:
        ang = arc_center - 0.5 * arc_span + arc_span * np.arange(n_det) / (n_det - 1)
    return np.stack([cx + radius * np.cos(ang), cy + radius * np.sin(ang)], axis=1)


def make_geometry(desc: dict) -> Geometry:
    """Geometry from a plain description (the fields of pat_geometry_desc)."""
    h = (desc["x_max"] - desc["x_min"]) / desc["nx"]
    hy = (desc["y_max"] - desc["y_min"]) / desc["ny"]
    if abs(h - hy) > 1e-12 * max(abs(h), 1.0):
        raise ValueError("pixels must be square")
    if desc.get("det_xy") is not None:
        det = np.asarray(desc["det_xy"], dtype=np.float64).reshape(-1, 2)
    else:
        det = detector_positions(desc["n_det"], desc["det_cx"], desc["det_cy"],
                                 desc["det_radius"], desc["arc_center"], desc["arc_span"])
    k = np.arange(desc["n_t"])
    radii = desc["c"] * (desc["t0"] + k * desc["dt"])
    return Geometry(desc["nx"], desc["ny"], desc["x_min"], desc["x_max"],
                    desc["y_min"], desc["y_max"], det, radii,
                    desc["samples_per_pixel"])


def hat(t: np.ndarray) -> np.ndarray:
    """Linear B-spline (tent) max(0, 1 - |t|)."""
    return np.maximum(0.0, 1.0 - np.abs(t))


def _samples(geom: Geometry, ks: np.ndarray):
    """All arc samples of the radii ks: (k index, r_k, cos phi, sin phi, M_k)."""
    M = geom.n_samples()[ks]
    kk = np.repeat(ks, M)
    start = np.repeat(np.cumsum(M) - M, M)
    m = np.arange(M.sum()) - start
    Mk = M.repeat(M).astype(np.float64)
    phi = 2.0 * math.pi * (m + 0.5) / Mk
    return kk, geom.radii[kk], np.cos(phi), np.sin(phi), Mk


def _detector_block(geom: Geometry, d: int, ks: np.ndarray):
    """COO triplets (k, pixel, value) of the rows (d, ks) of A."""
    kk, r, cphi, sphi, Mk = _samples(geom, ks)
    px, py = geom.det_xy[d]
    X = px + r * cphi
    Y = py + r * sphi
    h = geom.h
    # continuous pixel index: pixel i has its centre at gx == i
    gx = (X - geom.x_min) / h - 0.5
    gy = (Y - geom.y_min) / h - 0.5
    ix0 = np.floor(gx).astype(np.int64)
    iy0 = np.floor(gy).astype(np.int64)
    rows, cols, vals = [], [], []
    for dx in (0, 1):
        ix = ix0 + dx
        wx = hat(gx - ix)
        for dy in (0, 1):
            iy = iy0 + dy
            wy = hat(gy - iy)
            ok = (ix >= 0) & (ix < geom.nx) & (iy >= 0) & (iy < geom.ny) & (wx * wy > 0)
            rows.append(kk[ok])
            cols.append(iy[ok] * geom.nx + ix[ok])
            vals.append(wx[ok] * wy[ok] / Mk[ok])
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def forward_matrix(geom: Geometry) -> sp.csr_matrix:
    """A as an explicit CSR matrix of shape (n_det * n_t, ny * nx).

    Built detector by detector; duplicate (bin, pixel) pairs from neighbouring
    arc samples are summed.
    """
    ks = np.arange(geom.n_t)
    blocks = []
    for d in range(geom.n_det):
        k, c, v = _detector_block(geom, d, ks)
        blocks.append(sp.csr_matrix((v, (k, c)), shape=(geom.n_t, geom.n_pix)))
    A = sp.vstack(blocks, format="csr")
    A.sum_duplicates()
    return A


def forward_rows(geom: Geometry, bins: np.ndarray) -> sp.csr_matrix:
    """Selected rows of A (bins b = d * n_t + k), in the given order."""
    bins = np.asarray(bins, dtype=np.int64)
    out = []
    for b in bins:
        d, k = divmod(int(b), geom.n_t)
        kk, c, v = _detector_block(geom, d, np.array([k]))
        out.append(sp.csr_matrix((v, (np.zeros_like(kk), c)), shape=(1, geom.n_pix)))
    return sp.vstack(out, format="csr")
