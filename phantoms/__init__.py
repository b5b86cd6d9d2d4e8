"""Seeded synthetic inputs for the PAT reconstruction workloads.

This module only draws random numbers and rasterises test objects. It holds
none of the reconstruction arithmetic (no forward operator, no regulariser, no
solver step), so both the CPU oracle and the HIP library can take their inputs
from it without sharing any computation.

The paper's digital phantoms (Sec. 5.1: piecewise-constant shapes, a disc with
heterogeneous fluence, a vascular structure taken from a retinal image
database) are figures that are not available as data here; the families below
are synthetic stand-ins with the same character:

* ``disc``    -- random discs times an exponentially decaying fluence
                 (piecewise constant objects under heterogeneous fluence);
* ``vessel``  -- a branching tree of smooth Gaussian-profile tubes over a
                 linearly graded background (vascular structure);
* ``segment`` -- oriented line segments that follow a smooth random angle
                 field, times the fluence (anisotropic structure for the
                 directional regulariser).

All object support lies inside the unit disc, inside the detector circle of
radius 1.2 used by every workload. Phantoms are rasterised on a grid twice as
fine as the reconstruction grid, and the ground truth at reconstruction
resolution is its 2x2 block mean, so that synthetic data are not generated
with the discretisation used to invert them (Sec. 5.2, inverse crime).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage

__all__ = [
    "WORKLOADS",
    "Workload",
    "geometry_desc",
    "pixel_centres",
    "disc_phantom",
    "vessel_phantom",
    "segment_phantom",
    "angle_field",
    "make_case",
    "block_mean",
    "unit_noise",
    "rotated_array_angles",
    "uniform_subset",
    "detectors_xy",
]


# ---------------------------------------------------------------------------
# Workload descriptions (sizes only).
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    """One reconstruction workload: grid, detector arc, time samples, model."""

    name: str
    n: int                 # image is n x n on [-1, 1]^2
    n_det: int             # point detectors on an arc of radius 1.2
    arc_span: float        # 2*pi for a closed circle
    n_t: int               # time samples; radii 0 .. 2.4 inclusive
    family: str            # phantom family
    noise: float           # relative L2 noise level
    reg: str               # "tv" | "tgv" | "dtv" | "wav"
    lam: float             # TV / dTV / wavelet weight, TGV first-order weight alpha1
    alpha0: float = 0.0    # TGV second-order weight
    eta: float = 1.0       # dTV anisotropy
    levels: int = 3        # wavelet decomposition levels
    iters: int = 0         # fixed iteration count (0: run to gap_tol)
    gap_tol: float = 1e-4
    max_iter: int = 2000
    dtype: str = "f32"
    seeds: tuple = field(default_factory=tuple)


WORKLOADS = {
    # 64^2 TV-L2, 32 detectors on a closed circle, 128 samples, FP64.
    "tv64": Workload("tv64", 64, 32, 2 * math.pi, 128, "disc", 0.05, "tv", 0.05,
                     iters=200, dtype="f64", seeds=tuple(range(10))),
    # 256^2 TGV2-L2, 256 detectors closed, 512 samples, FP32, gap 1e-4.
    "tgv256": Workload("tgv256", 256, 256, 2 * math.pi, 512, "vessel", 0.10, "tgv",
                       0.02, alpha0=0.04, gap_tol=1e-4, max_iter=2000,
                       seeds=tuple(range(100, 110))),
    # 512^2 limited-angle dTV, 128 detectors over 90 degrees, 1024 samples.
    "dtv512": Workload("dtv512", 512, 128, 0.5 * math.pi, 1024, "segment", 0.05,
                       "dtv", 0.02, eta=0.1, gap_tol=1e-4, max_iter=2000,
                       seeds=tuple(range(200, 210))),
    # 256^2 dual-tree wavelet l1 (3 levels), geometry of tgv256, vascular
    # phantom (the paper's wavelet experiment reconstructs a vascular image).
    "wav256": Workload("wav256", 256, 256, 2 * math.pi, 512, "vessel", 0.05, "wav", 0.003,
                       gap_tol=1e-4, max_iter=2000, dtype="f64", seeds=tuple(range(300, 310))),
    # 256^2 TV, geometry of tgv256: the warm-start workload.
    "tv256": Workload("tv256", 256, 256, 2 * math.pi, 512, "mixed", 0.05, "tv", 0.02,
                      gap_tol=1e-4, max_iter=2000, seeds=tuple(range(50000, 50512))),
}


def geometry_desc(n: int, n_det: int, n_t: int, arc_span: float = 2 * math.pi,
                  det_radius: float = 1.2, r_max: float = 2.4,
                  samples_per_pixel: float = 1.0) -> dict:
    """Plain description of a workload geometry (numbers only)."""
    return dict(nx=n, ny=n, x_min=-1.0, x_max=1.0, y_min=-1.0, y_max=1.0,
                n_det=n_det, det_cx=0.0, det_cy=0.0, det_radius=det_radius,
                arc_center=0.0, arc_span=arc_span,
                n_t=n_t, t0=0.0, dt=r_max / (n_t - 1), c=1.0,
                samples_per_pixel=samples_per_pixel)


def rotated_array_angles(n_array: int = 64, span_deg: float = 172.0, n_rot: int = 6,
                         rot_deg: float = 60.0) -> np.ndarray:
    """Detector angles of an array of n_array elements spread evenly over
    span_deg (both ends included, centred on angle 0) scanned at n_rot
    rotations rot_deg apart (Sec. 6.1: 64 detectors over 172 degrees, six
    rotations of 60 degrees, 384 locations). Radians in [0, 2 pi), sorted."""
    base = np.deg2rad(-0.5 * span_deg + span_deg * np.arange(n_array) / (n_array - 1))
    ang = (base[None, :] + np.deg2rad(rot_deg) * np.arange(n_rot)[:, None]).ravel()
    return np.sort(np.mod(ang, 2 * math.pi))


def uniform_subset(angles: np.ndarray, count: int) -> np.ndarray:
    """A uniform compressive sampling of the scanned locations: for each of
    count equispaced target angles (starting at the first location) the
    nearest location not taken yet. The rotated arcs overlap (six 172-degree
    arcs cover 472 degrees), so every k-th of the sorted angles would not be
    even. Sorted radians."""
    if not 1 <= count <= len(angles):
        raise ValueError("count must be between 1 and the number of locations")
    free = np.ones(len(angles), dtype=bool)
    out = []
    for k in range(count):
        t = angles[0] + 2 * math.pi * k / count
        dist = np.abs(np.angle(np.exp(1j * (angles - t))))
        dist[~free] = np.inf
        i = int(np.argmin(dist))
        free[i] = False
        out.append(angles[i])
    return np.sort(np.mod(np.array(out), 2 * math.pi))


def detectors_xy(angles: np.ndarray, radius: float = 1.2) -> np.ndarray:
    """Point detectors at the given angles on a circle about the origin [n][2]."""
    return np.stack([radius * np.cos(angles), radius * np.sin(angles)], axis=1)


def pixel_centres(n: int, lo: float = -1.0, hi: float = 1.0):
    """Cell-centred coordinates of an n x n grid; returns (X, Y), row = y."""
    h = (hi - lo) / n
    c = lo + (np.arange(n) + 0.5) * h
    return np.meshgrid(c, c, indexing="xy")


def block_mean(u: np.ndarray) -> np.ndarray:
    """2x2 block mean (fine grid -> reconstruction grid)."""
    n2 = u.shape[0] // 2
    return u.reshape(n2, 2, n2, 2).mean(axis=(1, 3))


def unit_noise(rng: np.random.Generator, n_det: int, n_t: int) -> np.ndarray:
    """Standard normal draws in data layout [n_det][n_t].

    The caller scales them by p * ||f_clean||_2 / sqrt(n_det * n_t) for a
    relative noise level p.
    """
    return rng.standard_normal((n_det, n_t))


# ---------------------------------------------------------------------------
# Phantom families.
# ---------------------------------------------------------------------------

def _fluence(X, Y):
    r = np.sqrt(X * X + Y * Y)
    return np.where(r <= 1.0, np.exp(-2.0 * (1.0 - r)), 0.0)


def disc_phantom(rng: np.random.Generator, n_fine: int) -> np.ndarray:
    """3..8 discs (radius U(0.05,0.3), amplitude U(0.5,1)) inside |x|<=0.95,
    painted in order, times the fluence exp(-2*depth)."""
    X, Y = pixel_centres(n_fine)
    u = np.zeros_like(X)
    count = int(rng.integers(3, 9))
    for _ in range(count):
        rad = rng.uniform(0.05, 0.3)
        amp = rng.uniform(0.5, 1.0)
        rho = (0.95 - rad) * math.sqrt(rng.uniform())
        ang = rng.uniform(0.0, 2 * math.pi)
        cx, cy = rho * math.cos(ang), rho * math.sin(ang)
        inside = (X - cx) ** 2 + (Y - cy) ** 2 <= rad * rad
        u[inside] = amp
    return u * _fluence(X, Y)


def _bezier_points(p0, p1, p2, count=48):
    s = np.linspace(0.0, 1.0, count)[:, None]
    return (1 - s) ** 2 * p0 + 2 * (1 - s) * s * p1 + s * s * p2


def _tube(X, Y, pts, sigma):
    """max over the polyline pts of exp(-d^2 / 2 sigma^2), d = distance."""
    lo = pts.min(axis=0) - 5 * sigma
    hi = pts.max(axis=0) + 5 * sigma
    xs = (X[0] >= lo[0]) & (X[0] <= hi[0])
    ys = (Y[:, 0] >= lo[1]) & (Y[:, 0] <= hi[1])
    out = np.zeros_like(X)
    if not xs.any() or not ys.any():
        return out
    sub_x = X[np.ix_(ys, xs)]
    sub_y = Y[np.ix_(ys, xs)]
    d2 = np.full(sub_x.shape, np.inf)
    for a, b in zip(pts[:-1], pts[1:]):
        ab = b - a
        L2 = float(ab @ ab) or 1e-30
        t = np.clip(((sub_x - a[0]) * ab[0] + (sub_y - a[1]) * ab[1]) / L2, 0.0, 1.0)
        dx = sub_x - (a[0] + t * ab[0])
        dy = sub_y - (a[1] + t * ab[1])
        np.minimum(d2, dx * dx + dy * dy, out=d2)
    out[np.ix_(ys, xs)] = np.exp(-d2 / (2 * sigma * sigma))
    return out


def vessel_phantom(rng: np.random.Generator, n_fine: int, n_recon: int,
                   n_tubes: int = 20) -> np.ndarray:
    """Branching tree of quadratic-Bezier tubes over a graded background.

    Widths are 1..4 reconstruction pixels, the cross profile is Gaussian with
    sigma = width/2, amplitudes U(0.5,1); tubes are max-composited over a
    background rising linearly from 0.1 to 0.3 along x inside |x| <= 0.95.
    """
    X, Y = pixel_centres(n_fine)
    h = 2.0 / n_recon
    r = np.sqrt(X * X + Y * Y)
    u = np.where(r <= 0.95, 0.1 + 0.1 * (X + 1.0), 0.0)
    roots = []
    for _ in range(int(rng.integers(1, 3))):
        a = rng.uniform(0, 2 * math.pi)
        roots.append((np.array([0.85 * math.cos(a), 0.85 * math.sin(a)]), a + math.pi))
    branch_pts = []  # (point, heading) candidates to branch from
    for k in range(n_tubes):
        if k < len(roots) or not branch_pts:
            p0, head = roots[k % len(roots)]
        else:
            p0, head = branch_pts[int(rng.integers(len(branch_pts)))]
            head = head + rng.choice([-1.0, 1.0]) * rng.uniform(0.4, 1.1)
        length = rng.uniform(0.25, 0.6)
        bend = rng.uniform(-0.6, 0.6)
        p2 = p0 + length * np.array([math.cos(head + bend), math.sin(head + bend)])
        nrm = np.hypot(*p2)
        if nrm > 0.9:  # keep the tube inside the unit disc
            p2 = p2 * (0.9 / nrm)
        p1 = 0.5 * (p0 + p2) + 0.25 * length * rng.uniform(-1, 1) * np.array(
            [-math.sin(head), math.cos(head)])
        pts = _bezier_points(p0, p1, p2)
        width = rng.uniform(1.0, 4.0) * h
        amp = rng.uniform(0.5, 1.0)
        u = np.maximum(u, amp * _tube(X, Y, pts, 0.5 * width))
        for s_idx in (16, 32, 47):
            seg = pts[s_idx] - pts[s_idx - 1]
            branch_pts.append((pts[s_idx], math.atan2(seg[1], seg[0])))
    return np.where(r <= 0.95, u, 0.0)


def angle_field(rng: np.random.Generator, n: int, sigma_px: float = 16.0) -> np.ndarray:
    """Smooth random angle field theta = 0.5 * atan2(G*n2, G*n1).

    n1, n2 are per-pixel standard normal draws and G a Gaussian filter with
    the given width in pixels (reflecting boundary). Layout [n][n], row = y.
    """
    n1 = rng.standard_normal((n, n))
    n2 = rng.standard_normal((n, n))
    g1 = ndimage.gaussian_filter(n1, sigma_px, mode="reflect")
    g2 = ndimage.gaussian_filter(n2, sigma_px, mode="reflect")
    return 0.5 * np.arctan2(g2, g1)


def segment_phantom(rng: np.random.Generator, n_fine: int, n_recon: int,
                    theta: np.ndarray, n_seg: int = 40) -> np.ndarray:
    """Line segments oriented along theta at their centre, Gaussian profile of
    one reconstruction pixel, amplitude U(0.5,1), length U(0.1,0.5), times the
    fluence exp(-2*depth)."""
    X, Y = pixel_centres(n_fine)
    h = 2.0 / n_recon
    u = np.zeros_like(X)
    for _ in range(n_seg):
        rho = 0.8 * math.sqrt(rng.uniform())
        a = rng.uniform(0, 2 * math.pi)
        c = np.array([rho * math.cos(a), rho * math.sin(a)])
        i = min(n_recon - 1, max(0, int((c[0] + 1.0) / h)))
        j = min(n_recon - 1, max(0, int((c[1] + 1.0) / h)))
        th = float(theta[j, i])
        half = 0.5 * rng.uniform(0.1, 0.5)
        d = np.array([math.cos(th), math.sin(th)])
        pts = np.stack([c - half * d, c + half * d])
        amp = rng.uniform(0.5, 1.0)
        u = np.maximum(u, amp * _tube(X, Y, pts, h))
    return u * _fluence(X, Y)


def make_case(family: str, n: int, seed: int, n_det: int, n_t: int) -> dict:
    """Draw one synthetic case.

    Returns ``u_fine`` (2n x 2n phantom for data synthesis), ``u_gt`` (n x n
    ground truth, 2x2 block mean of u_fine), ``theta`` (n x n angle field,
    drawn for every family so the stream is the same) and ``noise`` (standard
    normal draws in data layout). ``family == "mixed"`` picks disc, vessel or
    segment round-robin by seed.
    """
    rng = np.random.default_rng(seed)
    if family == "mixed":
        family = ("disc", "vessel", "segment")[seed % 3]
    theta = angle_field(rng, n)
    if family == "disc":
        u_fine = disc_phantom(rng, 2 * n)
    elif family == "vessel":
        u_fine = vessel_phantom(rng, 2 * n, n)
    elif family == "segment":
        u_fine = segment_phantom(rng, 2 * n, n, theta)
    else:
        raise ValueError(f"unknown phantom family {family!r}")
    noise = unit_noise(np.random.default_rng([seed, 1]), n_det, n_t)
    return dict(family=family, u_fine=u_fine, u_gt=block_mean(u_fine),
                theta=theta, noise=noise)
