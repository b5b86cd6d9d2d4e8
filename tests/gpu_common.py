"""Shared helpers of the GPU parity tests (oracle on the CPU, library on the GPU)."""
import math

import numpy as np
import torch

import phantoms
from oracle import geometry as OG
from oracle import pdhg as OP

DT = {"f32": torch.float32, "f64": torch.float64}


def desc_for(n, n_det, n_t, **kw):
    d = phantoms.geometry_desc(n, n_det, n_t)
    d.update(kw)
    return d


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def to_dev(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def synth_data(desc, family, seed, noise=0.05):
    """Phantom data from the oracle on a 2x finer grid (no inverse crime)."""
    n = desc["nx"]
    case = phantoms.make_case(family, n, seed, desc["n_det"], desc["n_t"])
    fine = dict(desc, nx=2 * n, ny=2 * n)
    Af = OG.forward_matrix(OG.make_geometry(fine))
    fc = Af @ case["u_fine"].ravel()
    f = fc + noise * np.linalg.norm(fc) / math.sqrt(fc.size) * case["noise"].ravel()
    return f, case


def column_of_A(geom, j):
    """Column j of A from the oracle rows of the bins whose circles pass near
    pixel j (all others are zero)."""
    nx = geom.nx
    x = geom.pixel_x()[j % nx]
    y = geom.pixel_y()[j // nx]
    bins = []
    for d, (px, py) in enumerate(geom.det_xy):
        rho = math.hypot(x - px, y - py)
        ks = np.nonzero(np.abs(geom.radii - rho) <= 1.5 * math.sqrt(2) * geom.h)[0]
        bins.extend(d * geom.n_t + ks)
    bins = np.array(sorted(bins), dtype=np.int64)
    R = OG.forward_rows(geom, bins)
    col = np.zeros(geom.n_bins)
    col[bins] = R[:, j].toarray().ravel()
    return col


def split_state(st, kind, N, nb):
    st = np.asarray(st, dtype=np.float64)
    out = {"u": st[:N], "ubar": st[N:2 * N], "q": st[2 * N:2 * N + nb]}
    o = 2 * N + nb
    if kind == "wav":
        out["r"] = st[o:o + 4 * N].reshape(1, 4 * N)
        o += 4 * N
    elif kind != "tikhonov":
        out["r"] = st[o:o + 2 * N].reshape(2, N)
        o += 2 * N
    if kind == "tgv":
        out["v"] = st[o:o + 2 * N].reshape(2, N)
        out["vbar"] = st[o + 2 * N:o + 4 * N].reshape(2, N)
        s3 = st[o + 4 * N:o + 7 * N].reshape(3, N)
        out["s"] = np.stack([s3[0], s3[1], s3[1], s3[2]])
    return out


def oracle_problem(A, f, n, kind, lam, alpha0=0.0, eta=1.0, theta=None, ny=None, levels=3):
    ny = n if ny is None else ny
    return OP.Problem(A, f, n, ny, "lst" if kind == "tikhonov" else kind, lam,
                      alpha0=alpha0, eta=eta, theta=theta, levels=levels)
