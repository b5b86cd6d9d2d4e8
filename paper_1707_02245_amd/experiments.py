"""The paper's synthetic experiments (Sec. 6.1 and 6.2) as batched sweeps.

Sec. 6.1 compares reconstruction methods under uniform compressive sampling of
the detectors (16, 64, 192 or 384 of the locations that a 64-element array
over 172 degrees, scanned at six rotations of 60 degrees, provides) on data
without noise; Sec. 6.2 adds Gaussian noise to data from 192 detectors. For
each method the regularisation weight is the one that gives the best PSNR
against the ground truth (Sec. 6), so every point of a curve is a sweep over
lambda: all weights of all methods on one detector set share the geometry
and run as one batched solve (pat_pdhg_solve_batched), and pat_psnr scores
them on the GPU. The methods are the paper's variational ones available here
(TV, TGV) and its LS-T baseline; the phantom families and sizes are the
synthetic stand-ins of phantoms/.

python -m paper_1707_02245_amd.experiments detectors --n 128
python -m paper_1707_02245_amd.experiments noise --n 128
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import pat

# weights swept per method (with the circular-mean operator the data are
# means, so the useful weights are small)
DEFAULT_LAMBDAS = {
    "tv": tuple(float(x) for x in np.logspace(-6, -2, 9)),
    "tgv": tuple(float(x) for x in np.logspace(-6, -2, 9)),
    "lst": tuple(float(x) for x in np.logspace(-5, -1, 9)),
}


def sweep_geometry(n: int, count: int, n_t: int | None = None) -> dict:
    """Image n x n on [-1, 1]^2, `count` detectors of the rotated 172-degree
    array on the circle of radius 1.2, 2n time samples over radii 0..2.4."""
    import phantoms
    n_t = 2 * n if n_t is None else n_t
    desc = phantoms.geometry_desc(n, count, n_t)
    ang = phantoms.uniform_subset(phantoms.rotated_array_angles(), count)
    desc["det_xy"] = phantoms.detectors_xy(ang)
    desc["n_det"] = count
    return desc


def library_data(desc: dict, case: dict, noise: float) -> np.ndarray:
    """Data of a phantom by the library's FP64 forward operator on the grid
    twice as fine (same detectors and times), plus relative Gaussian noise."""
    n = desc["nx"]
    fine = pat.Geometry(dtype=torch.float64, **dict(desc, nx=2 * n, ny=2 * n))
    fc = fine.forward(torch.tensor(case["u_fine"], dtype=torch.float64, device="cuda")).cpu().numpy().ravel()
    fine.close()
    nz = case["noise"].ravel()[:fc.size]
    return fc + noise * np.linalg.norm(fc) / math.sqrt(fc.size) * nz


def _reg(method: str, lam: float) -> pat.Reg:
    if method == "lst":
        return pat.Reg("tikhonov", lam)
    if method == "tgv":
        return pat.Reg("tgv", lam, 2.0 * lam)
    return pat.Reg(method, lam)


def sweep_point(desc: dict, f: np.ndarray, u_gt: np.ndarray, methods, lambdas=None, gap_tol=1e-3,
                max_iter=20000, iters=None, dtype=torch.float64, sequential=False):
    """One point of a curve: every (method, lambda) on one geometry and data
    set, solved in one batch (or one by one with sequential=True); returns
    per instance the PSNR (printed and standard), iterations and the best
    lambda per method (by the printed PSNR), plus the wall time."""
    lambdas = lambdas or DEFAULT_LAMBDAS
    g = pat.Geometry(dtype=dtype, **desc)
    fd = torch.tensor(np.asarray(f).reshape(desc["n_det"], desc["n_t"]), dtype=dtype, device="cuda")
    gt = torch.tensor(u_gt, dtype=dtype, device="cuda").contiguous()
    problems, labels = [], []
    for m in methods:
        for lam in lambdas[m]:
            problems.append((g, fd, _reg(m, lam)))
            labels.append((m, lam))
    kw = dict(max_iter=iters or max_iter, gap_tol=0.0 if iters else gap_tol, gap_every=50, graph_block=50)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if sequential:
        us, infos = [], []
        for gg, ff, rr in problems:
            u, info, _ = pat.solve(gg, ff, rr, **kw)
            us.append(u)
            infos.append(info)
    else:
        us, infos, _ = pat.solve_batched(problems, **kw)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    rows = []
    for (m, lam), u, info in zip(labels, us, infos):
        pp, ps = pat.psnr(u, gt)
        rows.append(dict(method=m, lam=lam, psnr_printed=pp, psnr_standard=ps, iters=info["iters"],
                         rel_gap=info["rel_gap"], converged=info["converged"]))
    best = {}
    for r in rows:
        if r["method"] not in best or r["psnr_printed"] > best[r["method"]]["psnr_printed"]:
            best[r["method"]] = r
    g.close()
    return dict(rows=rows, best=best, seconds=secs, instances=len(problems))


def detector_curve(n=128, counts=(16, 64, 192, 384), family="disc", seed=0, methods=("tv", "lst"),
                   noise=0.0, data_fn=None, **kw):
    """Sec. 6.1: best PSNR per method against the number of detectors
    (no noise by default, as in the paper)."""
    import phantoms
    case = phantoms.make_case(family, n, seed, 384, 2 * n)
    data_fn = data_fn or library_data
    out = []
    for c in counts:
        desc = sweep_geometry(n, c)
        f = data_fn(desc, case, noise)
        res = sweep_point(desc, f, case["u_gt"], methods, **kw)
        out.append(dict(detectors=c, **res))
    return out


def noise_curve(n=128, levels=(0.01, 0.02, 0.05, 0.1, 0.2), count=192, family="disc", seed=0,
                methods=("tv", "lst"), data_fn=None, **kw):
    """Sec. 6.2: best PSNR per method against the relative noise level, 192
    detectors."""
    import phantoms
    case = phantoms.make_case(family, n, seed, 384, 2 * n)
    data_fn = data_fn or library_data
    desc = sweep_geometry(n, count)
    out = []
    for p in levels:
        f = data_fn(desc, case, p)
        res = sweep_point(desc, f, case["u_gt"], methods, **kw)
        out.append(dict(noise=p, **res))
    return out


def _summary(points, key):
    lines = []
    for pt in points:
        best = pt["best"]
        cells = ", ".join(f"{m}: {b['psnr_printed']:.2f} dB (lambda {b['lam']:.1e}, {b['iters']} it)"
                          for m, b in best.items())
        lines.append(f"{key} {pt[key]}: {cells}; {pt['instances']} instances in {pt['seconds']:.2f} s")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["detectors", "noise"])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--family", default="disc")
    ap.add_argument("--methods", default="tv,lst")
    ap.add_argument("--gap-tol", type=float, default=1e-3)
    ap.add_argument("--sequential-too", action="store_true",
                    help="also solve every point one instance at a time and report both times")
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    methods = tuple(a.methods.split(","))
    fn = detector_curve if a.which == "detectors" else noise_curve
    key = "detectors" if a.which == "detectors" else "noise"
    pts = fn(n=a.n, family=a.family, methods=methods, gap_tol=a.gap_tol)
    print(_summary(pts, key), flush=True)
    res = dict(which=a.which, n=a.n, family=a.family, methods=methods, gap_tol=a.gap_tol,
               batched_s=sum(p["seconds"] for p in pts), points=pts)
    if a.sequential_too:
        seq = fn(n=a.n, family=a.family, methods=methods, gap_tol=a.gap_tol, sequential=True)
        res["sequential_s"] = sum(p["seconds"] for p in seq)
        print(f"batched {res['batched_s']:.2f} s, one by one {res['sequential_s']:.2f} s", flush=True)
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(res, fh, indent=1)
    return res


if __name__ == "__main__":
    main(sys.argv[1:])
