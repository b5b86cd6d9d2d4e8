"""Fixed sequences of stand-alone applies, for kernel traces and counter runs.

python -m paper_1707_02245_amd.kernel_runs forward-paths [--dtype f64|f32] [--reps 20]
python -m paper_1707_02245_amd.kernel_runs wavelet [--dtype f64|f32] [--reps 20]

runs, on the 256x256 ring of 256 detectors x 512 samples (a random image on the
zero-bordered grid), `reps` forwards by each path in turn: the gather with 16 lanes
per bin, its quarter-turn form with 32 lanes, the LDS-tiled gather and the stored A by
pixel tiles; then `reps` applies of A^T. Under rocprofv3 each kernel is one group of
`reps` dispatches (plus the padding pass of the quarter-turn form and the per-bin
passes of the tiled and stored paths).

`wavelet` runs `reps` dual-tree transforms W and then `reps` adjoints W^T (3
levels, a caller's work buffer) at 256 x 256 and at 4096 x 4096: per transform
one analysis launch per level (level 1 its own kernel instance), per adjoint one
synthesis launch per level. Then 200 solver iterations of the 256^2 wavelet model
(the ring of 256 detectors x 512 samples, lambda 0.003, 3 levels; gap every 50) put
the wavelet steps beside the forward, A^T and primal launches of an iteration.
"""
from __future__ import annotations

import argparse
import sys

import torch

from . import pat


def forward_paths(dtype=torch.float64, reps=20, log=print):
    import phantoms
    desc = phantoms.geometry_desc(256, 256, 512)
    g = pat.Geometry(dtype=dtype, **desc)
    upad = torch.zeros((258, 258), dtype=dtype, device="cuda")
    upad[1:-1, 1:-1] = torch.rand((256, 256), dtype=dtype, device="cuda")
    out = g.data()
    runs = (("gather, 16 lanes", 0, 4, False), ("quarter-turn gather, 32 lanes", 0, 5, True),
            ("LDS-tiled gather", 2, 4, False), ("stored A by pixel tiles", 3, 4, False))
    for label, path, lanes, sym in runs:
        g.set_forward_symmetry(sym)
        g.set_launch(lanes, g.info["adj_tile"], g.info["adj_det_group"])
        g.set_forward_path(path)
        for _ in range(reps):
            g.forward_padded(upad, out)
        torch.cuda.synchronize()
        log(f"{label}: {reps} applies (path {g.info['fwd_path']}, quarter-turn form {g.info['fwd_sym'] == 4})")
    y = g.data()
    y.copy_(out)
    u = g.image()
    for _ in range(reps):
        g.adjoint(y, u)
    torch.cuda.synchronize()
    log(f"A^T: {reps} applies (mode {g.info['adj_mode']}, {g.info['csr_rot']} quarter-turn slots)")
    g.close()


def wavelet(dtype=torch.float64, reps=20, log=print):
    for n in (256, 4096):
        u = torch.rand((n, n), dtype=dtype, device="cuda")
        c = torch.empty(4 * n * n, dtype=dtype, device="cuda")
        v = torch.empty((n, n), dtype=dtype, device="cuda")
        work = pat.wavelet_work(n, n, dtype)
        for _ in range(reps):
            pat.wavelet_forward(u, 3, out=c, work=work)
        torch.cuda.synchronize()
        log(f"W at {n}x{n}: {reps} transforms")
        for _ in range(reps):
            pat.wavelet_adjoint(c, n, n, 3, out=v, work=work)
        torch.cuda.synchronize()
        log(f"W^T at {n}x{n}: {reps} transforms")
        del u, c, v, work
        torch.cuda.empty_cache()
    import phantoms
    g = pat.Geometry(dtype=dtype, **phantoms.geometry_desc(256, 256, 512))
    f = torch.rand(256 * 512, dtype=dtype, device="cuda")
    pat.solve(g, f, pat.Reg("wav", 0.003, levels=3), max_iter=200, gap_tol=0.0, gap_every=50, graph_block=50)
    torch.cuda.synchronize()
    log("wavelet model at 256x256: 200 solver iterations")
    g.close()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["forward-paths", "wavelet"])
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--reps", type=int, default=20)
    a = ap.parse_args(argv)
    dt = torch.float64 if a.dtype == "f64" else torch.float32
    log = lambda m: print(f"[kernel_runs] {m}", flush=True)  # noqa: E731
    if a.what == "wavelet":
        wavelet(dt, a.reps, log=log)
    else:
        forward_paths(dt, a.reps, log=log)


if __name__ == "__main__":
    main(sys.argv[1:])
