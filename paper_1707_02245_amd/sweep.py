"""The batched sweep workload: 64 reconstructions of uneven sizes run to the
gap target in one batched solve, against the same 64 solved one by one.

16 phantom groups, each on its own geometry: image N x N with N drawn from
{128, 192, 256, 384, 512}, 64..256 detectors on a closed circle or a half
circle, 2N time samples, phantom family disc, vessel or segment; 4
wavelengths per group (the group's data times U(0.3, 1), independent 5%
noise) share the geometry. Every instance has its own regulariser (TV, TGV
with alpha0 = 2 lambda, or directional TV with eta = 0.1) and lambda
log-uniform in [1e-3, 1e-1], and runs to relative gap 1e-4 in FP64 (FP32
iterates cannot certify 1e-4: the rounding of the stored duals floors the
gap's ||K^T y||_1 term near 1e-3). Launch shapes come from the library's
autotuner per geometry; iterations run in captured graph blocks of 50.

python -m paper_1707_02245_amd.sweep --json out.json [--one-by-one]
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

SIZES = (128, 192, 256, 384, 512)


def build_instances(seed=300, n_groups=16, n_wl=4, noise=0.05, dtype=torch.float64, autotune=True, log=print,
                    groups=None):
    """Geometries, data and regularisers of the sweep (seeded); returns
    (problems, meta) with problems as (geometry, data, regulariser) tuples.
    groups: optional range of group indices to build (the random draws of
    the others are still made, so every group is the same in any subset)."""
    import phantoms
    rng = np.random.default_rng(seed)
    problems, meta, geoms = [], [], []
    for gi in range(n_groups):
        n = int(rng.choice(SIZES))
        n_det = int(rng.integers(64, 257))
        span = 2 * math.pi if rng.random() < 0.5 else math.pi
        family = ("disc", "vessel", "segment")[int(rng.integers(3))]
        if groups is not None and gi not in groups:
            for w in range(n_wl):  # the draws of this group's wavelengths
                rng.uniform(0.3, 1.0)
                rng.integers(3)
                rng.uniform(-3, -1)
            continue
        desc = phantoms.geometry_desc(n, n_det, 2 * n, arc_span=span)
        g = pat.Geometry(dtype=dtype, **desc)
        if autotune:
            g.autotune(None, reps=5)
        geoms.append(g)
        case = phantoms.make_case(family, n, seed * 100 + gi, n_det, 2 * n)
        fine = pat.Geometry(dtype=torch.float64, **dict(desc, nx=2 * n, ny=2 * n))
        fc = fine.forward(torch.tensor(case["u_fine"], dtype=torch.float64, device="cuda")).cpu().numpy()
        fine.close()
        theta = torch.tensor(case["theta"], dtype=dtype, device="cuda")
        for w in range(n_wl):
            fw = rng.uniform(0.3, 1.0) * fc
            nz = phantoms.unit_noise(np.random.default_rng([seed, gi, w]), n_det, 2 * n)
            fw = fw + noise * np.linalg.norm(fw) / math.sqrt(fw.size) * nz
            kind = ("tv", "tgv", "dtv")[int(rng.integers(3))]
            lam = float(10 ** rng.uniform(-3, -1))
            reg = pat.Reg(kind, lam, 2 * lam if kind == "tgv" else 0.0, 0.1 if kind == "dtv" else 1.0,
                          theta if kind == "dtv" else None)
            problems.append((g, torch.tensor(fw, dtype=dtype, device="cuda"), reg))
            meta.append(dict(group=gi, n=n, n_det=n_det, arc="full" if span > 4 else "half", family=family,
                             reg=kind, lam=lam, csr_rot=g.info["csr_rot"]))
        log(f"group {gi}: {n}^2, {n_det} detectors, {'full' if span > 4 else 'half'} arc, {family}")
    return problems, meta, geoms


def solve_in_chunks(problems, gap_tol, cap, chunk, log, tag):
    """Batched solve to the gap target in calls of at most `chunk`
    iterations, each resuming every unfinished instance from the state the
    previous call exported (the resumed iterates equal the uninterrupted ones
    bit for bit); one progress line per call. Returns the per-instance
    results and the summed wall time of the calls."""
    n = len(problems)
    states = [torch.empty(g.state_elems(r.kind), dtype=g.dtype, device="cuda") for g, _, r in problems]
    done = [None] * n
    iters = [0] * n
    started = [False] * n
    secs = 0.0
    while any(d is None for d in done):
        act = [k for k in range(n) if done[k] is None]
        step = min(chunk, cap - iters[act[0]])
        outs = [torch.empty_like(states[k]) for k in act]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, infos, _ = pat.solve_batched([problems[k] for k in act], max_iter=step, gap_tol=gap_tol, gap_every=50,
                                        graph_block=50, states_out=outs,
                                        states_in=[states[k] if started[k] else None for k in act])
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        for k, info, o in zip(act, infos, outs):
            states[k] = o
            started[k] = True
            iters[k] += info["iters"]
            if info["converged"] or iters[k] >= cap:
                done[k] = dict(iters=iters[k], rel_gap=info["rel_gap"], converged=info["converged"])
        left = sum(d is None for d in done)
        log(f"{tag}: {iters[act[0]]} iterations, {n - left}/{n} finished, {secs:.1f} s")
    return done, secs


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, default=300)
    ap.add_argument("--gap-tol", type=float, default=1e-4)
    ap.add_argument("--cap", type=int, default=200000)
    ap.add_argument("--groups", type=int, default=16)
    ap.add_argument("--chunk", type=int, default=10000,
                    help="iterations per batched call (the solve resumes from the exported state)")
    ap.add_argument("--one-by-one", action="store_true", help="also solve every instance alone")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched solve")
    ap.add_argument("--only", default=None, metavar="A:B",
                    help="one by one: only instances A..B-1 (the rest in other calls)")
    ap.add_argument("--group-range", default=None, metavar="A:B",
                    help="build and solve only groups A..B-1 (same instances as in the full sweep)")
    ap.add_argument("--single-rate", type=int, default=0, metavar="N",
                    help="time N iterations of every instance solved alone (seconds per iteration of the "
                         "one-by-one solves, to extrapolate their time to each instance's iteration count)")
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)

    def log(msg):
        print(f"[sweep] {msg}", flush=True)

    grp = range(*(int(x) for x in a.group_range.split(":"))) if a.group_range else None
    problems, meta, geoms = build_instances(seed=a.seed, n_groups=a.groups, log=log, groups=grp)
    res = dict(instances=len(problems), gap_tol=a.gap_tol, cap=a.cap, meta=meta)
    if not a.no_batched:
        log(f"batched solve of {len(problems)} instances")
        infos, res["batched_s"] = solve_in_chunks(problems, a.gap_tol, a.cap, a.chunk, log, "batched")
        res["batched"] = infos
        log(f"batched: {res['batched_s']:.1f} s, {sum(i['converged'] for i in infos)}/{len(infos)} converged, "
            f"iterations {min(i['iters'] for i in infos)}..{max(i['iters'] for i in infos)}")
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(res, fh, indent=1)
    if a.single_rate > 0:
        rates = []
        for k, (g, f, reg) in enumerate(problems):
            pat.solve(g, f, reg, max_iter=50, gap_tol=0.0, gap_every=50, graph_block=50)  # graphs, buffers
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pat.solve(g, f, reg, max_iter=a.single_rate, gap_tol=0.0, gap_every=50, graph_block=50)
            torch.cuda.synchronize()
            rates.append((time.perf_counter() - t0) / a.single_rate)
            log(f"instance {k} alone: {rates[-1] * 1e6:.1f} us per iteration")
        res["single_s_per_iteration"] = rates
        if "batched" in res:
            est = sum(r * b["iters"] for r, b in zip(rates, res["batched"]))
            res["one_by_one_estimated_s"] = est
            log(f"one by one, extrapolated from {a.single_rate} iterations each to the batched run's "
                f"iteration counts: {est:.1f} s against batched {res['batched_s']:.1f} s")
        if a.json:
            with open(a.json, "w") as fh:
                json.dump(res, fh, indent=1)
    if a.one_by_one:
        seq, t_seq = [], 0.0
        lo, hi = (int(x) for x in a.only.split(":")) if a.only else (0, len(problems))
        res["one_by_one_range"] = [lo, hi]
        for k in range(lo, hi):
            one, dt = solve_in_chunks([problems[k]], a.gap_tol, a.cap, a.chunk, log, f"instance {k}")
            t_seq += dt
            seq.append(dict(one[0], s=dt))
            log(f"one by one {k}: {meta[k]['n']}^2 {meta[k]['reg']} lambda {meta[k]['lam']:.2e}: "
                f"{one[0]['iters']} iterations, {dt:.2f} s")
            res["sequential"] = seq
            res["sequential_s"] = t_seq
            if a.json:
                with open(a.json, "w") as fh:
                    json.dump(res, fh, indent=1)
        if "batched_s" in res and (lo, hi) == (0, len(problems)):
            res["speedup"] = t_seq / res["batched_s"]
            log(f"batched {res['batched_s']:.1f} s against one by one {t_seq:.1f} s ({res['speedup']:.2f}x)")
        else:
            log(f"one by one {lo}..{hi - 1}: {t_seq:.1f} s")
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(res, fh, indent=1)
    return res


if __name__ == "__main__":
    main(sys.argv[1:])
