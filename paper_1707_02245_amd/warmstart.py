"""Learned warm start for PDHG: training pairs from the solver, training and
evaluation, all through the C ABI (marshalling only).

The network maps the normalised backprojection of the data to the normalised
TV reconstruction and its dual variable (three output planes); at test time
PDHG starts from its output: u0, q0 = A u0 - f and r0. The solver's gap decides
the result and a start that is non-finite or worse than zero falls back to
zero, so the fixed point never depends on the network.

python -m paper_1707_02245_amd.warmstart train --n-train 256 --out weights.npy
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import math
import sys
import time

import numpy as np
import torch

from . import _lib as L
from . import pat


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class WarmStartNet:
    """pat_unet handle."""

    def __init__(self, levels=4, base=32, out_ch=3, seed=0):
        lib = L.load()
        h = C.c_void_p()
        L.check(lib.pat_warmstart_create(levels, base, out_ch, seed, C.byref(h)))
        self._h = h
        n = C.c_int64()
        L.check(lib.pat_warmstart_num_params(h, C.byref(n)))
        self.n_params = n.value
        self.levels, self.base, self.out_ch = levels, base, out_ch

    def params(self) -> np.ndarray:
        t = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        L.check(L.load().pat_warmstart_get_params(self._h, C.c_void_p(t.data_ptr()), _stream()))
        return t.cpu().numpy()

    def set_params(self, v: np.ndarray):
        t = torch.tensor(np.asarray(v, dtype=np.float32), device="cuda")
        L.check(L.load().pat_warmstart_set_params(self._h, C.c_void_p(t.data_ptr()), _stream()))
        torch.cuda.synchronize()

    def save_weights(self, path):
        np.save(path, self.params())

    def load_weights(self, path, check_operator=True):
        """Parameters from a .npy file; with check_operator the manifest beside
        it (same name, .json) must carry this library's operator fingerprint."""
        v = np.load(path, allow_pickle=False)
        if v.shape != (self.n_params,):
            raise ValueError(f"{path}: {v.shape} parameters, network has {self.n_params}")
        if check_operator:
            import os
            man = os.path.splitext(path)[0] + ".json"
            with open(man) as fh:
                fp = json.load(fh).get("operator_fingerprint")
            if fp != operator_fingerprint():
                raise ValueError(f"{path} was trained on another forward operator (fingerprint {fp}, "
                                 f"this library {operator_fingerprint()})")
        self.set_params(v)

    def train(self, inputs, targets, epochs, batch, lr, seed=0):
        n, h, w = inputs.shape
        opts = L.TrainOpts(epochs=epochs, batch=batch, lr=lr, seed=seed)
        loss = C.c_double()
        L.check(L.load().pat_warmstart_train(self._h, n, h, w, C.c_void_p(inputs.data_ptr()),
                                             C.c_void_p(targets.data_ptr()), C.byref(opts),
                                             C.byref(loss), _stream()))
        return loss.value

    def infer(self, geom: pat.Geometry, f, reg: pat.Reg, dual=True):
        """(u0, y0): the primal start and, with dual, the dual start q0 then r0."""
        u0 = geom.image()
        y0 = (torch.empty(geom.n_det * geom.n_t + 2 * geom.nx * geom.ny, dtype=geom.dtype,
                          device="cuda") if dual else None)
        r = reg.c_struct()
        L.check(L.load().pat_warmstart_infer(self._h, geom.handle, C.byref(r), C.c_void_p(f.data_ptr()),
                                             C.c_void_p(u0.data_ptr()),
                                             C.c_void_p(y0.data_ptr()) if dual else None, _stream()))
        return u0, y0

    def close(self):
        if getattr(self, "_h", None):
            L.load().pat_warmstart_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_FINGERPRINT = []


def operator_fingerprint() -> str:
    """Fingerprint of the discrete forward operator this library computes: a
    hash of the FP64 A u of a fixed image on a small geometry (32^2, 8
    detectors x 64 samples), rounded to 9 decimals. It changes when the
    operator's definition changes (sample counts, phases, weights), not when
    its kernels are tuned."""
    if not _FINGERPRINT:
        import hashlib
        import phantoms
        g = pat.Geometry(dtype=torch.float64, **phantoms.geometry_desc(32, 8, 64))
        i = np.arange(32)
        u = ((7 * i[:, None] + 3 * i[None, :]) % 11) / 10.0
        f = g.forward(torch.tensor(u, dtype=torch.float64, device="cuda")).cpu().numpy()
        g.close()
        txt = ",".join(f"{x:.9f}" for x in f.ravel())
        _FINGERPRINT.append(hashlib.sha256(txt.encode()).hexdigest()[:16])
    return _FINGERPRINT[0]


def normalize(geom: pat.Geometry, f, reg: pat.Reg | None = None, state=None, channels=3):
    """(x, t, scale): normalised backprojection, target planes (from a solver
    state, else None), scale."""
    x = torch.empty(geom.ny, geom.nx, dtype=torch.float32, device="cuda")
    t = (torch.empty(channels, geom.ny, geom.nx, dtype=torch.float32, device="cuda")
         if state is not None else None)
    s = torch.empty(1, dtype=torch.float32, device="cuda")
    r = reg.c_struct() if reg is not None else None
    L.check(L.load().pat_warmstart_normalize(
        geom.handle, C.byref(r) if r is not None else None, C.c_void_p(f.data_ptr()),
        C.c_void_p(state.data_ptr()) if state is not None else None,
        C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()) if t is not None else None, channels,
        C.c_void_p(s.data_ptr()), _stream()))
    return x, t, s


_FINE = {}


def _fine_geometry(desc):
    key = tuple(sorted(desc.items()))
    if key not in _FINE:
        n = desc["nx"]
        _FINE.clear()
        _FINE[key] = pat.Geometry(dtype=torch.float64, **dict(desc, nx=2 * n, ny=2 * n))
    return _FINE[key]


def synth_data(desc, seed, noise=None, dtype=torch.float64):
    """Data of one seeded phantom: the library's forward operator on the 2x
    finer grid, plus relative Gaussian noise (level U(1%, 10%) by seed if not
    given). Returns (f device tensor, ground truth [n][n], noise level)."""
    import phantoms
    n = desc["nx"]
    case = phantoms.make_case("mixed", n, seed, desc["n_det"], desc["n_t"])
    if noise is None:
        noise = float(np.random.default_rng([seed, 7]).uniform(0.01, 0.10))
    fine = _fine_geometry(desc)
    fc = fine.forward(torch.tensor(case["u_fine"], dtype=torch.float64, device="cuda")).cpu().numpy()
    f = fc + noise * np.linalg.norm(fc) / math.sqrt(fc.size) * case["noise"]
    return torch.tensor(f, dtype=dtype, device="cuda"), case["u_gt"], noise


def make_pairs(geom, desc, seeds, lam, gap_tol, cap, group=8, channels=3, log=None):
    """Training pairs: PDHG (TV, lam) solutions to gap_tol in batches that
    share the geometry; unconverged solves are dropped and counted.
    Returns (inputs [n][h][w], targets [n][channels][h][w], stats)."""
    reg = pat.Reg("tv", lam)
    pc = pat.Precond(geom, reg, "diag")
    n_state = geom.state_elems("tv")
    xs, ts, iters, dropped = [], [], [], 0
    t0 = time.perf_counter()
    for g0 in range(0, len(seeds), group):
        fs = [synth_data(desc, s, dtype=geom.dtype)[0] for s in seeds[g0:g0 + group]]
        states = [torch.empty(n_state, dtype=geom.dtype, device="cuda") for _ in fs]
        us, infos, st = pat.solve_batched([(geom, f, reg, pc) for f in fs], max_iter=cap,
                                          gap_tol=gap_tol, gap_every=50, graph_block=50,
                                          states_out=states)
        for f, state, info in zip(fs, states, infos):
            if not info["converged"]:
                dropped += 1
                continue
            x, t, _ = normalize(geom, f, reg, state, channels)
            xs.append(x)
            ts.append(t)
            iters.append(info["iters"])
        if log:
            log(f"pairs {g0 + len(fs)}/{len(seeds)}: iters {[i['iters'] for i in infos]} "
                f"({time.perf_counter() - t0:.1f} s)")
    return (torch.stack(xs).contiguous(), torch.stack(ts).contiguous(),
            dict(seconds=time.perf_counter() - t0, iters=iters, dropped=dropped))


STARTS = ("zero", "backprojection", "network_primal", "network")


def evaluate(geom, desc, net, seeds, lam, gap_tol, cap, starts=STARTS, log=None):
    """Iterations and seconds to gap_tol from zero, from the backprojection
    A^T f / A^T 1, from the network's primal output alone and from its primal
    and dual output (inference included in the seconds)."""
    reg = pat.Reg("tv", lam)
    pc = pat.Precond(geom, reg, "diag")
    out = []
    for s in seeds:
        f, u_gt, noise = synth_data(desc, s, dtype=geom.dtype)
        rec = {"seed": s, "noise": noise}
        x, _, sc = normalize(geom, f)
        bp = (x.double() * sc.double()).to(geom.dtype).contiguous()
        for name in starts:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u0 = y0 = None
            if name == "backprojection":
                u0 = bp
            elif name == "network_primal":
                u0, _ = net.infer(geom, f, reg, dual=False)
            elif name == "network":
                u0, y0 = net.infer(geom, f, reg, dual=True)
            u, info, st = pat.solve(geom, f, reg, max_iter=cap, gap_tol=gap_tol, gap_every=50,
                                    graph_block=50, u0=u0, y0=y0, precond=pc)
            torch.cuda.synchronize()
            rec[name] = dict(iters=info["iters"], seconds=time.perf_counter() - t0,
                             rel_gap=info["rel_gap"], primal=info["primal"],
                             fallback=info["fallback"], status=st)
        out.append(rec)
        if log:
            log(json.dumps(rec))
    return out


def val_loss(net, x, t, batch=8):
    """Mean squared error of the network on held-out pairs."""
    n, h, w = x.shape
    y = torch.empty(batch, net.out_ch, h, w, dtype=torch.float32, device="cuda")
    tot, cnt = 0.0, 0
    for i in range(0, n - batch + 1, batch):
        L.check(L.load().pat_warmstart_forward(net._h, batch, h, w, C.c_void_p(x[i:i + batch].data_ptr()),
                                               C.c_void_p(y.data_ptr()), _stream()))
        tot += float(((y - t[i:i + batch]) ** 2).sum())
        cnt += y.numel()
    return tot / max(cnt, 1)


def unet_flops(base=32, levels=4, h=256, w=256, cout=3):
    """Multiply-adds x 2 of one forward pass of the network on an h x w image."""
    ch = [base * 2 ** l for l in range(levels)]
    f, cin = 0, 1
    for l in range(levels):
        px = (h >> l) * (w >> l)
        f += 2 * px * 9 * (cin * ch[l] + ch[l] * ch[l])
        cin = ch[l]
    for l in range(levels - 2, -1, -1):
        px = (h >> l) * (w >> l)
        f += 2 * px * (ch[l + 1] * ch[l] + 9 * (2 * ch[l] * ch[l] + ch[l] * ch[l]))
    return f + 2 * h * w * ch[0] * cout


def throughput(batch=8, steps=20, size=256, base=32, log=print):
    """Training and inference rate of the network on random data (no solver):
    seconds per Adam step and per forward batch, and the matrix-core rate
    counting 3 forward passes per training image."""
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn(batch * steps, size, size, device="cuda", generator=g)
    t = torch.randn(batch * steps, 3, size, size, device="cuda", generator=g)
    net = WarmStartNet(4, base, 3, seed=0)
    net.train(x[:batch], t[:batch], 1, batch, 1e-4)  # warm-up (buffers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.train(x, t, 1, batch, 1e-4)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / steps
    y = torch.empty(batch, 3, size, size, device="cuda")
    fwd = lambda: L.check(L.load().pat_warmstart_forward(net._h, batch, size, size, C.c_void_p(x.data_ptr()),
                                                         C.c_void_p(y.data_ptr()), _stream()))
    fwd()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fwd()
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / steps
    f1 = unet_flops(base, 4, size, size, 3)
    res = dict(batch=batch, size=size, step_ms=t_step * 1e3, forward_ms=t_fwd * 1e3,
               train_tflops=3 * f1 * batch / t_step * 1e-12, forward_tflops=f1 * batch / t_fwd * 1e-12,
               gflop_forward_per_image=f1 * 1e-9)
    log(f"throughput: {res}")
    return res


def _summarise(ev, log):
    """Mean and median iterations and seconds (inference included) per start."""
    summary = {}
    if not ev:
        return summary
    for name in STARTS:
        if name not in ev[0]:
            continue
        it = [r[name]["iters"] for r in ev]
        sec = [r[name]["seconds"] for r in ev]
        fb = sum(r[name]["fallback"] for r in ev)
        summary[name] = dict(iters_mean=float(np.mean(it)), iters_median=float(np.median(it)),
                             seconds_mean=float(np.mean(sec)), seconds_median=float(np.median(sec)),
                             fallbacks=fb)
        log(f"{name:15s} mean iters {np.mean(it):8.0f} median {np.median(it):8.0f}  mean s {np.mean(sec):7.3f} "
            f"median s {np.median(sec):7.3f}  fallbacks {fb}")
    return summary


def _evaluate_cmd(argv):
    """evaluate --weights W --seeds A:B [--report R]: time to the gap from
    zero, the backprojection and the network's starts on held-out seeds; the
    summary is also written into the weights' manifest."""
    import os
    import phantoms
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd")
    ap.add_argument("--weights", required=True)
    ap.add_argument("--seeds", default="50000:50064")
    ap.add_argument("--lam", type=float, default=0.02)
    ap.add_argument("--gap-tol", type=float, default=1e-4)
    ap.add_argument("--cap", type=int, default=200000)
    ap.add_argument("--report", default=None)
    a = ap.parse_args(argv)

    def log(m):
        print(f"[warmstart] {m}", flush=True)

    wl = phantoms.WORKLOADS["tv256"]
    desc = phantoms.geometry_desc(wl.n, wl.n_det, wl.n_t)
    geom = pat.Geometry(dtype=torch.float64, **desc)
    net = WarmStartNet(4, 32, 3, seed=0)
    net.load_weights(a.weights)
    lo, hi = (int(x) for x in a.seeds.split(":"))
    f0, _, _ = synth_data(desc, lo, dtype=geom.dtype)
    net.infer(geom, f0, pat.Reg("tv", a.lam), dual=True)  # untimed warm-up of the inference buffers
    ev = evaluate(geom, desc, net, list(range(lo, hi)), a.lam, a.gap_tol, a.cap, log=log)
    summary = _summarise(ev, log)
    if a.report:
        with open(a.report, "w") as fh:
            json.dump(dict(eval=ev, summary=summary, args=vars(a)), fh)
    man = os.path.splitext(a.weights)[0] + ".json"
    with open(man) as fh:
        m = json.load(fh)
    m["evaluation"] = dict(seeds=f"{lo}..{hi - 1}", gap_tol=a.gap_tol, dtype="f64",
                           note="seconds include the network's inference", summary=summary)
    with open(man, "w") as fh:
        json.dump(m, fh, indent=1)
    return 0


def _main(argv=None):
    import phantoms
    if argv is None:
        argv = sys.argv[1:]
    if argv and argv[0] == "throughput":
        tp = argparse.ArgumentParser()
        tp.add_argument("cmd")
        tp.add_argument("--batch", type=int, default=8)
        tp.add_argument("--steps", type=int, default=20)
        b = tp.parse_args(argv)
        throughput(b.batch, b.steps, log=lambda m: print(f"[warmstart] {m}", flush=True))
        return 0
    if argv and argv[0] == "evaluate":
        return _evaluate_cmd(argv)
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train"])
    ap.add_argument("--n-train", type=int, default=512)
    ap.add_argument("--n-val", type=int, default=16)
    ap.add_argument("--n-test", type=int, default=4)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--lam", type=float, default=0.02)
    ap.add_argument("--target-dtype", choices=["f32", "f64"], default="f32")
    ap.add_argument("--target-gap", type=float, default=1e-3)
    ap.add_argument("--gap-tol", type=float, default=1e-4)
    ap.add_argument("--cap", type=int, default=200000)
    ap.add_argument("--epochs", type=int, default=240)
    ap.add_argument("--chunk", type=int, default=10, help="epochs per training call")
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--out", required=True)
    ap.add_argument("--report", default=None)
    a = ap.parse_args(argv)

    def log(m):
        print(f"[warmstart] {m}", flush=True)

    wl = phantoms.WORKLOADS["tv256"]
    desc = phantoms.geometry_desc(a.size, wl.n_det, wl.n_t)
    geom = pat.Geometry(dtype=torch.float64, **desc)
    tgeom = geom if a.target_dtype == "f64" else pat.Geometry(dtype=torch.float32, **desc)
    train_seeds = list(range(10000, 10000 + a.n_train))
    val_seeds = list(range(40000, 40000 + a.n_val))
    test_seeds = list(range(50000, 50000 + a.n_test))
    x, t, st = make_pairs(tgeom, desc, train_seeds, a.lam, a.target_gap, a.cap, log=log)
    log(f"pairs done: {st['seconds']:.1f} s, mean iters {np.mean(st['iters']):.0f}, "
        f"dropped {st['dropped']}")
    xv, tv, _ = make_pairs(tgeom, desc, val_seeds, a.lam, a.target_gap, a.cap)
    net = WarmStartNet(4, a.base, 3, seed=1)
    t0 = time.perf_counter()
    done, hist = 0, []
    while done < a.epochs:
        ep = min(a.chunk, a.epochs - done)
        # step schedule: lr for 60% of the epochs, lr/3 for the next 25%, lr/10 after
        frac = done / a.epochs
        lr = a.lr if frac < 0.6 else (a.lr / 3 if frac < 0.85 else a.lr / 10)
        loss = net.train(x, t, ep, a.batch, lr, seed=2 + done)
        done += ep
        vl = val_loss(net, xv, tv, a.batch)
        hist.append(dict(epoch=done, lr=lr, loss=loss, val=vl))
        log(f"epoch {done}: lr {lr:.1e} train {loss:.4e} val {vl:.4e} ({time.perf_counter() - t0:.0f} s)")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    net.save_weights(a.out)
    ev = evaluate(geom, desc, net, test_seeds, a.lam, a.gap_tol, a.cap, log=log) if a.n_test > 0 else []
    summary = _summarise(ev, log)
    rep = dict(pairs=st, train_seconds=t_train, history=hist, eval=ev, summary=summary, args=vars(a))
    if a.report:
        with open(a.report, "w") as fh:
            json.dump(rep, fh)
    import os
    manifest = dict(
        network=dict(levels=4, base_channels=a.base, outputs=["u/s", "r_x/lambda", "r_y/lambda"],
                     parameters=net.n_params),
        operator_fingerprint=operator_fingerprint(),
        workload=(f"{a.size}x{a.size} TV (lambda {a.lam}), {wl.n_det} detectors on a closed circle of radius "
                  f"1.2, {wl.n_t} time samples; mixed disc/vessel/segment phantoms, noise U(1%, 10%)"),
        training=dict(pairs=len(st["iters"]), dropped=st["dropped"], train_seeds=f"10000..{10000 + a.n_train - 1}",
                      val_seeds=f"40000..{40000 + a.n_val - 1}",
                      targets=f"PDHG TV solutions in {a.target_dtype.upper()} to rel_gap {a.target_gap} (batched)",
                      target_generation_s=st["seconds"], epochs=a.epochs, batch=a.batch,
                      lr=f"{a.lr}, /3 after 60% of the epochs, /10 after 85%", train_s=t_train,
                      final_train_loss=hist[-1]["loss"], final_val_loss=hist[-1]["val"]),
        evaluation=dict(seeds=f"50000..{50000 + a.n_test - 1}", gap_tol=a.gap_tol, dtype="f64",
                        summary=summary))
    with open(os.path.splitext(a.out)[0] + ".json", "w") as fh:
        json.dump(manifest, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(_main())
