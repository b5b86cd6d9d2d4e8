"""Preconditioned PDHGM (Algorithms 1 and 2) with its gap, in float64.

Test infrastructure only (see the package docstring).

Models (Sec. 3.1, eqs. PD_TV and PD_TGV), with F1 = 1/2 ||. - f||^2:

  tv  : x = u,      K x = (A u, grad u),            F2 = lam ||.||_{2,1},  G = 0
  dtv : x = u,      K x = (A u, D grad u),          F2 = lam ||.||_{2,1},  G = 0
  tgv : x = (u, v), K x = (A u, grad u - v, E v),   F2 = alpha1 ||.||_{2,1},
                                                    F3 = alpha0 ||.||_{F,1}, G = 0
  lst : x = u,      K x = A u,                      G = alpha/2 ||u||^2
        (Tikhonov least squares of Sec. 2; a pin with a closed-form solution)
  wav : x = u,      K x = (A u, W u),               F2 = lam ||.||_1,      G = 0
        (eq. min_wav: Algorithm 1 with grad -> W and div -> W^{-1} = W^T,
        W the dual-tree transform of oracle.wavelet; the dual r holds one
        real number per coefficient, so the prox of F2* clips it to [-lam, lam])

Step sizes (Sec. 3.3.2):
  diag  -- sigma_i = 1/sum_j |K_ij|, tau_j = 1/sum_i |K_ij| over the stacked K
           (diagonal preconditioning); the rows of one pixel's dual vector share
           the smallest of their sigmas so that the pointwise projection stays
           the exact prox; rows without entries get sigma = 1. For wav the W
           rows take sigma = 1 and W's column sums are replaced by 1: in the
           lemma behind the diagonal steps, Cauchy-Schwarz on the W rows gives
           way to Parseval's identity ||W x|| = ||x||, so with tau_j =
           1/(sum_i |A_ij| + 1) the preconditioned operator still has norm <= 1.
  block -- the paper's two-block rule: sigma1 tau L1^2 < 1/4, sigma2 tau L2^2 < 1/4
           with L1 = ||A|| and L2 the norm of the regulariser block, here
           tau = 1/(2 max(L1, L2)), sigma_i = 0.99/(4 tau L_i^2), norms by power
           iteration (1000 steps) times 1.05 (the top of the gradient's spectrum is
           clustered, so the power estimate approaches from below slowly).

Accelerated PDHGM (Sec. 3.3 mentions the O(1/n^2) rate of Chambolle and
Pock's Algorithm 2 when part of the objective is uniformly convex):
accel_schedule gives per-iteration multipliers of the primal and dual steps
and the extrapolation theta_n. The rate holds for LS-T, whose G is strongly
convex; for TV, TGV and dTV (G = 0) a positive gamma only makes the schedule
shift weight from the primal to the dual steps until its bound freezes it.

Gap (Sec. 3.3.3): with G = 0 the conjugate G* is the indicator of {0}, so the
printed gap is infinite until K^T y = 0 exactly. The gap used restricts x to the
box ||x||_inf <= C, whose conjugate is C ||.||_1:

  gap = P(x) + F*(y) + C ||K^T y||_1,   F*(y) = 1/2||q||^2 + <q, f>  (r, s feasible)

which bounds P(x) - min P from above whenever the box holds a minimiser.
rel_gap = gap / P(x). For lst the gap is the exact Fenchel gap.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .operators import grad_matrix, sym_grad_matrix, dtv_matrix
from .wavelet import dtwt_matrix
from .prox import prox_f1_conj, project_ball, prox_tikhonov


class Problem:
    """One reconstruction problem: A, data f, regulariser and its weights."""

    def __init__(self, A, f, nx, ny, kind, lam, alpha0=0.0, eta=1.0, theta=None, levels=3):
        self.A = sp.csr_matrix(A)
        self.f = np.asarray(f, dtype=np.float64).reshape(-1)
        self.nx, self.ny = nx, ny
        self.N = nx * ny
        self.kind = kind
        self.lam = float(lam)
        self.alpha0 = float(alpha0)
        self.eta = float(eta)
        self.theta = theta
        if kind in ("tv", "tgv"):
            self.B = grad_matrix(nx, ny)
        elif kind == "dtv":
            self.B = dtv_matrix(nx, ny, theta, eta)
        elif kind == "lst":
            self.B = None
        elif kind == "wav":
            self.levels = int(levels)
            self.B = dtwt_matrix(nx, ny, self.levels)
        else:
            raise ValueError(kind)
        self.E = sym_grad_matrix(nx, ny) if kind == "tgv" else None

    # -- the stacked operator of Sec. 3.3.2 ------------------------------------
    def stacked(self) -> sp.csr_matrix:
        A, N = self.A, self.N
        if self.kind == "lst":
            return A
        if self.kind in ("tv", "dtv", "wav"):
            return sp.vstack([A, self.B], format="csr")
        Z = sp.csr_matrix((A.shape[0], 2 * N))
        I2 = sp.identity(2 * N, format="csr")
        Z2 = sp.csr_matrix((4 * N, N))
        return sp.vstack([sp.hstack([A, Z]),
                          sp.hstack([self.B, -I2]),
                          sp.hstack([Z2, self.E])], format="csr")

    def reg_block(self) -> sp.csr_matrix:
        """The part of K that is not A (acting on x)."""
        N = self.N
        if self.kind in ("tv", "dtv", "wav"):
            return self.B
        I2 = sp.identity(2 * N, format="csr")
        Z2 = sp.csr_matrix((4 * N, N))
        return sp.vstack([sp.hstack([self.B, -I2]), sp.hstack([Z2, self.E])], format="csr")


def precond_diag(p: Problem) -> dict:
    """sigma_i = 1/sum_j|K_ij|, tau_j = 1/sum_i|K_ij|, block-min over dual vectors
    (wav: sigma_r = 1, tau_j = 1/(sum_i|A_ij| + 1); see the module doc)."""
    if p.kind == "wav":
        A = abs(p.A)
        rs = np.asarray(A.sum(axis=1)).reshape(-1)
        cs = np.asarray(A.sum(axis=0)).reshape(-1)
        sig = np.where(rs > 0, 1.0 / np.where(rs > 0, rs, 1.0), 1.0)
        return dict(sigma_q=sig, tau_u=1.0 / (cs + 1.0), sigma_r=np.ones(p.B.shape[0]))
    K = abs(p.stacked())
    rs = np.asarray(K.sum(axis=1)).reshape(-1)
    cs = np.asarray(K.sum(axis=0)).reshape(-1)
    sig = np.where(rs > 0, 1.0 / np.where(rs > 0, rs, 1.0), 1.0)
    tau = np.where(cs > 0, 1.0 / np.where(cs > 0, cs, 1.0), 1.0)
    m, N = p.A.shape[0], p.N
    out = dict(sigma_q=sig[:m], tau_u=tau[:N])
    if p.kind in ("tv", "dtv", "tgv"):
        out["sigma_r"] = sig[m:m + 2 * N].reshape(2, N).min(axis=0)
    if p.kind == "tgv":
        out["sigma_s"] = sig[m + 2 * N:m + 6 * N].reshape(4, N).min(axis=0)
        out["tau_v"] = tau[N:].reshape(2, N)
    return out


def power_norm(M: sp.spmatrix, iters: int = 200) -> float:
    """||M||_2 by power iteration on M^T M.

    The start vector x_j = 1 + (j mod 5)/4 is deterministic and, unlike the
    all-ones vector, not in the kernel of the gradient.
    """
    x = 1.0 + (np.arange(M.shape[1]) % 5) / 4.0
    x /= np.linalg.norm(x)
    lam = 0.0
    for _ in range(iters):
        y = M.T @ (M @ x)
        lam = np.linalg.norm(y)
        if lam == 0.0:
            return 0.0
        x = y / lam
    return float(np.sqrt(lam))


BLOCK_POWER_ITERS = 1000
BLOCK_SAFETY = 1.05


def precond_block(p: Problem, iters: int = BLOCK_POWER_ITERS) -> dict:
    """The paper's two-block scalar step sizes (Sec. 3.3.2)."""
    L1 = BLOCK_SAFETY * power_norm(p.A, iters)
    if p.kind == "lst":
        tau = 1.0 / (2.0 * L1)
        return dict(sigma_q=np.full(p.A.shape[0], 0.99 / (4 * tau * L1 * L1)),
                    tau_u=np.full(p.N, tau), L1=L1, L2=0.0)
    L2 = BLOCK_SAFETY * power_norm(p.reg_block(), iters)
    tau = 1.0 / (2.0 * max(L1, L2))
    s1 = 0.99 / (4.0 * tau * L1 * L1)
    s2 = 0.99 / (4.0 * tau * L2 * L2)
    N = p.N
    out = dict(sigma_q=np.full(p.A.shape[0], s1),
               sigma_r=np.full(p.B.shape[0] if p.kind == "wav" else N, s2),
               tau_u=np.full(N, tau), L1=L1, L2=L2)
    if p.kind == "tgv":
        out["sigma_s"] = np.full(N, s2)
        out["tau_v"] = np.full((2, N), tau)
    return out


# -- objective, conjugates and the gap -------------------------------------------

def _pointwise_norm_sum(z: np.ndarray) -> float:
    return float(np.sum(np.sqrt(np.sum(z * z, axis=0))))


def primal_objective(p: Problem, u, v=None) -> float:
    """P(x) of eq. min_TV / min_TGV (and LS-T)."""
    res = p.A @ u - p.f
    P = 0.5 * float(res @ res)
    if p.kind in ("tv", "dtv"):
        P += p.lam * _pointwise_norm_sum((p.B @ u).reshape(2, p.N))
    elif p.kind == "wav":
        P += p.lam * float(np.sum(np.abs(p.B @ u)))
    elif p.kind == "tgv":
        P += p.lam * _pointwise_norm_sum((p.B @ u).reshape(2, p.N) - v)
        P += p.alpha0 * _pointwise_norm_sum((p.E @ v.reshape(-1)).reshape(4, p.N))
    elif p.kind == "lst":
        P += 0.5 * p.lam * float(u @ u)
    return P


def gap_terms(p: Problem, st: dict, box: float) -> dict:
    """P, F*, ||K^T y||_1 and the (box-restricted) gap at the state st."""
    u, q = st["u"], st["q"]
    P = primal_objective(p, u, st.get("v"))
    Fs = 0.5 * float(q @ q) + float(q @ p.f)
    Atq = p.A.T @ q
    if p.kind == "lst":
        dual_g = float(Atq @ Atq) / (2.0 * p.lam)   # G*(-A^T q) for G = alpha/2||.||^2
        gap = P + Fs + dual_g
        return dict(P=P, Fstar=Fs, R=dual_g, gap=gap, rel_gap=gap / P if P > 0 else 0.0)
    r = st["r"]
    ku = Atq + p.B.T @ r.reshape(-1)
    R = float(np.sum(np.abs(ku)))
    if p.kind == "tgv":
        kv = (p.E.T @ st["s"].reshape(-1)).reshape(2, p.N) - r
        R += float(np.sum(np.abs(kv)))
    gap = P + Fs + box * R
    return dict(P=P, Fstar=Fs, R=R, gap=gap, rel_gap=gap / P if P > 0 else 0.0)


def warm_start_rejected(p: Problem, u0, v0=None) -> bool:
    """Fallback rule for a warm start: non-finite, or P(u0) > P(0) = 1/2||f||^2."""
    if not np.all(np.isfinite(u0)):
        return True
    if v0 is None and p.kind == "tgv":
        v0 = np.zeros((2, p.N))
    return primal_objective(p, u0, v0) > 0.5 * float(p.f @ p.f)


# -- Algorithms 1 and 2 -----------------------------------------------------------

def init_state(p: Problem, u0=None) -> dict:
    N, m = p.N, p.A.shape[0]
    u = np.zeros(N) if u0 is None else np.asarray(u0, dtype=np.float64).reshape(-1).copy()
    st = dict(u=u, ubar=u.copy(), q=np.zeros(m), n=0)
    if p.kind in ("tv", "dtv", "tgv"):
        st["r"] = np.zeros((2, N))
    elif p.kind == "wav":
        st["r"] = np.zeros((1, p.B.shape[0]))
    if p.kind == "tgv":
        st["v"] = np.zeros((2, N))
        st["vbar"] = np.zeros((2, N))
        st["s"] = np.zeros((4, N))
    return st


def pdhg_step(p: Problem, pc: dict, st: dict, theta: float = 1.0,
              dual_mult: float = 1.0, primal_mult: float = 1.0) -> None:
    """One iteration: the dual steps at (ubar[, vbar]), then the primal steps,
    then the extrapolation (Algorithm 1 for tv/dtv, Algorithm 2 for tgv).

    dual_mult and primal_mult scale every dual step size (sigma) and every
    primal step size (tau) of this iteration; the accelerated variant varies
    them from one iteration to the next (see accel_schedule)."""
    A, N = p.A, p.N
    if dual_mult != 1.0 or primal_mult != 1.0:
        pc = {k: (v * primal_mult if k.startswith("tau") else v * dual_mult)
              for k, v in pc.items() if k.startswith(("tau", "sigma"))}
    sq = pc["sigma_q"]
    # q^{n+1} = prox_{sigma1 F1*}(q^n + sigma1 K ubar^n)
    st["q"] = prox_f1_conj(st["q"] + sq * (A @ st["ubar"]), p.f, sq)
    q = st["q"]
    u_old = st["u"]
    if p.kind in ("tv", "dtv", "wav"):
        # r^{n+1} = prox_{sigma2 F2*}(r^n + sigma2 B ubar^n)
        Bu = (p.B @ st["ubar"]).reshape(st["r"].shape)
        st["r"] = project_ball(st["r"] + pc["sigma_r"] * Bu, p.lam)
        # u^{n+1} = u^n - tau (A^T q^{n+1} + B^T r^{n+1})
        u_new = u_old - pc["tau_u"] * (A.T @ q + p.B.T @ st["r"].reshape(-1))
    elif p.kind == "tgv":
        Gu = (p.B @ st["ubar"]).reshape(2, N)
        st["r"] = project_ball(st["r"] + pc["sigma_r"] * (Gu - st["vbar"]), p.lam)
        Ev = (p.E @ st["vbar"].reshape(-1)).reshape(4, N)
        st["s"] = project_ball(st["s"] + pc["sigma_s"] * Ev, p.alpha0)
        u_new = u_old - pc["tau_u"] * (A.T @ q + p.B.T @ st["r"].reshape(-1))
        Ets = (p.E.T @ st["s"].reshape(-1)).reshape(2, N)
        v_new = st["v"] - pc["tau_v"] * (Ets - st["r"])
        st["vbar"] = v_new + theta * (v_new - st["v"])
        st["v"] = v_new
    elif p.kind == "lst":
        u_new = prox_tikhonov(u_old - pc["tau_u"] * (A.T @ q), pc["tau_u"], p.lam)
    st["ubar"] = u_new + theta * (u_new - u_old)
    st["u_prev"] = u_old
    st["u"] = u_new
    st["n"] += 1


def accel_schedule(gamma: float, step_max: float):
    """Step multipliers of the accelerated PDHGM (Chambolle and Pock's
    Algorithm 2, the O(1/n^2) variant that Sec. 3.3 mentions), applied to the
    preconditioned steps: iteration n takes the dual steps b_n Sigma and the
    primal steps a_n T, then extrapolates with theta_n, where

      a_0 = b_0 = 1,  theta_n = 1 / sqrt(1 + 2 gamma a_n),
      a_{n+1} = theta_n a_n,  b_{n+1} = b_n / theta_n   (so a_n b_n = 1).

    gamma is the modulus of strong convexity of G in the metric of T (for
    G = alpha/2 ||u||^2 with diagonal T: alpha min_j T_jj). The first
    update that would take b above step_max is not made: from then on
    theta_n = 1 and a_n, b_n stay fixed, i.e. plain PDHGM with the steps
    (a T, b Sigma), whose product is unchanged, so the iteration converges to
    a saddle point of the same problem. Yields (b_n, a_n, theta_n)."""
    a = b = 1.0
    frozen = gamma <= 0.0
    while True:
        th = 1.0
        if not frozen:
            th = 1.0 / np.sqrt(1.0 + 2.0 * gamma * a)
            if b / th > step_max:
                frozen, th = True, 1.0
        yield b, a, th
        if not frozen:
            a, b = th * a, b / th


def residual(st: dict) -> float:
    """||u^n - u^{n-1}|| / ||u^{n-1}|| (Sec. 3.3.3, norm in the denominator)."""
    prev = st.get("u_prev")
    if prev is None:
        return float("nan")
    den = np.linalg.norm(prev)
    return float(np.linalg.norm(st["u"] - prev) / den) if den > 0 else float("inf")


def pdhg_solve(p: Problem, pc: dict, iters: int | None = None, tol: float | None = None,
               max_iter: int = 2000, gap_every: int = 10, box: float = 2.0,
               u0=None, theta: float = 1.0, state: dict | None = None,
               accel_gamma: float = 0.0, accel_step_max: float = 1.0) -> dict:
    """Run PDHGM for a fixed number of iterations, or until rel_gap <= tol
    (checked every gap_every iterations, capped at max_iter). With
    accel_gamma > 0 the step sizes and the extrapolation follow
    accel_schedule (theta is then 1 after the schedule freezes)."""
    st = state if state is not None else init_state(p, u0)
    history = []
    n_target = iters if iters is not None else max_iter
    sched = accel_schedule(accel_gamma, accel_step_max) if accel_gamma > 0.0 else None
    while st["n"] < n_target:
        if sched is not None:
            b, a, th = next(sched)
            pdhg_step(p, pc, st, th, dual_mult=b, primal_mult=a)
        else:
            pdhg_step(p, pc, st, theta)
        if tol is not None and (st["n"] % gap_every == 0 or st["n"] == n_target):
            g = gap_terms(p, st, box)
            g["n"] = st["n"]
            g["residual"] = residual(st)
            history.append(g)
            if g["rel_gap"] <= tol:
                break
    st["history"] = history
    return st
