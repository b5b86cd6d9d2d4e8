"""Pins of the FP64 oracle against mathematics it does not compute itself.

Each test would fail on a plausible slip in the oracle: a swapped x/y, a wrong
arc phase or normalisation, a dropped boundary row, a wrong prox sign, a step
size that breaks the preconditioning bound, a gap with a wrong term.
"""
import math

import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

import phantoms
from oracle import geometry as G
from oracle import metrics as M
from oracle import operators as O
from oracle import pdhg as P
from oracle import prox as X

from closed_forms import (disc_circular_mean, gaussian_circular_mean,
                          grad_norm_squared, textbook_divergence)


def _geom(n, n_det, n_t, **kw):
    d = phantoms.geometry_desc(n, n_det, n_t)
    d.update(kw)
    return G.make_geometry(d)


# ---------------------------------------------------------------- forward operator

def test_forward_reproduces_bilinear_polynomials():
    """Bilinear interpolation reproduces span{1, x, y, xy}; equispaced arc
    samples average cos, sin and sin(2 phi) to zero (M >= 2). So for circles
    inside the pixel-centre hull the circular mean of a + bx + cy + dxy is the
    value at the detector: a + b px + c py + d px py."""
    n = 48
    dets = np.array([[0.05, -0.1], [-0.3, 0.2], [0.41, 0.37]])
    g = _geom(n, 3, 40, det_xy=dets, dt=0.6 / 39)
    A = G.forward_matrix(g)
    Xc, Yc = phantoms.pixel_centres(n)
    a, b, c, d = 0.3, -1.7, 0.9, 2.3
    u = a + b * Xc + c * Yc + d * Xc * Yc
    f = (A @ u.ravel()).reshape(3, 40)
    lo, hi = g.pixel_x()[0], g.pixel_x()[-1]
    Ms = g.n_samples()
    checked = 0
    for k_det, (px, py) in enumerate(dets):
        want = a + b * px + c * py + d * px * py
        for k, r in enumerate(g.radii):
            inside = (px - r >= lo) and (px + r <= hi) and (py - r >= lo) and (py + r <= hi)
            if inside and Ms[k] >= 2:
                assert f[k_det, k] == pytest.approx(want, abs=1e-12)
                checked += 1
    assert checked > 40


@pytest.mark.parametrize("kind", ["disc", "gauss"])
def test_forward_converges_to_circular_mean(kind):
    """Against closed-form circular means: O(h) for a uniform disc (circle-circle
    intersection arc), O(h^2) for a Gaussian blob."""
    c = np.array([0.2, -0.1])
    errs = []
    for n in (64, 128, 256):
        g = _geom(n, 4, 96, arc_center=0.3)
        A = G.forward_matrix(g)
        Xc, Yc = phantoms.pixel_centres(n)
        if kind == "disc":
            R, ss, h = 0.4, 8, 2.0 / n
            off = (np.arange(ss) + 0.5) / ss * h - h / 2
            u = np.zeros_like(Xc)
            for ox in off:
                for oy in off:
                    u += ((Xc + ox - c[0]) ** 2 + (Yc + oy - c[1]) ** 2) <= R * R
            u /= ss * ss
        else:
            s = 0.15
            u = np.exp(-((Xc - c[0]) ** 2 + (Yc - c[1]) ** 2) / (2 * s * s))
        f = (A @ u.ravel()).reshape(4, 96)
        ref = np.empty_like(f)
        for d in range(4):
            rho = float(np.hypot(*(g.det_xy[d] - c)))
            ref[d] = (disc_circular_mean(g.radii, rho, 0.4) if kind == "disc"
                      else gaussian_circular_mean(g.radii, rho, 0.15))
        errs.append(np.linalg.norm(f - ref) / np.linalg.norm(ref))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    if kind == "disc":
        assert errs[-1] < 0.01 and all(1.6 < q < 2.5 for q in ratios), (errs, ratios)
    else:
        assert errs[-1] < 3e-4 and all(3.3 < q < 4.8 for q in ratios), (errs, ratios)


def test_forward_invariants():
    """A >= 0; rows sum to at most 1 (partition of unity of the hat basis),
    exactly 1 when every sample of the arc lies inside the pixel-centre hull,
    0 when the circle misses the grid."""
    g = _geom(32, 8, 64)
    A = G.forward_matrix(g)
    assert A.data.min() >= 0.0
    rs = np.asarray(A.sum(axis=1)).reshape(-1)
    assert rs.max() <= 1.0 + 1e-12
    lo, hi = g.pixel_x()[0], g.pixel_x()[-1]
    full = 0
    for d, (px, py) in enumerate(g.det_xy):
        for k, r in enumerate(g.radii):
            b = d * g.n_t + k
            if px - r >= lo and px + r <= hi and py - r >= lo and py + r <= hi:
                assert rs[b] == pytest.approx(1.0, abs=1e-12)
                full += 1
            far = max(math.hypot(px - sx, py - sy) for sx in (-1, 1) for sy in (-1, 1))
            if r > far + 0.1:
                assert rs[b] == 0.0
    # detectors at 45 degrees lie inside the square, so some circles fit
    assert full > 0
    g2 = _geom(32, 2, 20, det_xy=np.array([[0.0, 0.0], [0.1, -0.2]]), dt=0.5 / 19)
    rs2 = np.asarray(G.forward_matrix(g2).sum(axis=1)).reshape(-1)
    assert np.allclose(rs2, 1.0, atol=1e-12)


def test_forward_rows_match_matrix():
    g = _geom(24, 5, 30)
    A = G.forward_matrix(g)
    bins = np.array([0, 7, 33, 99, 149])
    R = G.forward_rows(g, bins)
    assert abs(R - A[bins]).max() < 1e-15


def test_arc_detector_positions():
    """Closed circle: 2 pi d / n from the centre angle; arcs: both ends included."""
    p = G.detector_positions(4, 0.0, 0.0, 1.2, 0.0, 2 * math.pi)
    assert np.allclose(p, [[1.2, 0], [0, 1.2], [-1.2, 0], [0, -1.2]], atol=1e-15)
    q = G.detector_positions(3, 0.0, 0.0, 2.0, 0.0, math.pi / 2)
    s = math.sqrt(2.0)
    assert np.allclose(q, [[s, -s], [2.0, 0.0], [s, s]], atol=1e-15)


def test_arc_sample_count_and_phase():
    """M_k is 2 pi r_k / h rounded up to a multiple of 4 (h = 1/8, r_k = k/20:
    2.51, 5.03, 7.54, 10.05 samples of arc length give 4, 8, 8, 12); r_0 = 0
    is a single sample."""
    g = _geom(16, 1, 5, det_xy=np.array([[0.0, 0.0]]), dt=0.05)
    assert list(g.n_samples()) == [1, 4, 8, 8, 12]
    # r_0 = 0: one sample at the detector itself, which is a pixel corner here,
    # so the four surrounding pixels share weight 1/4 each
    row = G.forward_rows(g, np.array([0])).toarray().reshape(16, 16)
    assert np.allclose(row[7:9, 7:9], 0.25) and row.sum() == pytest.approx(1.0)


def test_arc_sample_phase_by_hand():
    """A detector on the centre of pixel (i, j) = (5, 9) and r = 0.3 h gives
    M = 4 samples at phi = pi/4 + k pi/2, i.e. at offsets (+-a, +-a) pixels with
    a = 0.3 / sqrt(2). Worked by hand from the hat functions, averaged over
    the four samples: the pixel keeps (1 - a)^2, each of its four edge
    neighbours gets a (1 - a) / 2 and each diagonal neighbour a^2 / 4 =
    0.01125."""
    n, h = 16, 2.0 / 16
    x = -1.0 + 5.5 * h
    y = -1.0 + 9.5 * h
    g = _geom(n, 1, 2, det_xy=np.array([[x, y]]), dt=0.3 * h)
    assert list(g.n_samples()) == [1, 4]
    row = G.forward_rows(g, np.array([1])).toarray().reshape(n, n)
    a = 0.3 / math.sqrt(2.0)
    want = np.zeros((n, n))
    want[9, 5] = (1 - a) ** 2
    want[8, 5] = want[10, 5] = want[9, 4] = want[9, 6] = a * (1 - a) / 2
    want[8, 4] = want[8, 6] = want[10, 4] = want[10, 6] = 0.01125
    assert np.allclose(row, want, atol=1e-14)


def _quarter_turn(u):
    """Image rotated by +90 degrees about the grid centre: pixel (col i, row j)
    moves to (col n-1-j, row i)."""
    n = u.shape[0]
    out = np.empty_like(u)
    j, i = np.mgrid[0:n, 0:n]
    out[i, n - 1 - j] = u[j, i]
    return out


@pytest.mark.parametrize("n,n_det,n_t", [(24, 8, 40), (17, 12, 33)])
def test_quarter_turn_equivariance(n, n_det, n_t):
    """Detectors evenly spaced on a closed circle about the grid centre, n_det
    a multiple of 4: turning the image by 90 degrees about the centre moves
    the data of detector d to detector d + n_det/4 (the samples of every
    circle turn into samples of the same circle because M_k is a multiple of
    four). With the arc length rounded up to any integer instead, the
    sample sets no longer turn into each other and the identity fails."""
    g = _geom(n, n_det, n_t)
    A = G.forward_matrix(g)
    u = np.random.default_rng(8).standard_normal((n, n))
    f = (A @ u.ravel()).reshape(n_det, n_t)
    fr = (A @ _quarter_turn(u).ravel()).reshape(n_det, n_t)
    assert np.abs(fr - np.roll(f, n_det // 4, axis=0)).max() <= 1e-13 * np.abs(f).max()
    # control: the same identity under M_k = ceil(2 pi r_k s / h)
    plain = np.maximum(1, np.ceil(2 * math.pi * g.radii * g.samples_per_pixel / g.h)).astype(np.int64)
    assert np.any(plain % 4 != 0)
    orig = G.Geometry.n_samples
    try:
        G.Geometry.n_samples = lambda self: np.maximum(
            1, np.ceil(2 * math.pi * self.radii * self.samples_per_pixel / self.h)).astype(np.int64)
        A2 = G.forward_matrix(g)
    finally:
        G.Geometry.n_samples = orig
    f2 = (A2 @ u.ravel()).reshape(n_det, n_t)
    fr2 = (A2 @ _quarter_turn(u).ravel()).reshape(n_det, n_t)
    assert np.abs(fr2 - np.roll(f2, n_det // 4, axis=0)).max() > 1e-4 * np.abs(f2).max()


@pytest.mark.parametrize("n,n_det,n_t", [(24, 8, 40), (17, 16, 33)])
def test_mirror_equivariance(n, n_det, n_t):
    """Detectors at angles 2 pi d / n_det from angle 0: mirroring the image
    across the horizontal centre line (row j -> n-1-j) moves the data of
    detector d to detector n_det - d (every circle's samples at angles
    2 pi (m + 1/2) / M_k are mirror symmetric, m -> M_k - 1 - m). A ring
    started half a spacing off has no such pairing."""
    g = _geom(n, n_det, n_t)
    A = G.forward_matrix(g)
    u = np.random.default_rng(10).standard_normal((n, n))
    f = (A @ u.ravel()).reshape(n_det, n_t)
    fm = (A @ u[::-1].ravel()).reshape(n_det, n_t)
    idx = (n_det - np.arange(n_det)) % n_det
    assert np.abs(fm[idx] - f).max() <= 1e-13 * np.abs(f).max()
    g2 = _geom(n, n_det, n_t, arc_center=math.pi / (2 * n_det))
    A2 = G.forward_matrix(g2)
    f2 = (A2 @ u.ravel()).reshape(n_det, n_t)
    fm2 = (A2 @ u[::-1].ravel()).reshape(n_det, n_t)
    assert np.abs(fm2[idx] - f2).max() > 1e-3 * np.abs(f2).max()


# ---------------------------------------------------------------- regulariser operators

def test_grad_norm_closed_form():
    for nx, ny in [(6, 6), (7, 5)]:
        Gm = O.grad_matrix(nx, ny).toarray()
        lam = np.linalg.eigvalsh(Gm.T @ Gm).max()
        assert lam == pytest.approx(grad_norm_squared(nx, ny), rel=1e-12)
        assert P.power_norm(O.grad_matrix(nx, ny), 2000) ** 2 == pytest.approx(lam, rel=1e-6)


def test_grad_on_ramps_and_divergence():
    nx, ny = 7, 5
    Gm = O.grad_matrix(nx, ny)
    iy, ix = np.mgrid[0:ny, 0:nx]
    gx = (Gm @ ix.ravel().astype(float)).reshape(2, ny, nx)
    assert np.all(gx[0][:, :-1] == 1.0) and np.all(gx[0][:, -1] == 0.0) and np.all(gx[1] == 0)
    gy = (Gm @ iy.ravel().astype(float)).reshape(2, ny, nx)
    assert np.all(gy[1][:-1] == 1.0) and np.all(gy[1][-1] == 0.0) and np.all(gy[0] == 0)
    rng = np.random.default_rng(3)
    p = rng.standard_normal((2, ny, nx))
    div = -(Gm.T @ p.ravel()).reshape(ny, nx)
    assert np.allclose(div, textbook_divergence(p[0], p[1]), atol=1e-14)


def test_sym_grad_on_affine_fields():
    """E of v = (a + b i + c j, d + e i + g j) in the interior is
    [b, (c+e)/2, (c+e)/2, g]; on the first column dx- returns the value itself."""
    nx, ny = 6, 5
    E = O.sym_grad_matrix(nx, ny)
    jj, ii = np.mgrid[0:ny, 0:nx].astype(float)
    a, b, c, d, e, g = 0.5, 1.5, -2.0, 0.25, 3.0, -0.75
    vx, vy = a + b * ii + c * jj, d + e * ii + g * jj
    out = (E @ np.concatenate([vx.ravel(), vy.ravel()])).reshape(4, ny, nx)
    inner = (slice(1, ny - 1), slice(1, nx - 1))
    assert np.allclose(out[0][inner], b) and np.allclose(out[3][inner], g)
    assert np.allclose(out[1][inner], 0.5 * (c + e)) and np.array_equal(out[1], out[2])
    assert np.allclose(out[0][:, 0], vx[:, 0])            # dx-: first column = v
    assert np.allclose(out[0][:, -1], -vx[:, -2])         # last column = -v[n-2]


def test_directional_gradient():
    """Ramp along t = (cos th, sin th): D grad u = t; ramp along the normal xi:
    D grad u = eta xi (interior); eta = 1 is the plain gradient."""
    nx = ny = 9
    th, eta = 0.6, 0.1
    theta = np.full((ny, nx), th)
    D = O.dtv_matrix(nx, ny, theta, eta)
    jj, ii = np.mgrid[0:ny, 0:nx].astype(float)
    t = np.array([math.cos(th), math.sin(th)])
    xi = np.array([-math.sin(th), math.cos(th)])
    inner = (slice(0, ny - 1), slice(0, nx - 1))
    out = (D @ (t[0] * ii + t[1] * jj).ravel()).reshape(2, ny, nx)
    assert np.allclose(out[0][inner], t[0]) and np.allclose(out[1][inner], t[1])
    out = (D @ (xi[0] * ii + xi[1] * jj).ravel()).reshape(2, ny, nx)
    assert np.allclose(out[0][inner], eta * xi[0]) and np.allclose(out[1][inner], eta * xi[1])
    D1 = O.dtv_matrix(nx, ny, theta, 1.0)
    assert abs(D1 - O.grad_matrix(nx, ny)).max() < 1e-15


# ---------------------------------------------------------------- proximal maps

def test_prox_f1_conj_brute_force_and_moreau():
    rng = np.random.default_rng(0)
    f = rng.standard_normal(5)
    z = rng.standard_normal(5)
    for gam in (0.3, 2.0):
        def obj(w):
            # F1*(w) = 1/2||w||^2 + <w, f> is the conjugate of 1/2||. - f||^2
            return 0.5 * np.sum((w - z) ** 2) + gam * (0.5 * w @ w + w @ f)
        w = so.minimize(obj, np.zeros(5), method="BFGS", options=dict(gtol=1e-12)).x
        assert np.allclose(X.prox_f1_conj(z, f, gam), w, atol=1e-7)
        # Moreau: prox_{g F*}(z) = z - g prox_{F/g}(z/g); prox_{F1/g}(y) = (g y + f)/(g + 1)
        moreau = z - gam * ((gam * (z / gam) + f) / (gam + 1.0))
        assert np.allclose(X.prox_f1_conj(z, f, gam), moreau, atol=1e-14)


def test_project_ball_brute_force():
    rng = np.random.default_rng(1)
    for dim in (2, 4):
        zs = rng.standard_normal((dim, 6)) * 2
        P_ = X.project_ball(zs, 0.7)
        for p in range(6):
            z = zs[:, p]
            cons = {"type": "ineq", "fun": lambda w: 0.49 - w @ w}
            w = so.minimize(lambda w: 0.5 * np.sum((w - z) ** 2), np.zeros(dim),
                            constraints=[cons], method="SLSQP",
                            options=dict(ftol=1e-14, maxiter=500)).x
            assert np.allclose(P_[:, p], w, atol=1e-6)


# ---------------------------------------------------------------- tiny problems

def _tiny(kind, n=8, n_det=6, n_t=16, seed=0, lam=0.02):
    g = _geom(n, n_det, n_t)
    A = G.forward_matrix(g)
    rng = np.random.default_rng(seed)
    u_true = np.clip(rng.uniform(-0.2, 1.0, (n, n)), 0, None)
    f = A @ u_true.ravel() + 0.01 * rng.standard_normal(A.shape[0])
    theta = rng.uniform(-1.5, 1.5, (n, n))
    return P.Problem(A, f, n, n, kind, lam, alpha0=2 * lam, eta=0.3, theta=theta)


@pytest.mark.parametrize("kind", ["tv", "tgv", "dtv", "lst"])
def test_diag_preconditioner_bound(kind):
    """||Sigma^{1/2} K T^{1/2}|| <= 1 for the diagonal rule (Pock & Chambolle)."""
    p = _tiny(kind)
    pc = P.precond_diag(p)
    K = p.stacked().toarray()
    m, N = p.A.shape[0], p.N
    if kind == "lst":
        sig, tau = pc["sigma_q"], pc["tau_u"]
    elif kind in ("tv", "dtv"):
        sig = np.concatenate([pc["sigma_q"], np.tile(pc["sigma_r"], 2)])
        tau = pc["tau_u"]
    else:
        sig = np.concatenate([pc["sigma_q"], np.tile(pc["sigma_r"], 2), np.tile(pc["sigma_s"], 4)])
        tau = np.concatenate([pc["tau_u"], pc["tau_v"].ravel()])
    assert sig.shape[0] == K.shape[0] and tau.shape[0] == K.shape[1]
    S = np.sqrt(sig)[:, None] * K * np.sqrt(tau)[None, :]
    assert np.linalg.norm(S, 2) <= 1.0 + 1e-12
    assert np.all(sig > 0) and np.all(tau > 0)


@pytest.mark.parametrize("kind", ["tv", "tgv", "dtv"])
def test_block_preconditioner_bound(kind):
    """sqrt(s1 tau) L1 + sqrt(s2 tau) L2 < 1 with the exact norms (Sec. 3.3.2)."""
    p = _tiny(kind)
    pc = P.precond_block(p)
    L1 = np.linalg.norm(p.A.toarray(), 2)
    L2 = np.linalg.norm(p.reg_block().toarray(), 2)
    tau = pc["tau_u"][0]
    assert pc["L1"] >= L1 and pc["L2"] >= L2
    assert math.sqrt(pc["sigma_q"][0] * tau) * L1 + math.sqrt(pc["sigma_r"][0] * tau) * L2 < 1.0


def test_lst_converges_to_normal_equations():
    """LS-T (Sec. 2): u = (A^T A + alpha I)^{-1} A^T f. The objective is
    alpha-strongly convex, so ||u - u*||^2 <= 2 gap / alpha along the way."""
    p = _tiny("lst", lam=0.05)
    Ad = p.A.toarray()
    want = np.linalg.solve(Ad.T @ Ad + p.lam * np.eye(p.N), Ad.T @ p.f)
    st = P.init_state(p)
    pc = P.precond_diag(p)
    for _ in range(20):
        for _ in range(100):
            P.pdhg_step(p, pc, st)
        g = P.gap_terms(p, st, 0.0)
        assert g["gap"] >= -1e-15
        # allowance: the gap's own rounding (about 1e-16 of P)
        assert np.sum((st["u"] - want) ** 2) <= 2 * (max(g["gap"], 0.0) + 1e-15) / p.lam
    st = P.pdhg_solve(p, pc, tol=1e-14, max_iter=400000, gap_every=500, state=st)
    assert np.max(np.abs(st["u"] - want)) < 1e-8


def _smoothed_minimum(p, eps=1e-7):
    """Independent solver: L-BFGS on the objective with every pointwise norm
    |z| replaced by sqrt(|z|^2 + eps^2) (minimum within N eps of the exact one)."""
    A, f, lam, N = p.A, p.f, p.lam, p.N
    B = p.B

    def snorm(z):
        return np.sqrt(np.sum(z * z, axis=0) + eps * eps)

    def fun(x):
        u = x[:N]
        res = A @ u - f
        val = 0.5 * res @ res
        gu = A.T @ res
        if p.kind == "tgv":
            v = x[N:].reshape(2, N)
            z = (B @ u).reshape(2, N) - v
            nz = snorm(z)
            w = (p.E @ v.ravel()).reshape(4, N)
            nw = snorm(w)
            val += lam * nz.sum() + p.alpha0 * nw.sum()
            gu = gu + lam * (B.T @ (z / nz).ravel())
            gv = -lam * (z / nz) + p.alpha0 * (p.E.T @ (w / nw).ravel()).reshape(2, N)
            return val, np.concatenate([gu, gv.ravel()])
        z = (B @ u).reshape(2, N)
        nz = snorm(z)
        return val + lam * nz.sum(), gu + lam * (B.T @ (z / nz).ravel())

    n0 = 3 * N if p.kind == "tgv" else N
    r = so.minimize(fun, np.zeros(n0), jac=True, method="L-BFGS-B",
                    options=dict(maxiter=200000, maxfun=400000, ftol=1e-16, gtol=1e-12))
    return r.fun


@pytest.mark.parametrize("kind,tol", [("tv", 1e-9), ("tgv", 1e-7), ("dtv", 1e-8)])
def test_gap_certificate_and_independent_minimum(kind, tol):
    """PDHG reaches a tiny gap; the gap stays >= 0 with a box holding the
    minimiser; its running maximum over doubling windows decreases; and the
    objective matches an independent smooth solver."""
    p = _tiny(kind, lam=0.01)
    pc = P.precond_diag(p)
    st = P.pdhg_solve(p, pc, tol=tol, max_iter=400000, gap_every=25, box=2.0)
    hist = st["history"]
    assert hist[-1]["rel_gap"] <= tol
    assert np.max(np.abs(st["u"])) < 2.0
    gaps = np.array([h["gap"] for h in hist])
    ns = np.array([h["n"] for h in hist])
    assert np.all(gaps >= -1e-14)
    env = [gaps[(ns >= 2 ** j) & (ns < 2 ** (j + 1))].max()
           for j in range(5, int(np.log2(ns[-1]))) if np.any((ns >= 2 ** j) & (ns < 2 ** (j + 1)))]
    assert all(b < a for a, b in zip(env, env[1:]))
    eps = 1e-7
    ref = _smoothed_minimum(p, eps)
    # min of the smoothed objective lies in [P*, P* + eps * sum of the weights
    # of the pointwise norms]; P(u_pdhg) lies in [P*, P* + gap]
    bias = eps * p.N * (p.lam + (p.alpha0 if kind == "tgv" else 0.0))
    Pn, gap = hist[-1]["P"], hist[-1]["gap"]
    assert ref - bias - 1e-12 <= Pn <= ref + gap + 1e-12, (Pn, ref, bias, gap)


def test_gap_bounds_suboptimality():
    """At any iterate, gap >= P(u) - P* (P* from a far-converged run)."""
    p = _tiny("tgv", lam=0.01)
    pc = P.precond_diag(p)
    ref = P.pdhg_solve(p, pc, tol=1e-10, max_iter=400000, gap_every=50)
    Pstar = ref["history"][-1]["P"] - ref["history"][-1]["gap"]
    st = P.init_state(p)
    for _ in range(6):
        for _ in range(40):
            P.pdhg_step(p, pc, st)
        g = P.gap_terms(p, st, 2.0)
        assert g["gap"] >= g["P"] - Pstar - 1e-12


def test_tgv_without_second_order_is_tv():
    """Alg. 2 with tau_v = 0 and sigma_s = 0 keeps v = s = 0 and takes exactly
    the steps of Alg. 1."""
    p_tgv, p_tv = _tiny("tgv", lam=0.02), _tiny("tv", lam=0.02)
    pc_tv = P.precond_diag(p_tv)
    pc = P.precond_diag(p_tgv)
    pc.update(sigma_r=pc_tv["sigma_r"], tau_u=pc_tv["tau_u"],
              sigma_s=np.zeros(p_tgv.N), tau_v=np.zeros((2, p_tgv.N)))
    a = P.pdhg_solve(p_tgv, pc, iters=60)
    b = P.pdhg_solve(p_tv, pc_tv, iters=60)
    assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["q"], b["q"])
    assert not a["v"].any() and not a["s"].any()


def test_dtv_with_eta_one_is_tv():
    p_tv = _tiny("tv")
    p_d = P.Problem(p_tv.A, p_tv.f, 8, 8, "dtv", p_tv.lam, eta=1.0,
                    theta=np.random.default_rng(5).uniform(-1, 1, (8, 8)))
    a = P.pdhg_solve(p_d, P.precond_diag(p_d), iters=50)
    b = P.pdhg_solve(p_tv, P.precond_diag(p_tv), iters=50)
    assert np.allclose(a["u"], b["u"], rtol=0, atol=1e-15)


def test_warm_start_rule():
    p = _tiny("tv")
    assert P.warm_start_rejected(p, np.full(p.N, np.nan))
    assert P.warm_start_rejected(p, np.full(p.N, 1e3))
    st = P.pdhg_solve(p, P.precond_diag(p), iters=200)
    assert not P.warm_start_rejected(p, st["u"])


def test_psnr_closed_form():
    u = np.zeros((4, 4))
    u[0, 0] = 2.0
    v = u + 0.1
    assert M.psnr(v, u) == pytest.approx(10 * math.log10(4.0 / 0.01))
    assert M.psnr_as_printed(v, u) == pytest.approx(10 * math.log10(2.0 / 0.01))


def test_residual_two_lst_steps_by_hand():
    """Residual of Sec. 3.3.3, ||u^n - u^(n-1)|| / ||u^(n-1)||, after two LS-T
    steps worked by hand. A = diag(1, 2), f = (1, 1), alpha = 1; DIAG steps
    sigma = tau = (1, 1/2); from zero:
      pixel 1: q1 = -1/2, u1 = 1/4, ubar1 = 1/2; q2 = -1/2, u2 = 3/8
      pixel 2: q1 = -1/3, u1 = 2/9, ubar1 = 4/9; q2 = -7/27, u2 = 26/81
    so u2 - u1 = (1/8, 8/81) and the residual is
      sqrt(1/64 + 64/6561) / sqrt(1/16 + 4/81).
    A 1-norm, a missing norm in the denominator or a wrong iterate pair gives
    another number."""
    A = sp.csr_matrix(np.diag([1.0, 2.0]))
    p = P.Problem(A, np.array([1.0, 1.0]), 2, 1, "lst", 1.0)
    pc = P.precond_diag(p)
    assert np.allclose(pc["sigma_q"], [1.0, 0.5]) and np.allclose(pc["tau_u"], [1.0, 0.5])
    st = P.init_state(p)
    P.pdhg_step(p, pc, st)
    assert np.allclose(st["q"], [-1 / 2, -1 / 3], rtol=0, atol=1e-15)
    assert np.allclose(st["u"], [1 / 4, 2 / 9], rtol=0, atol=1e-15)
    assert np.allclose(st["ubar"], [1 / 2, 4 / 9], rtol=0, atol=1e-15)
    assert math.isinf(P.residual(st))  # u^0 = 0: no relative change defined
    P.pdhg_step(p, pc, st)
    assert np.allclose(st["q"], [-1 / 2, -7 / 27], rtol=0, atol=1e-15)
    assert np.allclose(st["u"], [3 / 8, 26 / 81], rtol=0, atol=1e-15)
    want = math.sqrt(1 / 64 + 64 / 6561) / math.sqrt(1 / 16 + 4 / 81)
    assert P.residual(st) == pytest.approx(want, rel=1e-14)


# ---------------------------------------------------------------- accelerated PDHGM

def test_accel_two_lst_steps_by_hand():
    """Two steps of the accelerated variant worked by hand on the 1-pixel LS-T
    problem A = 1, f = 1, alpha = 1 (sigma = tau = 1) with gamma = 1:
      n = 0: b = a = 1: q1 = -1/2, u1 = 1/4; theta0 = 1/sqrt(3),
             ubar1 = u1 + theta0 u1, a1 = 1/sqrt(3), b1 = sqrt(3)
      n = 1: q2 = (q1 + sqrt(3) (ubar1 - 1)) / (1 + sqrt(3))
                = ((-1 - 3 sqrt(3)) / 4) / (1 + sqrt(3)),
             u2 = (u1 - q2 / sqrt(3)) / (1 + 1/sqrt(3)),
             theta1 = 1 / sqrt(1 + 2/sqrt(3)), ubar2 = u2 + theta1 (u2 - u1).
    Using the updated a or b within a step, or the next theta in the
    extrapolation, gives other numbers."""
    r3 = math.sqrt(3.0)
    p = P.Problem(sp.csr_matrix(np.array([[1.0]])), np.array([1.0]), 1, 1, "lst", 1.0)
    pc = P.precond_diag(p)
    st = P.init_state(p)
    sched = P.accel_schedule(1.0, 1e9)
    b, a, th = next(sched)
    assert (b, a) == (1.0, 1.0) and th == pytest.approx(1 / r3, rel=1e-15)
    P.pdhg_step(p, pc, st, th, dual_mult=b, primal_mult=a)
    assert st["q"][0] == pytest.approx(-0.5, rel=1e-15)
    assert st["u"][0] == pytest.approx(0.25, rel=1e-15)
    assert st["ubar"][0] == pytest.approx(0.25 * (1 + 1 / r3), rel=1e-15)
    b, a, th = next(sched)
    assert b == pytest.approx(r3, rel=1e-15) and a == pytest.approx(1 / r3, rel=1e-15)
    P.pdhg_step(p, pc, st, th, dual_mult=b, primal_mult=a)
    q2 = ((-1 - 3 * r3) / 4) / (1 + r3)
    u2 = (0.25 - q2 / r3) / (1 + 1 / r3)
    th1 = 1 / math.sqrt(1 + 2 / r3)
    assert st["q"][0] == pytest.approx(q2, rel=1e-14)
    assert st["u"][0] == pytest.approx(u2, rel=1e-14)
    assert st["ubar"][0] == pytest.approx(u2 + th1 * (u2 - 0.25), rel=1e-14)


def test_accel_schedule_invariants_and_freeze():
    """a_n b_n = 1 at every step, theta_n in (0, 1], b_n never above the
    bound, and after the freeze theta = 1 with constant steps."""
    sched = P.accel_schedule(0.7, 5.0)
    seen_freeze, prev = False, None
    for n in range(400):
        b, a, th = next(sched)
        assert a * b == pytest.approx(1.0, rel=1e-12)
        assert 0.0 < th <= 1.0 and b <= 5.0
        if prev is not None and th == 1.0 and prev[2] == 1.0:
            assert (b, a) == prev[:2]
            seen_freeze = True
        prev = (b, a, th)
    assert seen_freeze and prev[0] > 4.0
    # without a bound the primal multiplier decays as 1/(gamma n): from
    # 1/a_{n+1}^2 = 1/a_n^2 + 2 gamma / a_n, 1/a_n = gamma n + O(log n)
    sched = P.accel_schedule(0.7, math.inf)
    for n in range(200001):
        b, a, th = next(sched)
        if n in (20000, 200000):
            assert 0.7 * n * a == pytest.approx(1.0, rel=2e-3 if n == 20000 else 3e-4), (n, 0.7 * n * a)


def test_accel_rate_bound_on_lst():
    """LS-T (G = alpha/2 ||u||^2 is alpha min(tau)-strongly convex in the
    metric of T): Chambolle-Pock's Theorem 2 bound for Algorithm 2 (an
    invariant the plain iteration also satisfies here, since F1* is strongly
    convex as well; the two hand-worked steps pin the schedule's arithmetic),
    N^2 ||u^N - u*||_T^-1^2 <= (1 + eps) (||u0 - u*||_T^-1^2 + ||y0 - y*||_S^-1^2) / gamma^2,
    with u* the normal-equations solution and y* = A u* - f."""
    p = _tiny("lst", lam=0.05)
    pc = P.precond_diag(p)
    Ad = p.A.toarray()
    us = np.linalg.solve(Ad.T @ Ad + p.lam * np.eye(p.N), Ad.T @ p.f)
    ys = Ad @ us - p.f
    gamma = p.lam * pc["tau_u"].min()
    rhs = (np.sum(us ** 2 / pc["tau_u"]) + np.sum(ys ** 2 / pc["sigma_q"])) / gamma ** 2
    st = P.init_state(p)
    sched = P.accel_schedule(gamma, math.inf)
    n = 0
    for N in (50, 200, 800, 3200):
        while n < N:
            b, a, th = next(sched)
            P.pdhg_step(p, pc, st, th, dual_mult=b, primal_mult=a)
            n += 1
        lhs = N * N * np.sum((st["u"] - us) ** 2 / pc["tau_u"])
        assert lhs <= 1.25 * rhs, (N, lhs, rhs)


def test_accel_gamma_zero_is_plain():
    p = _tiny("tgv", lam=0.02)
    pc = P.precond_diag(p)
    a = P.pdhg_solve(p, pc, iters=40)
    b = P.pdhg_solve(p, pc, iters=40, accel_gamma=0.0, accel_step_max=7.0)
    assert all(np.array_equal(a[k], b[k]) for k in ("u", "ubar", "q", "r", "v", "s"))


@pytest.mark.parametrize("kind,tol", [("tv", 1e-9), ("tgv", 1e-7)])
def test_accel_same_minimiser(kind, tol):
    """With the schedule frozen at a bounded step ratio the accelerated
    iteration is plain PDHGM with rescaled steps: it reaches the same tiny
    gap, and its objective matches the independent smooth solver."""
    p = _tiny(kind, lam=0.01)
    pc = P.precond_diag(p)
    st = P.pdhg_solve(p, pc, tol=tol, max_iter=400000, gap_every=25, box=2.0,
                      accel_gamma=1.0, accel_step_max=4.0)
    h = st["history"][-1]
    assert h["rel_gap"] <= tol and h["gap"] >= -1e-14
    eps = 1e-7
    ref = _smoothed_minimum(p, eps)
    bias = eps * p.N * (p.lam + (p.alpha0 if kind == "tgv" else 0.0))
    assert ref - bias - 1e-12 <= h["P"] <= ref + h["gap"] + 1e-12, (h["P"], ref, bias, h["gap"])
