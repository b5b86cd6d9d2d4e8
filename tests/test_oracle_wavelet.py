"""Pins of the oracle's dual-tree transform W and of the wavelet model
(Sec. 2.2 eq. min_wav; Algorithm 1 with grad -> W, div -> W^{-1}) against
facts that do not come from the oracle itself: the closed-form Daubechies
filter's defining identities, orthogonality of every level and tree, the
Parseval identity W^T W = I and ||W|| = 1 that the paper states, the response
to constant and linear images (two vanishing moments), the norm bound of the
preconditioned operator, and the optimality conditions at the solver's limit.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import pdhg as OP
from oracle import wavelet as OW


def test_daubechies_filter_identities():
    h = OW.H_D4
    g = OW.highpass(h)
    assert h.sum() == pytest.approx(np.sqrt(2.0), abs=1e-15)
    assert float(h @ h) == pytest.approx(1.0, abs=1e-15)
    assert h[0] * h[2] + h[1] * h[3] == pytest.approx(0.0, abs=1e-15)  # orthogonal to its shift by 2
    k = np.arange(4)
    assert g.sum() == pytest.approx(0.0, abs=1e-15)         # vanishing moment 0
    assert float(k @ g) == pytest.approx(0.0, abs=1e-15)    # vanishing moment 1
    assert float((k * k) @ g) != pytest.approx(0.0, abs=1e-3)  # but not 2: D4 has exactly two
    # the closed form: (1 + sqrt3) / (4 sqrt2) etc.
    assert h[0] == pytest.approx((1 + np.sqrt(3)) / (4 * np.sqrt(2)), abs=1e-16)


@pytest.mark.parametrize("n", [2, 4, 8, 16])
@pytest.mark.parametrize("tree,level", [("a", 1), ("b", 1), ("a", 2), ("b", 2)])
def test_each_analysis_pair_is_orthogonal(n, tree, level):
    h, g, shift = OW.tree_filters(tree, level)
    M = sp.vstack([OW.analysis_1d(n, h, shift), OW.analysis_1d(n, g, shift)]).toarray()
    assert np.allclose(M @ M.T, np.eye(n), atol=1e-14)


@pytest.mark.parametrize("nx,ny,J", [(16, 16, 2), (32, 16, 3), (8, 8, 3), (24, 8, 3)])
def test_parseval_and_norm(nx, ny, J):
    W = OW.dtwt_matrix(nx, ny, J)
    N = nx * ny
    assert W.shape == (4 * N, N)
    assert OW.band_offsets(nx, ny, J)["total"] == 4 * N
    G = (W.T @ W).toarray()
    assert np.abs(G - np.eye(N)).max() <= 1e-13
    assert np.linalg.norm(W.toarray(), 2) == pytest.approx(1.0, abs=1e-12)


def test_constant_and_linear_images():
    nx, ny, J = 32, 16, 3
    W = OW.dtwt_matrix(nx, ny, J)
    off = OW.band_offsets(nx, ny, J)
    c = W @ np.full(nx * ny, 3.0)
    first_ll = off[("LL", "aa")]
    assert np.abs(c[:first_ll]).max() <= 1e-13           # no detail
    # each tree's lowpass multiplies a constant by (sum h)^2 = 2 per level; scale 1/2
    assert np.allclose(c[first_ll:], 3.0 * 2 ** J / 2, atol=1e-12)
    # a plane has no level-1 detail away from the periodic seam (two vanishing moments)
    y, x = np.mgrid[0:ny, 0:nx]
    c = W @ (0.7 * x + 0.3 * y + 1.0).ravel()
    for o in ("LH", "HL", "HH"):
        for b in "pqst":
            band = c[off[(1, o, b)]:off[(1, o, b)] + (nx // 2) * (ny // 2)].reshape(ny // 2, nx // 2)
            # taps of coefficient i reach samples 2i .. 2i+4: inside for i <= n/2 - 3
            assert np.abs(band[: ny // 2 - 2, : nx // 2 - 2]).max() <= 1e-12, (o, b)


def test_mismatched_sizes_are_refused():
    with pytest.raises(ValueError):
        OW.dtwt_matrix(12, 8, 3)


def _small_problem(kind="wav", seed=0, levels=2):
    rng = np.random.default_rng(seed)
    nx = ny = 8
    N = nx * ny
    A = sp.random(40, N, density=0.3, random_state=seed, format="csr")
    A.data = np.abs(A.data)
    u_true = np.zeros((ny, nx))
    u_true[2:6, 3] = 1.0  # a thin vertical structure
    f = A @ u_true.ravel() + 0.01 * rng.standard_normal(40)
    return OP.Problem(A, f, nx, ny, kind, 0.05, levels=levels)


def test_preconditioned_wavelet_operator_norm():
    """||Sigma^(1/2) K T^(1/2)|| <= 1 for K = [A; W] with the wav steps."""
    p = _small_problem()
    pc = OP.precond_diag(p)
    K = p.stacked()
    sig = np.concatenate([pc["sigma_q"], pc["sigma_r"]])
    M = sp.diags(np.sqrt(sig)) @ K @ sp.diags(np.sqrt(pc["tau_u"]))
    assert np.linalg.norm(M.toarray(), 2) <= 1.0 + 1e-12
    # doubling tau breaks it: the bound is not loose by a factor of two
    M2 = sp.diags(np.sqrt(sig)) @ K @ sp.diags(np.sqrt(2.0 * pc["tau_u"]))
    assert np.linalg.norm(M2.toarray(), 2) > 1.0


def test_wavelet_model_reaches_its_optimality_conditions():
    """At the limit: A^T(Au - f) + W^T r = 0 with |r| <= lam and r = lam sign(Wu)
    on the coefficients of W u that are clearly non-zero; the gap goes to 0."""
    p = _small_problem()
    pc = OP.precond_diag(p)
    st = OP.pdhg_solve(p, pc, iters=20000)
    u, r = st["u"], st["r"].reshape(-1)
    grad = p.A.T @ (p.A @ u - p.f) + p.B.T @ r
    assert np.abs(grad).max() <= 1e-8
    assert np.abs(r).max() <= p.lam * (1 + 1e-12)
    c = p.B @ u
    big = np.abs(c) > 1e-6
    assert big.sum() > 10
    assert np.allclose(r[big], p.lam * np.sign(c[big]), atol=1e-8)
    g = OP.gap_terms(p, st, 2.0)
    assert g["rel_gap"] <= 1e-9
    # the primal objective is the model's: data term plus lam ||W u||_1
    res = p.A @ u - p.f
    assert g["P"] == pytest.approx(0.5 * res @ res + p.lam * np.abs(c).sum(), rel=1e-14)
