"""The dual-tree wavelet transform W of the wavelet model (Sec. 2.2, eq.
min_wav; Sec. 3.3.1 uses W and, for its adjoint, W^{-1} = W^T), as an explicit
sparse matrix in float64. Test infrastructure only (see the package
docstring).

The paper takes W from third-party code whose filters it does not print. Here
W is a dual-tree transform built from the construction of Kingsbury's
dual-tree complex wavelet transform (Sec. 2.2 cites it) with filters that
have a closed form:

* 1-D filters: the 4-tap orthonormal Daubechies lowpass h (two vanishing
  moments), h = (1+s, 3+s, 3-s, 1-s) / (4 sqrt 2), s = sqrt 3, and its
  quadrature mirror highpass g[k] = (-1)^k h[3-k].
* Two trees a and b. Level 1: tree b is tree a on the signal advanced by one
  sample. Levels 2, 3, ...: tree b uses the time-reversed filters of tree a
  (the structure of Kingsbury's quarter-shift filter pairs).
* Periodic boundaries; analysis y[i] = sum_k c[k] x[(2 i + k + shift) mod n].
* 2-D: four separable trees (y tree, x tree) in {a, b}^2, each a J-level
  orthonormal 2-D transform of the image (rows y with the y tree's filters,
  columns x with the x tree's) recursing on its own lowpass band.
* Per level and orientation (LH: lowpass in y, highpass in x; HL; HH) the
  four trees' bands are combined into oriented bands by the orthonormal
  sums and differences of the complex dual-tree transform:
  p = (aa - bb)/sqrt2, q = (aa + bb)/sqrt2, s = (ab + ba)/sqrt2,
  t = (ab - ba)/sqrt2; the four final lowpass bands are kept as they are.
* Everything is scaled by 1/2, so that W^T W = I (a Parseval frame with four
  times as many coefficients as pixels, ||W|| = 1 as the paper states).

Coefficient order (length 4 N): for level j = 1..J, for orientation LH, HL,
HH, for band p, q, s, t, the (ny / 2^j) x (nx / 2^j) band row-major; then
the four level-J lowpass bands of trees aa, ab, ba, bb.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

S3 = np.sqrt(3.0)
H_D4 = np.array([1.0 + S3, 3.0 + S3, 3.0 - S3, 1.0 - S3]) / (4.0 * np.sqrt(2.0))


def highpass(h: np.ndarray) -> np.ndarray:
    """Quadrature mirror filter g[k] = (-1)^k h[L-1-k]."""
    L = len(h)
    return np.array([(-1.0) ** k * h[L - 1 - k] for k in range(L)])


def tree_filters(tree: str, level: int):
    """(lowpass, highpass, shift) of one tree at one level (see the module doc)."""
    h = H_D4
    if tree == "a":
        return h, highpass(h), 0
    if level == 1:
        return h, highpass(h), 1
    hr = h[::-1].copy()
    return hr, highpass(hr), 0


def analysis_1d(n: int, c: np.ndarray, shift: int) -> sp.csr_matrix:
    """(n/2) x n periodic filter-and-downsample: y[i] = sum_k c[k] x[(2i+k+shift) mod n]."""
    rows, cols, vals = [], [], []
    for i in range(n // 2):
        for k, ck in enumerate(c):
            rows.append(i)
            cols.append((2 * i + k + shift) % n)
            vals.append(ck)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n // 2, n))  # duplicates add up


def tree_bands(nx: int, ny: int, levels: int, ty: str, tx: str):
    """One 2-D tree: {(j, 'LH'|'HL'|'HH'): matrix, ('LL', J): matrix} acting on
    the image (row-major, x fastest), each band (ny/2^j)(nx/2^j) x N."""
    out = {}
    cur = sp.identity(nx * ny, format="csr")
    cx, cy = nx, ny
    for j in range(1, levels + 1):
        hy, gy, sy = tree_filters(ty, j)
        hx, gx, sx = tree_filters(tx, j)
        Ly, Hy = analysis_1d(cy, hy, sy), analysis_1d(cy, gy, sy)
        Lx, Hx = analysis_1d(cx, hx, sx), analysis_1d(cx, gx, sx)
        out[(j, "LH")] = sp.kron(Ly, Hx, format="csr") @ cur
        out[(j, "HL")] = sp.kron(Hy, Lx, format="csr") @ cur
        out[(j, "HH")] = sp.kron(Hy, Hx, format="csr") @ cur
        cur = sp.kron(Ly, Lx, format="csr") @ cur
        cx, cy = cx // 2, cy // 2
    out[("LL", levels)] = cur
    return out


def check_shape(nx: int, ny: int, levels: int) -> None:
    if levels < 1 or nx % (2 ** levels) or ny % (2 ** levels):
        raise ValueError("the image sides must be multiples of 2^levels")


def dtwt_matrix(nx: int, ny: int, levels: int) -> sp.csr_matrix:
    """W (4 N x N) in the coefficient order of the module doc."""
    check_shape(nx, ny, levels)
    trees = {(ty, tx): tree_bands(nx, ny, levels, ty, tx) for ty in "ab" for tx in "ab"}
    r2 = 1.0 / np.sqrt(2.0)
    blocks = []
    for j in range(1, levels + 1):
        for o in ("LH", "HL", "HH"):
            aa, ab = trees[("a", "a")][(j, o)], trees[("a", "b")][(j, o)]
            ba, bb = trees[("b", "a")][(j, o)], trees[("b", "b")][(j, o)]
            blocks += [r2 * (aa - bb), r2 * (aa + bb), r2 * (ab + ba), r2 * (ab - ba)]
    for t in (("a", "a"), ("a", "b"), ("b", "a"), ("b", "b")):
        blocks.append(trees[t][("LL", levels)])
    return (0.5 * sp.vstack(blocks, format="csr")).tocsr()


def band_offsets(nx: int, ny: int, levels: int) -> dict:
    """Start of every band in the coefficient vector: {(j, o, band): offset},
    {('LL', tree): offset}, and the total (4 N)."""
    off, pos = {}, 0
    for j in range(1, levels + 1):
        size = (nx >> j) * (ny >> j)
        for o in ("LH", "HL", "HH"):
            for b in "pqst":
                off[(j, o, b)] = pos
                pos += size
    size = (nx >> levels) * (ny >> levels)
    for t in ("aa", "ab", "ba", "bb"):
        off[("LL", t)] = pos
        pos += size
    off["total"] = pos
    return off
