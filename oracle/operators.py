"""Regulariser operators as explicit sparse matrices, float64.

Test infrastructure only (see the package docstring).

Images are flattened row-major (j = iy * nx + ix). Sec. 3.3.1 uses matrix
versions of the gradient and of the symmetrised gradient; the discretisation
below is:

* grad = [dx+; dy+]: forward differences with unit spacing and a zero last
  difference (Neumann), so div = -grad^T (Sec. 3.3, Alg. 1 uses -div as the
  adjoint of grad).
* d- := -(d+)^T (backward differences with the matching boundary rows).
* E v = [dx- vx;  (dy- vx + dx- vy)/2;  (dy- vx + dx- vy)/2;  dy- vy], four rows
  per pixel so that its pointwise norm is the Frobenius norm of the symmetric
  2x2 matrix (Sec. 2.1, eq. min_TGV; the symmetrised gradient).
* Directional gradient D grad, D(p) = I - (1 - eta) xi xi^T with
  xi = (-sin theta, cos theta) the normal of the local structure direction
  theta; eta = 1 gives the plain gradient.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def diff_forward_1d(n: int) -> sp.csr_matrix:
    """n x n forward difference, row i: u[i+1] - u[i]; last row zero."""
    main = -np.ones(n)
    main[-1] = 0.0
    upper = np.ones(n - 1)
    return sp.diags([main, upper], [0, 1], shape=(n, n), format="csr")


def dx_plus(nx: int, ny: int) -> sp.csr_matrix:
    return sp.kron(sp.identity(ny), diff_forward_1d(nx), format="csr")


def dy_plus(nx: int, ny: int) -> sp.csr_matrix:
    return sp.kron(diff_forward_1d(ny), sp.identity(nx), format="csr")


def grad_matrix(nx: int, ny: int) -> sp.csr_matrix:
    """grad: R^N -> R^{2N}, rows [dx+ (all pixels); dy+ (all pixels)]."""
    return sp.vstack([dx_plus(nx, ny), dy_plus(nx, ny)], format="csr")


def sym_grad_matrix(nx: int, ny: int) -> sp.csr_matrix:
    """E: R^{2N} -> R^{4N} acting on v = [vx; vy]."""
    dxm = -dx_plus(nx, ny).T.tocsr()
    dym = -dy_plus(nx, ny).T.tocsr()
    Z = sp.csr_matrix(dxm.shape)
    row1 = sp.hstack([dxm, Z])
    row2 = sp.hstack([0.5 * dym, 0.5 * dxm])
    row4 = sp.hstack([Z, dym])
    return sp.vstack([row1, row2, row2, row4], format="csr")


def dtv_matrix(nx: int, ny: int, theta: np.ndarray, eta: float) -> sp.csr_matrix:
    """D grad: R^N -> R^{2N} with D(p) = I - (1 - eta) xi xi^T per pixel."""
    th = np.asarray(theta, dtype=np.float64).reshape(-1)
    xi_x, xi_y = -np.sin(th), np.cos(th)
    g = 1.0 - eta
    d11 = sp.diags(1.0 - g * xi_x * xi_x)
    d12 = sp.diags(-g * xi_x * xi_y)
    d22 = sp.diags(1.0 - g * xi_y * xi_y)
    Dx, Dy = dx_plus(nx, ny), dy_plus(nx, ny)
    return sp.vstack([d11 @ Dx + d12 @ Dy, d12 @ Dx + d22 @ Dy], format="csr")
