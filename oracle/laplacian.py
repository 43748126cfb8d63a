"""1D finite-difference minus Laplacians and their Kronecker sums.

Test infrastructure (see the package docstring); never used by the product.

Sources in the paper:
  * eq. (3.1), Sec. 3.1: the n x n matrix L_n(alpha, beta, gamma) with 2 on the
    diagonal, -1 next to it, corners alpha (top-left) and beta (bottom-right),
    and gamma in the two far corners; periodic (2,2,-1), Dirichlet (2,2,0),
    Neumann (1,1,0), mixed Dirichlet-Neumann (2,1,0) and Neumann-Dirichlet
    (1,2,0); n >= 3.
  * eq. (3.2), Sec. 3.3: the minus Laplacian of a matrix or a 3-way tensor is
    the sum of mode products L_n x_1 U + L_q x_2 U (+ L_t x_3 U); the entrywise
    form is written out in Sec. 4.2 ("Application of minus Laplacian").
  * eq. (3.3), Sec. 3.3: the vectorised operators
    L_2D = I_q (x) L_n + L_q (x) I_n and
    L_3D = I_t (x) I_q (x) L_n + I_t (x) L_q (x) I_n + L_t (x) I_q (x) I_n.
  * Sec. 3.3 (end): L_2D / L_3D are singular iff every 1D factor is singular;
    Lemmas 3.1-3.4: exactly the periodic and Neumann factors are singular.
"""

import numpy as np
import scipy.sparse as sp

# Boundary conditions of eq. (3.1) and their corner entries (alpha, beta, gamma).
_CORNERS = {
    "P": (2.0, 2.0, -1.0),
    "D": (2.0, 2.0, 0.0),
    "N": (1.0, 1.0, 0.0),
    "DN": (2.0, 1.0, 0.0),
    "ND": (1.0, 2.0, 0.0),
}
BCS = ("P", "D", "N", "DN", "ND")


def bc_corners(bc):
    """(alpha, beta, gamma) of eq. (3.1) for a boundary-condition name."""
    if bc not in _CORNERS:
        raise ValueError(f"unknown boundary condition {bc!r}")
    return _CORNERS[bc]


def laplacian_1d(n, bc):
    """Dense L_n(alpha, beta, gamma) of eq. (3.1)."""
    if n < 3:
        raise ValueError("eq. (3.1) needs n >= 3")
    alpha, beta, gamma = bc_corners(bc)
    L = np.zeros((n, n))
    for r in range(n):
        L[r, r] = 2.0
        if r > 0:
            L[r, r - 1] = -1.0
        if r < n - 1:
            L[r, r + 1] = -1.0
    L[0, 0] = alpha
    L[n - 1, n - 1] = beta
    L[0, n - 1] = gamma
    L[n - 1, 0] = gamma
    return L


def laplacian_1d_sparse(n, bc):
    """The same matrix as `laplacian_1d`, stored sparse (CSR)."""
    return sp.csr_matrix(laplacian_1d(n, bc))


def is_singular(bcs):
    """True iff the 2D/3D operator is singular: all factors periodic or Neumann."""
    return all(bc in ("P", "N") for bc in bcs)


def _mode_product(M, U, mode):
    """M x_mode U (Sec. 2.2): multiply every mode-`mode` fibre of U by M.

    `M` may be dense or scipy-sparse.  Implemented by moving the mode to the
    front, flattening the other modes, multiplying and moving it back.
    """
    Um = np.moveaxis(U, mode, 0)
    shape = Um.shape
    flat = Um.reshape(shape[0], -1)
    out = M @ flat
    out = np.asarray(out).reshape((M.shape[0],) + shape[1:])
    return np.moveaxis(out, 0, mode)


def apply_minus_laplacian(U, bcs, dense=False):
    """W = -Delta_FD(U) of eq. (3.2): sum over axes of L_axis x_axis U.

    U is indexed as in the paper, U[i, j] or U[i, j, k]; `bcs` holds one
    boundary condition per axis.  With dense=True the 1D operators are dense
    (the "Full" column of Table 1); otherwise they are sparse.  Both give the
    same numbers up to the order of the three-term row sums.
    """
    U = np.asarray(U, dtype=np.float64)
    if U.ndim != len(bcs):
        raise ValueError("one boundary condition per axis is required")
    W = np.zeros_like(U)
    for axis, bc in enumerate(bcs):
        n = U.shape[axis]
        L = laplacian_1d(n, bc) if dense else laplacian_1d_sparse(n, bc)
        W += _mode_product(L, U, axis)
    return W


def kronecker_sum(shape, bcs):
    """Assembled L_2D or L_3D of eq. (3.3), acting on vec(U) = U.ravel('F')."""
    if len(shape) != len(bcs):
        raise ValueError("one boundary condition per axis is required")
    mats = [laplacian_1d(n, bc) for n, bc in zip(shape, bcs)]
    eyes = [np.eye(n) for n in shape]
    total = None
    for axis in range(len(shape)):
        # Kronecker factors are written from the last axis to the first, so
        # that the first index of U varies fastest in vec(U) (Sec. 2.1).
        term = np.ones((1, 1))
        for other in reversed(range(len(shape))):
            term = np.kron(term, mats[other] if other == axis else eyes[other])
        total = term if total is None else total + term
    return total
