"""Jacobi(p, omega) preconditioner: p steps of the (weighted) Jacobi method on
L x = R from x_0 = 0.

Test infrastructure (see the package docstring); never used by the product.

Sources in the paper (Sec. 4.3.1, "Preconditioning by several steps of
Jacobi-like method"):
  * the splitting A = D_omega(A) + O_omega(A) with D_omega(A) = omega D and
    O_omega(A) = O + (1 - omega) D, D the diagonal and O the off-diagonal
    part of A, omega >= 1; the stationary iteration
    x_j = D_omega(A)^{-1} (b - O_omega(A) x_{j-1})   (eq. 4.1), written with the
    Hadamard inverse of the diagonal (eq. 4.2);
  * for a Kronecker sum both parts split the same way (eq. 4.3), and the
    diagonal of the sum is the tensor of sums of the 1D diagonals times omega
    (eq. 4.4);
  * Algs. 2 (2D) and 3 (3D) apply eq. (4.1) to the residual p times from
    the zero start, with the off-diagonal part applied as one mode product
    per axis and the diagonal inverted entrywise.
Arrays are indexed in the paper's order U[i, j(, k)].
"""

import numpy as np

from .laplacian import laplacian_1d, _mode_product


def jacobi_init(shape, bcs, omega):
    """O_omega(L_l) per axis and the Hadamard inverse of the diagonal tensor."""
    if omega < 1.0:
        raise ValueError("the paper takes omega >= 1")
    O, diags = [], []
    for n, bc in zip(shape, bcs):
        L = laplacian_1d(n, bc)
        d = np.diag(L).copy()
        O.append(L - np.diag(d) + np.diag(d * (1.0 - omega)))   # O + (1 - omega) D
        diags.append(d)
    Dhat = np.zeros(shape)
    for a, d in enumerate(diags):
        sh = [1] * len(shape)
        sh[a] = len(d)
        Dhat = Dhat + d.reshape(sh)
    Dhat = Dhat * omega
    return O, 1.0 / Dhat


def jacobi_apply(R, O, Dinv, p):
    """Algs. 2 / 3: p sweeps of eq. (4.1) on L x = R from x = 0."""
    R = np.asarray(R, dtype=np.float64)
    x = np.zeros(R.shape)
    for _ in range(p):
        rhs = R.copy()
        for a, Oa in enumerate(O):
            rhs -= _mode_product(Oa, x, a)
        x = Dinv * rhs
    return x


class JacobiPreconditioner:
    """Callable R -> Z for the oracle's pcg."""

    def __init__(self, shape, bcs, p, omega):
        self.O, self.Dinv = jacobi_init(shape, bcs, omega)
        self.p = p

    def __call__(self, R):
        return jacobi_apply(R, self.O, self.Dinv, self.p)
