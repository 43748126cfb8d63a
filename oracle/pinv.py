"""Moore-Penrose pseudoinverse preconditioner, Sec. 4.3.3.

Test infrastructure (see the package docstring); never used by the product.

Initialisation (Algs. 4 and 5): eigendecompose every 1D operator L_l =
V_l Lambda_l V_l^T with orthonormal V_l (eq. 4.5; the paper uses MATLAB `eig`,
here LAPACK through numpy.linalg.eigh), then form the Hadamard pseudoinverse
G of the tensor of eigenvalue sums (eqs. 4.6-4.7): g = 1/(lambda_i + lambda_j
[+ lambda_k]), with sums of modulus below 1e-13 replaced by 0 (the threshold
stated with eq. 4.7 and in Algs. 4-5).

Application (Algs. 6 and 7): the residual's coefficients in the product
eigenbasis (each axis contracted with the transpose of its eigenvector
matrix), scaled entrywise by G, and taken back to the grid with the
eigenvector matrices themselves.
"""

import numpy as np

from .laplacian import laplacian_1d, _mode_product

# Threshold below which an eigenvalue sum counts as zero (eq. 4.7, Algs. 4-5).
ZERO_THRESHOLD = 1e-13


def pinv_init(shape, bcs):
    """Algorithms 4 (2D) and 5 (3D).

    Returns (V, lam, G): lists of orthonormal eigenvector matrices and
    eigenvalue vectors per axis, and the Hadamard pseudoinverse G of the sums.
    """
    if len(shape) != len(bcs):
        raise ValueError("one boundary condition per axis is required")
    V, lam = [], []
    for n, bc in zip(shape, bcs):
        w, Q = np.linalg.eigh(laplacian_1d(n, bc))
        V.append(Q)
        lam.append(w)
    # Tensor of all sums lambda_i(L_n) + lambda_j(L_q) [+ lambda_k(L_t)].
    sums = np.zeros(tuple(shape))
    for axis, w in enumerate(lam):
        bshape = [1] * len(shape)
        bshape[axis] = shape[axis]
        sums = sums + w.reshape(bshape)
    G = np.zeros_like(sums)
    nonzero = np.abs(sums) >= ZERO_THRESHOLD
    G[nonzero] = 1.0 / sums[nonzero]
    return V, lam, G


def pinv_apply(R, V, G):
    """Algorithms 6 (2D) and 7 (3D): Z = M(R) for the pseudoinverse."""
    coeff = np.asarray(R, dtype=np.float64)
    for axis, Q in enumerate(V):          # into the eigenbasis, axis by axis
        coeff = _mode_product(Q.T, coeff, axis)
    coeff = coeff * G                     # Hadamard pseudoinverse of the sums
    Z = coeff
    for axis, Q in enumerate(V):          # back to the grid
        Z = _mode_product(Q, Z, axis)
    return Z


class PinvPreconditioner:
    """Init once, apply per iteration (the two subroutines of Sec. 4.3)."""

    def __init__(self, shape, bcs):
        self.shape = tuple(shape)
        self.bcs = tuple(bcs)
        self.V, self.lam, self.G = pinv_init(self.shape, self.bcs)

    def __call__(self, R):
        return pinv_apply(R, self.V, self.G)
