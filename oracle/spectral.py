"""The minimum-norm solution of the discrete Poisson problem, written out from
the eigen-expansion of the operator.

Test infrastructure (see the package docstring); never used by the product.

Sources in the paper:
  * eq. (3.3), Sec. 3.3: the operator is the Kronecker sum of the 1D matrices
    of eq. (3.1), one per axis;
  * Sec. 3.2 (Lemmas 3.1-3.4) and eq. (4.5): each 1D matrix is symmetric, so
    it has an orthonormal eigenbasis; a product of one eigenvector per axis is
    then an eigenvector of the Kronecker sum, with the sum of the three (two)
    1D eigenvalues as its eigenvalue, and these products form an orthonormal
    basis of the whole grid space;
  * Sec. 3.4.1 and eqs. (4.6)-(4.7): the eigenvalue sums that vanish (the
    null space of a periodic / Neumann set) are dropped, with the paper's
    absolute threshold 1e-13.

Hence the Moore-Penrose solution is the plain expansion
    u = sum over modes m with mu_m != 0 of  <v_m, h> / mu_m * v_m,
which for a singular set is also the zero-mean solution of the centred
problem (eq. 3.6): the constant mode, the only one dropped, is exactly the
mean.  This is the converged answer that the preconditioned CG approaches;
it is computed here without any iteration, with LAPACK eigenvectors of the
assembled 1D matrices.
"""

import numpy as np

from .laplacian import is_singular, laplacian_1d

# |mu| below this counts as a zero eigenvalue (eq. 4.7 and Algs. 4-5).
NULL_THRESHOLD = 1e-13


def axis_eigenpairs(n, bc):
    """(eigenvalues ascending, orthonormal eigenvectors as columns) of the 1D
    matrix of eq. (3.1), from LAPACK."""
    return np.linalg.eigh(laplacian_1d(n, bc))


def _to_modes(H, bases):
    """Coefficients <v_a (x) v_b (x) v_c, H>: contract every axis with its
    eigenvectors."""
    C = np.asarray(H, dtype=np.float64)
    for axis, (_, V) in enumerate(bases):
        C = np.moveaxis(np.tensordot(V, C, axes=([0], [axis])), 0, axis)
    return C


def _from_modes(C, bases):
    """The grid function with mode coefficients C."""
    U = C
    for axis, (_, V) in enumerate(bases):
        U = np.moveaxis(np.tensordot(V, U, axes=([1], [axis])), 0, axis)
    return U


def eigenvalue_sums(shape, bases):
    """mu[a, b(, c)] = lambda_a + lambda_b (+ lambda_c) over the axes."""
    mu = np.zeros(tuple(shape))
    for axis, (w, _) in enumerate(bases):
        bshape = [1] * len(shape)
        bshape[axis] = shape[axis]
        mu = mu + w.reshape(bshape)
    return mu


def min_norm_solution(eta, bcs):
    """L^+ eta for the Kronecker-sum operator with boundary conditions `bcs`.

    eta is indexed in the paper's order, eta[i, j] or eta[i, j, k].  Returns
    (u, removed_mean): u = L^+ eta (zero-mean for a singular set) and the
    mean of eta that the projection of eq. (3.6) removes (0 for a
    nonsingular set)."""
    H = np.asarray(eta, dtype=np.float64)
    if H.ndim != len(bcs):
        raise ValueError("one boundary condition per axis is required")
    bases = [axis_eigenpairs(n, bc) for n, bc in zip(H.shape, bcs)]
    C = _to_modes(H, bases)
    mu = eigenvalue_sums(H.shape, bases)
    live = np.abs(mu) >= NULL_THRESHOLD
    C = np.where(live, C / np.where(live, mu, 1.0), 0.0)
    u = _from_modes(C, bases)
    removed = float(H.mean()) if is_singular(bcs) else 0.0
    return u, removed
