"""Brute-force Moore-Penrose solution of the assembled system, for tiny grids.

Test infrastructure (see the package docstring); never used by the product.

The vectorised system of eq. (3.3), L vec(U) = vec(H), is solved by
numpy.linalg.pinv (an SVD), which gives the minimum-norm solution L^+ vec(H).
For a singular operator its null space is spanned by the vector of ones
(Sec. 3.4.1), so L^+ H = L^+ H_c with H_c the centred right-hand side.
"""

import numpy as np

from .laplacian import kronecker_sum


def dense_pinv_solve(eta, bcs):
    H = np.asarray(eta, dtype=np.float64)
    if H.size > 4096:
        raise ValueError("brute force is meant for tiny grids only")
    L = kronecker_sum(H.shape, bcs)
    u = np.linalg.pinv(L, rcond=1e-12, hermitian=True) @ H.ravel(order="F")
    return u.reshape(H.shape, order="F")
