"""Low-Kronecker-rank approximation of the pseudoinverse (2D only).

Test infrastructure (see the package docstring); never used by the product.

Sources in the paper (Sec. 4.3.2):
  * the pseudoinverse of the 2D Kronecker sum is (V_q (x) V_n) diag(g_ij)
    (V_q (x) V_n)^T with the Hadamard pseudoinverse Ghat of the eigenvalue
    sums (eq. 4.7, entries below 1e-13 in modulus taken as zero);
  * the best rank-r approximation of Ghat (Eckart-Young-Mirsky) from its SVD
    Ghat = sum_rho x_rho sigma_rho y_rho^T, each dyad reshaped into a
    Kronecker product of diagonal matrices and transformed back, gives
    sum_rho M_{q,rho} (x) M_{n,rho};
  * application: Z = sum_rho M_{n,rho} R M_{q,rho}^T.
Reading: the paper attaches diag(x_rho sigma_rho) to V_q and diag(y_rho) to
V_n, which only type-checks when n = q.  Since x_rho has n entries (rows of
Ghat are indexed by the eigenvalues of L_n) and vec(x y^T) = y (x) x, the
consistent assignment is M_{n,rho} = V_n diag(sigma_rho x_rho) V_n^T and
M_{q,rho} = V_q diag(y_rho) V_q^T.  The eigenvectors come from LAPACK, as the
paper's `eig`; the SVD from LAPACK too.
Arrays are indexed in the paper's order R[i, j], i over n.
"""

import numpy as np

from .laplacian import laplacian_1d

_THRESHOLD = 1e-13


def lowrank_init(shape, bcs, rank):
    """The pairs (M_{n,rho}, M_{q,rho}), rho = 1..rank."""
    if len(shape) != 2:
        raise ValueError("the low-Kronecker-rank preconditioner is 2D only")
    n, q = shape
    ln, Vn = np.linalg.eigh(laplacian_1d(n, bcs[0]))
    lq, Vq = np.linalg.eigh(laplacian_1d(q, bcs[1]))
    S = ln[:, None] + lq[None, :]
    small = np.abs(S) < _THRESHOLD
    G = np.where(small, 0.0, 1.0 / np.where(small, 1.0, S))   # eq. 4.7
    X, sig, Yt = np.linalg.svd(G)
    pairs = []
    for r in range(rank):
        Mn = Vn @ np.diag(sig[r] * X[:, r]) @ Vn.T
        Mq = Vq @ np.diag(Yt[r, :]) @ Vq.T
        pairs.append((Mn, Mq))
    return pairs


def lowrank_apply(R, pairs):
    """Z = sum_rho M_{n,rho} R M_{q,rho}^T."""
    R = np.asarray(R, dtype=np.float64)
    Z = np.zeros_like(R)
    for Mn, Mq in pairs:
        Z += Mn @ R @ Mq.T
    return Z


class LowRankPreconditioner:
    """Callable R -> Z for the oracle's pcg."""

    def __init__(self, shape, bcs, rank):
        self.pairs = lowrank_init(shape, bcs, rank)

    def __call__(self, R):
        return lowrank_apply(R, self.pairs)
