"""Plain FP64 CPU oracle for the pseudoinverse-preconditioned CG solver of the
finite-difference Poisson equation  -Laplace(u) = eta  on a rectangle or cuboid.

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it.
The GPU library never calls it, and it shares no code with the GPU library.

Everything here is written from the paper (Chumchal, Marton, Plesinger,
Simunkova, "Tensor-structured PCG for finite difference solver of domain
patterns in ferroelectric material", arXiv 2501.03377) in its own notation:

  * arrays are indexed as in the paper, U[i, j, k] with i the first (x) index,
    so that vec(U) (Sec. 2.1, inverse lexicographic order) is U.ravel('F');
  * a 2D problem is an array U[i, j] and a 3D problem an array U[i, j, k];
  * boundary conditions are the strings 'P', 'D', 'N', 'DN', 'ND' of eq. (3.1).

Modules
  laplacian  1D operators of eq. (3.1), the minus Laplacian of eq. (3.2),
             the Kronecker-sum matrices of eq. (3.3) for brute force.
  pinv       pseudoinverse preconditioner: initialisation (Algs. 4 and 5) and
             application (Algs. 6 and 7); eigenvectors come from LAPACK, as the
             paper's `eig`.
  spectral   the minimum-norm solution L^+ eta written out from the
             eigen-expansion of the Kronecker sum (eq. 3.3): the converged
             answer, computed without iterating.
  pcg        preconditioned CG (Sec. 4.1) with the null-space centering of
             eq. (3.6) and Remark 4.1, optional warm start, iterated to
             stagnation of the true residual: the iteration-level checks.
  dense      Moore-Penrose solution of the assembled Kronecker-sum system.
  bcdata     right-hand side update for non-homogeneous Dirichlet / Neumann
             data (Sec. 3.4.2) and the field eps = -grad u (Sec. 1).
  jacobi     Jacobi(p, omega) preconditioner (Sec. 4.3.1, Algs. 2-3).
  lowrank    low-Kronecker-rank approximation of the pseudoinverse (Sec.
             4.3.2, 2D only).
  diagnostics  convergence descriptors of Experiment 5.4 (true residual,
             kappa_s, null-space component) and the Hestenes-Stiefel error
             estimate that Remark 4.2 points to.

Parity status: every function here is pinned by tests/test_oracle_*.py against
closed forms, brute force on tiny grids, invariants or numbers the paper
prints; none is "parity unpinned".
"""

from .laplacian import (BCS, bc_corners, laplacian_1d, laplacian_1d_sparse,
                        apply_minus_laplacian, kronecker_sum, is_singular)
from .pinv import pinv_init, pinv_apply, PinvPreconditioner
from .pcg import pcg, solve, PCGResult
from .spectral import min_norm_solution
from .dense import dense_pinv_solve
from .bcdata import assemble_rhs, field
from .diagnostics import iterate_descriptors, error_norm_proxy, hs_error_estimate

__all__ = [
    "BCS", "bc_corners", "laplacian_1d", "laplacian_1d_sparse",
    "apply_minus_laplacian", "kronecker_sum", "is_singular",
    "pinv_init", "pinv_apply", "PinvPreconditioner",
    "pcg", "solve", "PCGResult", "min_norm_solution", "dense_pinv_solve", "assemble_rhs", "field",
    "iterate_descriptors", "error_norm_proxy", "hs_error_estimate",
]
