"""Preconditioned conjugate gradients, Algorithm 1 (Sec. 4.1).

Test infrastructure (see the package docstring); never used by the product.

The loop follows Algorithm 1 in the paper's order and notation:
  W_0 = -Delta(U_0), R_0 = H - W_0, Z_0 = M(R_0), rho_0 = <R_0, Z_0>, P_0 = Z_0;
  repeat: W_s = -Delta(P_{s-1}); alpha_s = rho_{s-1} / <W_s, P_{s-1}>;
          U_s = U_{s-1} + alpha_s P_{s-1}; R_s = R_{s-1} - alpha_s W_s;
          Z_s = M(R_s); rho_s = <R_s, Z_s>; beta_s = rho_s / rho_{s-1};
          P_s = Z_s + beta_s P_{s-1}.
The 2D variant is the same with matrices in place of tensors (Sec. 4.1).

Singular boundary-condition sets (all axes periodic or Neumann):
  * the right-hand side is centred once, eq. (3.6) (Sec. 3.4.1);
  * Z_s is centred after every preconditioner application (Remark 4.1).

Stopping.  The paper stops after a fixed number of iterations chosen so that
the true residual is small enough (Remark 4.2, Sec. 5.2).  The oracle's job is
the converged answer, so it iterates until the true relative residual
||H - L U_s|| / ||H|| drops to `true_tol` (default 1e-14), or has not
decreased for `stall` consecutive iterations, or `max_iter` is reached.  The
answer it converges to is the minimum-norm solution L^+ H of eq. (3.3).
"""

from dataclasses import dataclass, field

import numpy as np

from .diagnostics import iterate_descriptors
from .laplacian import apply_minus_laplacian, is_singular
from .pinv import PinvPreconditioner


def _center(X):
    """Eq. (3.6): subtract the mean over all entries."""
    return X - X.mean()


def _inner(X, Y):
    """<X, Y> = <vec X, vec Y> (Sec. 4.2, inner product)."""
    return float(np.sum(X * Y))


@dataclass
class PCGResult:
    u: np.ndarray
    iterations: int
    true_rel_res: list = field(default_factory=list)     # index s = iterate U_s
    rec_rel_res: list = field(default_factory=list)      # ||R_s|| / ||H||
    removed_mean: float = 0.0
    h_norm: float = 0.0
    # per iterate U_s: (true relative residual, kappa_s, null-space
    # component, alpha_s rho_{s-1}) of Experiment 5.4 / Remark 4.2
    diagnostics: list = field(default_factory=list)


def pcg(eta, bcs, precond=None, true_tol=1e-14, stall=2, max_iter=20,
        fixed_iterations=None):
    """Run Algorithm 1 from U_0 = 0 (the paper's choice, Sec. 5.2).

    eta     right-hand side H indexed [i, j] or [i, j, k]
    bcs     one boundary condition per axis
    precond callable R -> Z; None means M = I (unpreconditioned CG)
    fixed_iterations  if given, run exactly that many iterations (Remark 4.2)
    """
    H = np.array(eta, dtype=np.float64)
    singular = is_singular(bcs)
    removed_mean = 0.0
    if singular:
        removed_mean = float(H.mean())
        H = _center(H)
    M = precond if precond is not None else (lambda R: R.copy())

    def apply_M(R):
        Z = M(R)
        return _center(Z) if singular else Z

    h_norm = float(np.linalg.norm(H))
    U = np.zeros_like(H)
    res = PCGResult(u=U, iterations=0, removed_mean=removed_mean, h_norm=h_norm)
    if h_norm == 0.0:
        res.true_rel_res.append(0.0)
        res.rec_rel_res.append(0.0)
        return res

    W = apply_minus_laplacian(U, bcs)        # W_0 = -Delta(U_0)
    R = H - W                                # R_0
    Z = apply_M(R)                           # Z_0
    rho = _inner(R, Z)                       # rho_0
    P = Z.copy()                             # P_0
    res.true_rel_res.append(float(np.linalg.norm(H - apply_minus_laplacian(U, bcs))) / h_norm)
    res.rec_rel_res.append(float(np.linalg.norm(R)) / h_norm)
    res.diagnostics.append(iterate_descriptors(U, H, bcs) + (0.0,))

    best = res.true_rel_res[0]
    no_progress = 0
    s = 0
    while True:
        if rho == 0.0:
            break
        s += 1
        W = apply_minus_laplacian(P, bcs)    # W_s = -Delta(P_{s-1})
        alpha = rho / _inner(W, P)           # alpha_s
        hs_term = alpha * rho                # alpha_s rho_{s-1}
        U = U + alpha * P                    # U_s
        R = R - alpha * W                    # R_s
        Z = apply_M(R)                       # Z_s
        rho_new = _inner(R, Z)               # rho_s
        beta = rho_new / rho                 # beta_s
        P = Z + beta * P                     # P_s
        rho = rho_new

        true_rel = float(np.linalg.norm(H - apply_minus_laplacian(U, bcs))) / h_norm
        res.true_rel_res.append(true_rel)
        res.rec_rel_res.append(float(np.linalg.norm(R)) / h_norm)
        res.diagnostics.append(iterate_descriptors(U, H, bcs) + (hs_term,))

        if fixed_iterations is not None:
            if s >= fixed_iterations:
                break
            continue
        if true_rel < best:
            best = true_rel
            no_progress = 0
        else:
            no_progress += 1
        if true_rel <= true_tol or no_progress >= stall or s >= max_iter:
            break

    if singular:
        U = _center(U)
    res.u = U
    res.iterations = s
    return res


def solve(eta, bcs, **kw):
    """Converged minimum-norm solution with the pseudoinverse preconditioner."""
    H = np.asarray(eta, dtype=np.float64)
    M = PinvPreconditioner(H.shape, bcs)
    return pcg(H, bcs, precond=M, **kw)
