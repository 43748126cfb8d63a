"""Preconditioned conjugate gradients for the discrete Poisson problem
(Sec. 4.1), for checks at the level of single iterations.

Test infrastructure (see the package docstring); never used by the product.

The converged answer has a direct definition, the minimum-norm solution
L^+ eta, which `oracle.spectral.min_norm_solution` computes without iterating.
This module is the iteration itself: residual histories, the convergence
descriptors of Experiment 5.4, iteration counts of the preconditioners of
Sec. 4.3 and warm starts.  It is a textbook preconditioned CG for a symmetric
positive semidefinite operator -- iterate x, residual r, preconditioned
residual z, search direction p, operator image q -- with what the paper adds:
  * the start is x = 0 unless a warm start is given (the paper's experiments
    start from 0, Sec. 5.2; the method itself takes any start, Sec. 4.1);
  * the direction update uses the ratio of consecutive <r, z> (the paper's
    choice of beta);
  * for a singular set of boundary conditions the right-hand side is centred
    once (eq. 3.6), every preconditioned residual is centred (Remark 4.1)
    and the returned iterate is centred, giving the minimum-norm solution.

Stopping.  The paper runs a fixed number of iterations (Remark 4.2, Sec. 5.2).
The default here iterates until the true relative residual ||h - L x|| / ||h||
is at most `true_tol` (1e-14), or has not improved for `stall` iterations, or
`max_iter` iterations were made; `fixed_iterations` runs exactly that many.
"""

from dataclasses import dataclass, field

import numpy as np

from .diagnostics import iterate_descriptors
from .laplacian import apply_minus_laplacian, is_singular
from .pinv import PinvPreconditioner


@dataclass
class PCGResult:
    u: np.ndarray
    iterations: int
    true_rel_res: list = field(default_factory=list)     # entry s: iterate after s steps
    rec_rel_res: list = field(default_factory=list)      # updated residual ||r|| / ||h||
    removed_mean: float = 0.0
    h_norm: float = 0.0
    # per iterate: (true relative residual, kappa, null-space component, the
    # energy decrease step * <r, z> of the step that produced it), the
    # descriptors of Experiment 5.4 and Remark 4.2
    diagnostics: list = field(default_factory=list)


def pcg(eta, bcs, precond=None, u0=None, true_tol=1e-14, stall=2, max_iter=20,
        fixed_iterations=None):
    """Preconditioned CG for L u = eta.

    eta     right-hand side indexed [i, j] or [i, j, k] (Sec. 2.1 order)
    bcs     one boundary condition per axis (eq. 3.1)
    precond callable r -> z; None means no preconditioning
    u0      starting iterate (same shape), default zero
    """
    h = np.array(eta, dtype=np.float64)
    singular = is_singular(bcs)
    removed_mean = float(h.mean()) if singular else 0.0
    if singular:
        h = h - removed_mean

    def operator(v):
        return apply_minus_laplacian(v, bcs)

    def preconditioned(v):
        z = precond(v) if precond is not None else v.copy()
        return z - z.mean() if singular else z

    h_norm = float(np.linalg.norm(h))
    res = PCGResult(u=np.zeros_like(h), iterations=0, removed_mean=removed_mean,
                    h_norm=h_norm)
    if h_norm == 0.0:
        # every right-hand side of the null space has the solution 0
        res.true_rel_res.append(0.0)
        res.rec_rel_res.append(0.0)
        return res

    x = np.zeros_like(h) if u0 is None else np.array(u0, dtype=np.float64)

    def record(x, r, energy_step):
        true_rel, kappa, null = iterate_descriptors(x, h, bcs)
        res.true_rel_res.append(true_rel)
        res.rec_rel_res.append(float(np.linalg.norm(r)) / h_norm)
        res.diagnostics.append((true_rel, kappa, null, energy_step))

    # inner products use numpy's pairwise summation, whose rounding error
    # grows like log N: long runs past convergence then keep the residual at
    # rounding level instead of drifting upward
    r = h - operator(x)
    record(x, r, 0.0)
    steps = 0
    best, since_best = res.true_rel_res[0], 0
    done = fixed_iterations is None and best <= true_tol
    if not done and (fixed_iterations is None or fixed_iterations > 0):
        z = preconditioned(r)
        p = z.copy()
        rz = float(np.sum(r * z))
        while rz != 0.0:
            q = operator(p)
            step = rz / float(np.sum(p * q))
            x = x + step * p
            r = r - step * q
            steps += 1
            record(x, r, step * rz)
            if fixed_iterations is not None:
                if steps >= fixed_iterations:
                    break
            else:
                now = res.true_rel_res[-1]
                if now < best:
                    best, since_best = now, 0
                else:
                    since_best += 1
                if now <= true_tol or since_best >= stall or steps >= max_iter:
                    break
            z = preconditioned(r)
            rz_next = float(np.sum(r * z))
            p = z + (rz_next / rz) * p
            rz = rz_next

    res.u = x - x.mean() if singular else x
    res.iterations = steps
    return res


def solve(eta, bcs, **kw):
    """PCG with the pseudoinverse preconditioner (Sec. 4.3.3), iterated to the
    stopping rule above."""
    h = np.asarray(eta, dtype=np.float64)
    return pcg(h, bcs, precond=PinvPreconditioner(h.shape, bcs), **kw)
