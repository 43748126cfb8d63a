"""Convergence descriptors of a PCG iterate (Experiment 5.4, Remark 4.2).

Test infrastructure (see the package docstring); never used by the product.

Sources in the paper:
  * Experiment 5.4 watches four quantities along the iterations:
      - the true residual ||H - L u_s||_2 and the computed (recursive) one
        ||r_s||_2 (the two agree until convergence, then the true residual
        stagnates while the recursive one keeps falling);
      - a quantity that behaves like the L-norm of the error: since L u = H,
          ||u_s - u||_L^2 = kappa_s + ||u||_L^2,
          kappa_s = u_s^T L u_s - 2 u_s^T H,
        where kappa_s is computable and ||u||_L^2 an unknown constant; the
        paper plots eta_s = sqrt(kappa_s - min_j kappa_j), scaled by
        ||H - L u_1|| / eta_1 and shifted by the machine epsilon 2^-52;
      - for a singular operator, the norm of the null-space component of the
        solution.
  * Remark 4.2 names a robust estimate of the A-norm of the error as the best
    stopping rule and points to the literature.  The estimate used here is
    the classical one of Hestenes and Stiefel (1952), studied in finite
    precision by Strakos and Tichy (2002): in PCG,
        ||e_{s}||_A^2 - ||e_{s+1}||_A^2 = alpha_{s+1} rho_s,
    so the sum of the next d terms is a lower bound on ||e_s||_A^2 that
    becomes tight as the error drops ("delay" d).  Here A = L.
Arrays are indexed in the paper's order U[i, j(, k)]; for a singular
operator H is the centred right-hand side of eq. (3.6).
"""

import numpy as np

from .laplacian import apply_minus_laplacian, is_singular


def iterate_descriptors(U, H, bcs):
    """(true relative residual, kappa_s, null-space component) of the
    iterate U for L U = H.  The null space of a singular L is spanned by the
    constant tensor, whose normalised form is 1/sqrt(N); its component is
    |sum U| / sqrt(N).  Nonsingular operators have none: 0."""
    U = np.asarray(U, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    LU = apply_minus_laplacian(U, bcs)
    h = float(np.linalg.norm(H))
    true_rel = float(np.linalg.norm(H - LU)) / h if h > 0.0 else 0.0
    kappa = float(np.sum(U * LU)) - 2.0 * float(np.sum(U * H))
    null = abs(float(U.sum())) / np.sqrt(U.size) if is_singular(bcs) else 0.0
    return true_rel, kappa, null


def error_norm_proxy(kappa):
    """Experiment 5.4's eta_s = sqrt(kappa_s - min_j kappa_j) over a run."""
    k = np.asarray(kappa, dtype=np.float64)
    return np.sqrt(np.maximum(k - k.min(), 0.0))


def plotted_proxy(kappa, true_res_1):
    """The curve Experiment 5.4 draws: alpha eta_s + beta with
    alpha = ||H - L u_1|| / eta_1 and beta = 2^-52."""
    eta = error_norm_proxy(kappa)
    return true_res_1 / eta[1] * eta + 2.0 ** -52


def hs_error_estimate(terms, delay):
    """Hestenes-Stiefel estimate of ||e_s||_L for every s: the square root of
    terms[s+1] + ... + terms[s+delay], where terms[j] = alpha_j rho_{j-1}
    (terms[0] unused); near the end of a run only the available terms are
    summed."""
    t = np.asarray(terms, dtype=np.float64)
    out = np.zeros(len(t))
    for s in range(len(t)):
        out[s] = np.sqrt(max(float(np.sum(t[s + 1:s + 1 + delay])), 0.0))
    return out


def hs_stop_iteration(terms, tol, delay=4):
    """The first iteration s >= delay at which the Hestenes-Stiefel estimate
    of the relative L-norm error of U_{s-delay},
        sqrt((terms[s-delay+1] + ... + terms[s]) / (terms[1] + ... + terms[s])),
    is <= tol (its denominator estimates ||u||_L^2, since U_0 = 0); None if
    no recorded iteration qualifies."""
    t = np.asarray(terms, dtype=np.float64)
    for s in range(delay, len(t)):
        total = float(np.sum(t[1:s + 1]))
        if total > 0.0 and np.sqrt(float(np.sum(t[s - delay + 1:s + 1])) / total) <= tol:
            return s
    return None


def lowmode_error_bound(R, U, bcs, m=32):
    """Relative error bound of an iterate U with residual R (the
    certificate the solver uses before its error estimate):
        ||L^+ R||^2 <= sum_box rhat^2 / lambda^2 + (||R||^2 - sum_box rhat^2) / theta^2
    divided by ||U||, where rhat are the coefficients of R on the box of the
    min(n_a, m) eigenmodes of smallest eigenvalue per axis (eigenvectors from
    LAPACK), lambda their eigenvalue sums (null modes skipped) and theta the
    smallest eigenvalue sum outside the box (exact when the box is
    everything).  L^+ R is the error of U when R = H - L U (eqs. 3.3, 4.6)."""
    from .laplacian import laplacian_1d
    R = np.asarray(R, dtype=np.float64)
    lams, Vs, ms = [], [], []
    for n, bc in zip(R.shape, bcs):
        lam, V = np.linalg.eigh(laplacian_1d(n, bc))
        lams.append(lam)
        Vs.append(V)
        ms.append(min(n, m))
    rhat = R
    for a in range(R.ndim):
        rhat = np.moveaxis(np.tensordot(rhat, Vs[a][:, :ms[a]], axes=([a], [0])), -1, a)
    lb = np.zeros(rhat.shape)
    for a in range(R.ndim):
        sh = [1] * R.ndim
        sh[a] = ms[a]
        lb = lb + lams[a][:ms[a]].reshape(sh)
    pos = np.abs(lb) > 1e-13
    low = float(np.sum(np.where(pos, rhat ** 2 / np.where(pos, lb, 1.0) ** 2, 0.0)))
    box = float(np.sum(rhat ** 2))
    theta = np.inf
    for a in range(R.ndim):
        if ms[a] < R.shape[a]:
            theta = min(theta, lams[a][ms[a]] + sum(lams[b][0] for b in range(R.ndim) if b != a))
    rest = max(float(np.sum(R * R)) - box, 0.0)
    tail = rest / theta ** 2 if np.isfinite(theta) else 0.0
    return np.sqrt(low + tail) / float(np.linalg.norm(U))
