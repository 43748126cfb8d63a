"""Pins of the oracle's convergence descriptors (Experiment 5.4, Remark 4.2):
the L-norm of the error against a dense solve, closed forms on eigenmodes,
the Hestenes-Stiefel identity, monotonicity, the null-space component
against an SVD null vector, and the true-versus-recursive residual
behaviour the experiment describes."""

import numpy as np
import pytest

import oracle
import synth
from oracle.diagnostics import hs_error_estimate, plotted_proxy
from oracle.jacobi import JacobiPreconditioner
from pins import lemma_eigenpairs


def _field(shape, seed):
    return synth.charge_field(shape[::-1], ncharges=12, seed=seed).T


def _vec(U):
    return U.ravel(order="F")


@pytest.mark.parametrize("bcs", [("D", "N", "P"), ("N", "N", "P"), ("DN", "D", "ND")])
def test_kappa_is_the_error_norm_up_to_a_constant(bcs):
    # ||u_s - u*||_L^2 = kappa_s + u*^T L u*, checked on the assembled
    # Kronecker sum (eq. 3.3) with the minimum-norm solution of a dense solve
    shape = (5, 4, 6)
    H = _field(shape, 11)
    L = np.asarray(oracle.kronecker_sum(shape, bcs))
    full = oracle.pcg(H, bcs, max_iter=8, stall=10**6, true_tol=0.0)
    Hc = H - H.mean() if oracle.is_singular(bcs) else H
    ustar = _vec(oracle.dense_pinv_solve(Hc, bcs))
    c = ustar @ L @ ustar
    for s in range(1, 6):
        us = _vec(oracle.pcg(H, bcs, fixed_iterations=s).u)
        e = us - ustar
        kappa = full.diagnostics[s][1]
        assert abs(kappa + c - e @ L @ e) <= 1e-10 * c, (s, kappa)


@pytest.mark.parametrize("bc", ["D", "P", "N", "DN"])
def test_kappa_on_an_eigenmode(bc):
    # eta = v (unit eigenvector, eigenvalue lam > 0): u* = v / lam, and the
    # pseudoinverse reaches it in one iteration, so kappa_1 = -1 / lam while
    # kappa_0 = 0 and the true residual falls from 1 to rounding
    n = (7, 6, 5)
    pairs = [lemma_eigenpairs(m, bc) for m in n]
    lam = pairs[0][2][0] + pairs[1][1][0] + pairs[2][3][0]
    v = np.einsum("i,j,k->ijk", *(np.asarray(pairs[a][(2, 1, 3)[a]][1], dtype=float)
                                  for a in range(3)))
    v /= np.linalg.norm(v)
    r = oracle.solve(v, (bc, bc, bc), true_tol=1e-14)
    d = np.array(r.diagnostics)
    assert d[0, 0] == 1.0 and d[0, 1] == 0.0
    assert r.iterations == 1
    assert abs(d[1, 1] + 1.0 / lam) <= 1e-13 / lam
    assert d[1, 0] <= 1e-14
    assert abs(d[1, 3] - 1.0 / lam) <= 1e-13 / lam      # alpha_1 rho_0 = kappa_0 - kappa_1


@pytest.mark.parametrize("bcs,precond", [(("D", "D", "N"), None), (("P", "N", "P"), None),
                                         (("D", "DN", "P"), "jacobi")])
def test_hestenes_stiefel_identity_and_monotone_kappa(bcs, precond):
    # kappa_{s-1} - kappa_s = alpha_s rho_{s-1} > 0: the L-norm of the error
    # falls by exactly the Hestenes-Stiefel term in every iteration
    shape = (10, 9, 8)
    H = _field(shape, 12)
    M = JacobiPreconditioner(shape, bcs, 3, 1.3) if precond else None
    r = oracle.pcg(H, bcs, precond=M, max_iter=25, stall=10**6, true_tol=0.0)
    d = np.array(r.diagnostics)
    scale = abs(d[:, 1]).max()
    for s in range(1, len(d)):
        assert d[s, 3] > 0.0
        assert abs((d[s - 1, 1] - d[s, 1]) - d[s, 3]) <= 1e-11 * scale, s
        assert d[s, 1] <= d[s - 1, 1] + 1e-13 * scale


def test_hs_estimate_is_a_lower_bound_that_tightens():
    shape, bcs = (12, 10, 9), ("D", "N", "D")
    H = _field(shape, 13)
    L = np.asarray(oracle.kronecker_sum(shape, bcs))
    ustar = _vec(oracle.dense_pinv_solve(H, bcs))
    r = oracle.pcg(H, bcs, max_iter=60, stall=10**6, true_tol=0.0)
    d = np.array(r.diagnostics)
    est = hs_error_estimate(d[:, 3], 12)
    for s in range(0, 30):
        us = _vec(oracle.pcg(H, bcs, fixed_iterations=s).u) if s else np.zeros_like(ustar)
        e = us - ustar
        err = np.sqrt(e @ L @ e)
        assert est[s] <= err * (1 + 1e-9)
        assert est[s] >= 0.5 * err, (s, est[s], err)


@pytest.mark.parametrize("bcs", [("N", "P", "N"), ("P", "P", "P")])
def test_null_space_component(bcs):
    # against the null vector of the assembled operator (SVD), for an
    # iterate with a planted constant shift
    shape = (4, 5, 3)
    rng = np.random.default_rng(14)
    U = rng.standard_normal(shape)
    U -= U.mean()
    U += 0.37
    H = _field(shape, 15)
    H = H - H.mean()
    _, sv, vt = np.linalg.svd(np.asarray(oracle.kronecker_sum(shape, bcs)))
    assert sv[-1] < 1e-12 and sv[-2] > 1e-3
    ref = abs(vt[-1] @ _vec(U))
    _, _, null = oracle.iterate_descriptors(U, H, bcs)
    assert abs(null - ref) <= 1e-12 * ref
    _, _, null_ns = oracle.iterate_descriptors(U, H, ("D",) + tuple(bcs[1:]))
    assert null_ns == 0.0


def test_true_and_recursive_residuals_as_in_experiment_5_4():
    # they agree until convergence; afterwards the true residual stagnates at
    # rounding level while the recursive one keeps falling
    shape, bcs = (9, 8, 10), ("N", "P", "N")
    H = _field(shape, 16)
    r = oracle.pcg(H, bcs, fixed_iterations=400)
    true = np.array(r.true_rel_res)
    rec = np.array(r.rec_rel_res)
    early = rec > 1e-9
    assert early.sum() > 10
    assert np.allclose(true[early], rec[early], rtol=1e-5, atol=0)
    assert true[-50:].min() > 1e-17 and rec[-1] < 1e-2 * true[-50:].min()
    assert np.allclose([d[0] for d in r.diagnostics], true, rtol=0, atol=0)


def test_plotted_proxy_passes_through_the_first_true_residual():
    shape, bcs = (8, 8, 8), ("D", "D", "D")
    r = oracle.pcg(_field(shape, 17), bcs, max_iter=20, stall=10**6, true_tol=0.0)
    d = np.array(r.diagnostics)
    curve = plotted_proxy(d[:, 1], d[1, 0])
    assert abs(curve[1] - (d[1, 0] + 2.0 ** -52)) <= 1e-15
    assert curve.min() == 2.0 ** -52


@pytest.mark.parametrize("precond", [None, "jacobi"])
def test_anorm_stopping_rule(precond):
    # Remark 4.2's A-norm stopping: the rule first holds at s*, the returned
    # U_{s*} meets the tolerance in the L-norm (dense check), the estimate is
    # a lower bound on the error of U_{s*-d}, and the terms add up to ||u||_L^2
    from oracle.diagnostics import hs_stop_iteration
    shape, bcs = (12, 10, 9), ("D", "N", "D")
    H = _field(shape, 18)
    L = np.asarray(oracle.kronecker_sum(shape, bcs))
    ustar = _vec(oracle.dense_pinv_solve(H, bcs))
    unorm = np.sqrt(ustar @ L @ ustar)
    M = JacobiPreconditioner(shape, bcs, 3, 1.3) if precond else None
    tol, d = 1e-6, 4
    r = oracle.pcg(H, bcs, precond=M, max_iter=300, stall=10**6, true_tol=0.0)
    t = np.array(r.diagnostics)[:, 3]
    s = hs_stop_iteration(t, tol, d)
    assert s is not None and s > d
    for q in range(d, s):
        assert np.sqrt(t[q - d + 1:q + 1].sum() / t[1:q + 1].sum()) > tol
    err = lambda q: np.sqrt(max((e := _vec(oracle.pcg(H, bcs, precond=M, fixed_iterations=q).u)
                                 - ustar) @ L @ e, 0.0))
    assert err(s) <= tol * unorm
    est = np.sqrt(t[s - d + 1:s + 1].sum())
    assert est <= err(s - d) * (1 + 1e-8)
    assert abs(t[1:].sum() - unorm ** 2) <= 1e-8 * unorm ** 2


@pytest.mark.parametrize("shape,bcs,m", [((9, 8, 10), ("P", "P", "DN"), 4), ((12, 10), ("N", "D"), 5),
                                         ((7, 6, 5), ("N", "N", "P"), 3)])
def test_lowmode_bound(shape, bcs, m):
    # an upper bound on the true relative error ||L^+ R|| / ||U||, exact when
    # the box holds every mode, and never weaker than ||R|| / lambda_min
    from oracle.diagnostics import lowmode_error_bound
    rng = np.random.default_rng(19)
    H = rng.standard_normal(shape)
    if oracle.is_singular(bcs):
        H -= H.mean()
    ustar = oracle.dense_pinv_solve(H, bcs)
    U = ustar + 1e-3 * rng.standard_normal(shape)
    R = H - oracle.apply_minus_laplacian(U, bcs)
    if oracle.is_singular(bcs):
        R -= R.mean()
    err = np.linalg.norm(oracle.dense_pinv_solve(R, bcs)) / np.linalg.norm(U)
    b = lowmode_error_bound(R, U, bcs, m)
    assert err <= b * (1 + 1e-12)
    assert abs(lowmode_error_bound(R, U, bcs, max(shape)) - err) <= 1e-10 * err
    ev = np.linalg.eigvalsh(np.asarray(oracle.kronecker_sum(shape, bcs)))
    crude = np.linalg.norm(R) / ev[ev > 1e-10].min() / np.linalg.norm(U)
    assert b <= crude * (1 + 1e-12)
