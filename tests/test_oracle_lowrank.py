"""Pins of the oracle's low-Kronecker-rank preconditioner (Sec. 4.3.2): full
rank is the pseudoinverse, the operator is diagonal in the eigenbasis with a
best rank-r multiplier matrix (Eckart-Young error, from an independent
eigenvalue routine and the lemmas' closed-form eigenvalues), symmetry, the
positivity facts the paper states, and the iteration ranking of
Experiment 5.5."""

import numpy as np
import pytest

import oracle
import synth
from oracle.jacobi import JacobiPreconditioner
from oracle.lowrank import LowRankPreconditioner, lowrank_apply, lowrank_init
from pins import lemma_eigenpairs


def _ghat_closed_form(n, q, bcs):
    ln = np.array([lam for lam, _ in lemma_eigenpairs(n, bcs[0])])
    lq = np.array([lam for lam, _ in lemma_eigenpairs(q, bcs[1])])
    S = ln[:, None] + lq[None, :]
    small = np.abs(S) < 1e-13
    return np.where(small, 0.0, 1.0 / np.where(small, 1.0, S)), lemma_eigenpairs(n, bcs[0]), \
        lemma_eigenpairs(q, bcs[1])


def _multipliers(shape, bcs, rank):
    """The operator applied to every (closed-form, normalised) eigenmode
    v_i (x) w_j: returns the matrix of Rayleigh quotients and the largest
    off-diagonal leakage."""
    n, q = shape
    _, pn, pq = _ghat_closed_form(n, q, bcs)
    pairs = lowrank_init(shape, bcs, rank)
    mult = np.zeros(shape)
    leak = 0.0
    for i, (_, v) in enumerate(pn):
        v = np.asarray(v, float) / np.linalg.norm(v)
        for j, (_, w) in enumerate(pq):
            w = np.asarray(w, float) / np.linalg.norm(w)
            mode = np.outer(v, w)
            z = lowrank_apply(mode, pairs)
            mult[i, j] = np.sum(z * mode)
            leak = max(leak, np.linalg.norm(z - mult[i, j] * mode))
    return mult, leak


@pytest.mark.parametrize("shape,bcs", [((6, 9), ("D", "DN")), ((7, 5), ("P", "N")),
                                       ((8, 8), ("ND", "D"))])
def test_full_rank_is_the_pseudoinverse(shape, bcs):
    rng = np.random.default_rng(30)
    R = rng.standard_normal(shape)
    V, lam, G = oracle.pinv_init(shape, bcs)
    ref = oracle.pinv_apply(R, V, G)
    z = lowrank_apply(R, lowrank_init(shape, bcs, min(shape)))
    assert np.allclose(z, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("shape,bcs,rank", [((9, 12), ("D", "DN"), 1), ((9, 12), ("D", "DN"), 3),
                                            ((10, 7), ("ND", "D"), 2), ((11, 13), ("DN", "D"), 4)])
def test_best_rank_r_multipliers(shape, bcs, rank):
    # diagonal in the eigenbasis (no leakage between modes); the multiplier
    # matrix has rank r and the optimal Frobenius distance to Ghat, i.e. the
    # sum of the discarded squared singular values (Eckart-Young-Mirsky),
    # here from the eigenvalues of Ghat^T Ghat (Ghat from the lemmas)
    mult, leak = _multipliers(shape, bcs, rank)
    G, _, _ = _ghat_closed_form(*shape, bcs)
    assert leak <= 1e-12 * np.abs(mult).max()
    s2 = np.sort(np.linalg.eigvalsh(G.T @ G))[::-1]
    assert s2[rank - 1] > 1.01 * s2[rank]          # a unique best approximation
    err2 = np.sum((G - mult) ** 2)
    assert abs(err2 - s2[rank:].sum()) <= 1e-10 * s2[0]
    sv = np.linalg.svd(mult, compute_uv=False)
    assert sv[rank - 1] > 1e-6 * sv[0] and (rank == len(sv) or sv[rank] <= 1e-12 * sv[0])


def test_symmetric_operator():
    shape, bcs = (10, 14), ("N", "DN")
    rng = np.random.default_rng(31)
    a, b = rng.standard_normal(shape), rng.standard_normal(shape)
    pairs = lowrank_init(shape, bcs, 3)
    lhs, rhs = np.sum(lowrank_apply(a, pairs) * b), np.sum(a * lowrank_apply(b, pairs))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_positivity_facts():
    # rank 1 is positive semi-definite (Ghat is entrywise non-negative, so its
    # leading singular vectors are); intermediate ranks need not be: here a
    # rank-2 approximation has a negative eigenvalue
    for shape, bcs in [((9, 12), ("D", "DN")), ((12, 8), ("N", "P"))]:
        mult, _ = _multipliers(shape, bcs, 1)
        assert mult.min() >= -1e-14
    mult, _ = _multipliers((20, 30), ("N", "P"), 2)
    assert mult.min() < -0.05


@pytest.mark.parametrize("shape,bcs", [((50, 100), ("N", "P")), ((64, 64), ("D", "D"))])
def test_iteration_ranking_of_experiment_5_5(shape, bcs):
    # M = I worst, then Jacobi(3, 1.3), then low-rank(3), the pseudoinverse
    # best (one iteration), on Gaussian-blob fields
    eta = synth.gaussian_blobs_2d(shape[0], shape[1], 16, 2.0, seed=1).T
    kw = dict(true_tol=1e-10, max_iter=2000, stall=10**6)
    it = lambda M: oracle.pcg(eta, bcs, precond=M, **kw).iterations
    i_pinv = it(oracle.PinvPreconditioner(shape, bcs))
    i_lr = it(LowRankPreconditioner(shape, bcs, 3))
    i_jac = it(JacobiPreconditioner(shape, bcs, 3, 1.3))
    i_cg = it(None)
    assert i_pinv <= 3 < i_lr < i_jac < i_cg, (i_pinv, i_lr, i_jac, i_cg)


def test_indefinite_on_a_live_mode():
    # the low-rank operator can be indefinite away from the null space: on a
    # 100 x 100 (D, DN) grid the rank-3 approximation of Ghat has a negative
    # entry at the eigenmode pair (1, 99) (ascending eigenvalues), so that
    # mode has <v, M v> < 0 and preconditioned CG started on it breaks down
    # at once (rho_0 < 0); rank 1 stays positive there
    from pins import lemma_basis
    n, q, bcs = 100, 100, ("D", "DN")
    Qn, _ = lemma_basis(n, "D")
    Qq, _ = lemma_basis(q, "DN")
    v = np.outer(Qn[:, 1], Qq[:, 99])
    rq3 = float(np.sum(lowrank_apply(v, lowrank_init((n, q), bcs, 3)) * v))
    rq1 = float(np.sum(lowrank_apply(v, lowrank_init((n, q), bcs, 1)) * v))
    assert rq3 < 0.0 < rq1
    # the same entry of G_r from the SVD of Ghat (Eckart-Young), independently
    ghat, _, _ = _ghat_closed_form(n, q, bcs)
    X, sig, Yt = np.linalg.svd(ghat)
    g3 = (X[:, :3] * sig[:3]) @ Yt[:3]
    assert abs(g3[1, 99] - rq3) <= 1e-10 * np.abs(g3).max()
