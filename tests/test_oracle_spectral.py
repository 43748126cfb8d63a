"""Oracle pins: the minimum-norm solution from the eigen-expansion, and the
preconditioned CG started from a given iterate."""

import itertools

import numpy as np
import pytest

import oracle
import oracle.spectral as ospec
import synth
from pins import lemma_basis

ALL3 = list(itertools.product(oracle.BCS, repeat=3))
ALL2 = list(itertools.product(oracle.BCS, repeat=2))


def _brute(shape, bcs, seed):
    H = np.random.default_rng(seed).standard_normal(shape)
    return H, oracle.dense_pinv_solve(H, bcs)


@pytest.mark.parametrize("bcs", ALL3)
@pytest.mark.parametrize("shape", [(3, 4, 5), (4, 4, 4), (6, 5, 3)])
def test_min_norm_vs_svd_3d(shape, bcs):
    # the assembled eq. (3.3) solved by an SVD pseudoinverse
    H, ref = _brute(shape, bcs, 1)
    u, removed = oracle.min_norm_solution(H, bcs)
    assert np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref), (shape, bcs)
    assert np.max(np.abs(u - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert removed == (H.mean() if oracle.is_singular(bcs) else 0.0)


@pytest.mark.parametrize("bcs", ALL2)
@pytest.mark.parametrize("shape", [(5, 7), (8, 3)])
def test_min_norm_vs_svd_2d(shape, bcs):
    H, ref = _brute(shape, bcs, 2)
    u, _ = oracle.min_norm_solution(H, bcs)
    assert np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref), (shape, bcs)


@pytest.mark.parametrize("shape,bcs", [((7, 6, 5), ("DN", "P", "N")), ((8, 8, 6), ("P", "P", "P")),
                                       ((9, 5, 4), ("ND", "D", "DN")), ((6, 10), ("N", "P"))])
def test_min_norm_on_closed_form_modes(shape, bcs):
    # a product of lemma eigenvectors (Lemmas 3.1-3.4) is an eigenvector of
    # the Kronecker sum: its solution is itself over the eigenvalue sum, and
    # the null mode of a singular set maps to 0
    rng = np.random.default_rng(3)
    bases = [lemma_basis(n, bc) for n, bc in zip(shape, bcs)]
    picks = [[0] * len(shape)] + [[int(rng.integers(0, n)) for n in shape] for _ in range(5)]
    for idx in picks:
        H = np.ones([1] * len(shape))
        mu = 0.0
        for a, (Q, lam) in enumerate(bases):
            sh = [1] * len(shape)
            sh[a] = shape[a]
            H = H * Q[:, idx[a]].reshape(sh)
            mu += lam[idx[a]]
        u, _ = oracle.min_norm_solution(H, bcs)
        expect = np.zeros_like(H) if abs(mu) < 1e-12 else H / mu
        assert np.max(np.abs(u - expect)) <= 1e-12 * max(1.0, np.max(np.abs(expect))), (bcs, idx)


@pytest.mark.parametrize("shape,bcs", [((24, 20, 16), ("P", "P", "DN")),
                                       ((16, 16, 16), ("N", "N", "N")),
                                       ((12, 18, 30), ("P", "P", "D"))])
def test_min_norm_solves_the_centred_system(shape, bcs):
    # L u = eta_c (eq. 3.6) to rounding, zero mean for a singular set, and
    # the same answer as the preconditioned CG iterated to stagnation (two
    # routes to L^+ eta)
    H = synth.charge_field(shape[::-1], ncharges=300, seed=4, zero_mean=False).T
    u, removed = oracle.min_norm_solution(H, bcs)
    hc = H - removed
    res = oracle.apply_minus_laplacian(u, bcs) - hc
    assert np.linalg.norm(res) <= 1e-13 * np.linalg.norm(hc)
    if oracle.is_singular(bcs):
        assert abs(u.mean()) <= 1e-15 * np.max(np.abs(u))
    ref = oracle.solve(H, bcs).u
    assert np.linalg.norm(u - ref) <= 1e-13 * np.linalg.norm(ref)


def test_transposed_basis_is_caught(monkeypatch):
    # planted mistake: the forward transform contracts the wrong index of the
    # eigenvector matrix
    def wrong(H, bases):
        C = np.asarray(H, dtype=np.float64)
        for axis, (_, V) in enumerate(bases):
            C = np.moveaxis(np.tensordot(V, C, axes=([1], [axis])), 0, axis)
        return C
    monkeypatch.setattr(ospec, "_to_modes", wrong)
    H, ref = _brute((4, 5, 3), ("DN", "P", "N"), 5)
    u, _ = oracle.min_norm_solution(H, ("DN", "P", "N"))
    assert np.linalg.norm(u - ref) > 1e-6 * np.linalg.norm(ref)


def test_missing_null_threshold_is_caught(monkeypatch):
    monkeypatch.setattr(ospec, "NULL_THRESHOLD", -1.0)
    H, ref = _brute((4, 4, 3), ("P", "N", "P"), 6)
    with np.errstate(divide="ignore", invalid="ignore"):
        u, _ = oracle.min_norm_solution(H, ("P", "N", "P"))
    assert not (np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref))


# ------------------------------------------------------------ warm start ----
@pytest.mark.parametrize("bcs", [("D", "N", "P"), ("P", "P", "N"), ("DN", "D")])
def test_warm_start_at_the_solution_takes_no_iteration(bcs):
    # a start that already solves the system (to rounding) makes no step and
    # is returned (centred for a singular set)
    shape = (9, 7, 6)[: len(bcs)]
    H = np.random.default_rng(7).standard_normal(shape)
    u_star, _ = oracle.min_norm_solution(H, bcs)
    shift = 0.75 if oracle.is_singular(bcs) else 0.0   # a null-space component
    res = oracle.solve(H, bcs, u0=u_star + shift)
    assert res.iterations == 0
    assert res.true_rel_res[0] <= 1e-14
    assert np.linalg.norm(res.u - u_star) <= 1e-14 * np.linalg.norm(u_star)


@pytest.mark.parametrize("bcs", ALL3[::11])
def test_warm_start_reaches_the_minimum_norm_solution(bcs):
    # from an arbitrary start the iteration still converges to L^+ eta: the
    # start's null-space component is removed, the rest is corrected
    shape = (5, 4, 6)
    rng = np.random.default_rng(8)
    H = rng.standard_normal(shape)
    ref = oracle.dense_pinv_solve(H, bcs)
    res = oracle.solve(H, bcs, u0=rng.standard_normal(shape))
    assert np.linalg.norm(res.u - ref) <= 1e-12 * np.linalg.norm(ref), bcs
    # the first recorded residual is that of the start, not ||eta||
    assert res.rec_rel_res[0] > 1e-3


def test_warm_start_near_solution_saves_iterations_without_preconditioner():
    # plain CG (M = I) from a start close to the solution needs fewer steps
    # than from zero, and both end at the same answer
    shape = (10, 8, 6)
    bcs = ("D", "D", "N")
    H = np.random.default_rng(9).standard_normal(shape)
    u_star, _ = oracle.min_norm_solution(H, bcs)
    near = u_star + 1e-6 * np.random.default_rng(10).standard_normal(shape)
    cold = oracle.pcg(H, bcs, precond=None, max_iter=400, true_tol=1e-12)
    warm = oracle.pcg(H, bcs, precond=None, u0=near, max_iter=400, true_tol=1e-12)
    assert warm.iterations < cold.iterations
    for r in (cold, warm):
        assert np.linalg.norm(r.u - u_star) <= 1e-10 * np.linalg.norm(u_star)
