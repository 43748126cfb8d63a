"""Pins of the oracle's Jacobi(p, omega) preconditioner (Sec. 4.3.1, Algs.
2-3): closed forms on the diagonal and on Fourier modes, symmetry, the limit
of many steps, and the iteration counts of the preconditioned CG."""

import itertools

import numpy as np
import pytest

import oracle
from oracle.jacobi import JacobiPreconditioner, jacobi_apply, jacobi_init
from pins import lemma_eigenpairs

ALL3 = list(itertools.product(oracle.BCS, repeat=3))


def test_one_step_is_the_scaled_residual():
    # X_1 = Dhat^{o-1} o R with Dhat the omega-scaled sum of 1D diagonals
    # (corners alpha, beta of eq. 3.1 at the ends)
    rng = np.random.default_rng(1)
    shape, bcs, omega = (4, 5, 6), ("N", "DN", "P"), 1.5
    R = rng.standard_normal(shape)
    O, Dinv = jacobi_init(shape, bcs, omega)
    d = [np.full(n, 2.0) for n in shape]
    d[0][0] = d[0][-1] = 1.0            # N: alpha = beta = 1
    d[1][-1] = 1.0                      # DN: beta = 1
    D = d[0][:, None, None] + d[1][None, :, None] + d[2][None, None, :]
    assert np.allclose(jacobi_apply(R, O, Dinv, 1), R / (omega * D), rtol=1e-15)


@pytest.mark.parametrize("p,omega", [(1, 1.0), (3, 1.0), (4, 1.7), (10, 2.5)])
def test_fourier_modes_of_a_periodic_axis(p, omega):
    # on a periodic axis D = 2 omega I and L v = lam v for the lemma's modes,
    # so each Jacobi step maps v to a multiple of v:
    # X_j = X_{j-1} + (1 - X_{j-1} lam) / (2 omega) per unit coefficient,
    # i.e. X_p = (1 - (1 - lam / (2 omega))^p) / lam (and p / (2 omega) at lam = 0)
    n = 12
    O, Dinv = jacobi_init((n,), ("P",), omega)
    for lam, v in lemma_eigenpairs(n, "P"):
        v = np.asarray(v, dtype=float)
        x = jacobi_apply(v, O, Dinv, p)
        t = 1.0 - lam / (2.0 * omega)
        mu = p / (2.0 * omega) if lam < 1e-14 else (1.0 - t ** p) / lam
        assert np.allclose(x, mu * v, atol=1e-12 * np.abs(v).max()), lam


@pytest.mark.parametrize("bcs", ALL3[::9])
def test_operator_is_symmetric(bcs):
    # M = sum_j (I - D^{-1} L / omega)^j D^{-1} / omega is symmetric
    rng = np.random.default_rng(2)
    shape = (3, 4, 5)
    O, Dinv = jacobi_init(shape, bcs, 1.3)
    a, b = rng.standard_normal(shape), rng.standard_normal(shape)
    lhs = np.vdot(jacobi_apply(a, O, Dinv, 5), b)
    rhs = np.vdot(a, jacobi_apply(b, O, Dinv, 5))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_many_steps_solve_a_nonsingular_system():
    # for a Dirichlet problem Jacobi converges, so many steps give L^{-1} R
    rng = np.random.default_rng(3)
    shape, bcs = (6, 5, 4), ("D", "D", "D")
    R = rng.standard_normal(shape)
    O, Dinv = jacobi_init(shape, bcs, 1.0)
    x = jacobi_apply(R, O, Dinv, 2000)
    ref = oracle.dense_pinv_solve(R, bcs)
    assert np.allclose(x, ref, rtol=0, atol=1e-10 * np.abs(ref).max())


def test_iterations_rank_as_in_the_paper():
    # the paper's observation (Experiment 5.5, with its Jacobi(3, 1.3)): the
    # pseudoinverse needs two or three iterations, Jacobi fewer than plain CG
    import synth
    eta = synth.charge_field((20, 24, 16), ncharges=60, seed=4).T
    bcs = ("D", "N", "P")
    # (plain CG's residual is not monotone: count iterations to 1e-10 without
    # the oracle's stagnation stop)
    kw = dict(true_tol=1e-10, max_iter=1000, stall=10**6)
    it_pinv = oracle.pcg(eta, bcs, precond=oracle.PinvPreconditioner(eta.shape, bcs), **kw).iterations
    it_jac = oracle.pcg(eta, bcs, precond=JacobiPreconditioner(eta.shape, bcs, 3, 1.3),
                        **kw).iterations
    it_cg = oracle.pcg(eta, bcs, **kw).iterations
    assert it_pinv <= 3 < it_jac < it_cg, (it_pinv, it_jac, it_cg)
