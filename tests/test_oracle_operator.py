"""Oracle pins: the minus Laplacian of eq. (3.2) and the layout of Sec. 2."""

import itertools

import numpy as np
import pytest

import oracle
from pins import ghost_rule_stencil

ALL3 = list(itertools.product(oracle.BCS, repeat=3))
ALL2 = list(itertools.product(oracle.BCS, repeat=2))


def test_vec_and_kron_identity():
    # eq. (2.3): vec(A U B^T) = (B (x) A) vec(U), with vec = column stacking
    rng = np.random.default_rng(0)
    A = rng.standard_normal((3, 4)); U = rng.standard_normal((4, 5)); B = rng.standard_normal((2, 5))
    lhs = (A @ U @ B.T).ravel(order="F")
    rhs = np.kron(B, A) @ U.ravel(order="F")
    assert np.allclose(lhs, rhs)
    # the mode-1 product is multiplication of every column, the mode-2 product
    # of every row (Sec. 2.2)
    from oracle.laplacian import _mode_product
    assert np.allclose(_mode_product(A, U, 0), A @ U)
    assert np.allclose(_mode_product(B, U, 1), U @ B.T)
    T = rng.standard_normal((3, 4, 5)); C = rng.standard_normal((6, 5))
    # vec(C x_3 T) = (C (x) I_q (x) I_n) vec(T)
    lhs = _mode_product(C, T, 2).ravel(order="F")
    rhs = np.kron(C, np.kron(np.eye(4), np.eye(3))) @ T.ravel(order="F")
    assert np.allclose(lhs, rhs)


@pytest.mark.parametrize("bcs", ALL3)
def test_stencil_vs_kronecker_and_ghost_rule_3d(bcs):
    rng = np.random.default_rng(1)
    shape = (3, 4, 5)
    U = rng.standard_normal(shape)
    W = oracle.apply_minus_laplacian(U, bcs)
    Wk = (oracle.kronecker_sum(shape, bcs) @ U.ravel(order="F")).reshape(shape, order="F")
    Wg = ghost_rule_stencil(U, bcs)
    assert np.allclose(W, Wk, atol=1e-13, rtol=0)
    assert np.allclose(W, Wg, atol=1e-13, rtol=0)


@pytest.mark.parametrize("bcs", ALL2)
def test_stencil_vs_kronecker_and_ghost_rule_2d(bcs):
    rng = np.random.default_rng(2)
    shape = (5, 3)
    U = rng.standard_normal(shape)
    W = oracle.apply_minus_laplacian(U, bcs)
    Wk = (oracle.kronecker_sum(shape, bcs) @ U.ravel(order="F")).reshape(shape, order="F")
    assert np.allclose(W, Wk, atol=1e-13, rtol=0)
    assert np.allclose(W, ghost_rule_stencil(U, bcs), atol=1e-13, rtol=0)
    # 2D form of eq. (3.2): L_n U + U L_q^T
    Ln = oracle.laplacian_1d(shape[0], bcs[0]); Lq = oracle.laplacian_1d(shape[1], bcs[1])
    assert np.allclose(W, Ln @ U + U @ Lq.T)


def test_integer_stencil_is_exact():
    # integer coefficients: on integer data the result is exact
    rng = np.random.default_rng(3)
    U = rng.integers(-1000, 1000, size=(6, 5, 7)).astype(np.float64)
    for bcs in [("P", "D", "N"), ("DN", "ND", "P")]:
        W = oracle.apply_minus_laplacian(U, bcs)
        Wd = oracle.apply_minus_laplacian(U, bcs, dense=True)
        assert np.array_equal(W, Wd)
        assert np.array_equal(W, ghost_rule_stencil(U, bcs))


@pytest.mark.parametrize("bcs", [("P", "P", "P"), ("N", "N", "N"), ("P", "N", "P"), ("D", "P", "N")])
def test_symmetry_and_null_space(bcs):
    rng = np.random.default_rng(4)
    shape = (6, 5, 4)
    x = rng.standard_normal(shape); y = rng.standard_normal(shape)
    Lx = oracle.apply_minus_laplacian(x, bcs); Ly = oracle.apply_minus_laplacian(y, bcs)
    assert abs(np.sum(Lx * y) - np.sum(x * Ly)) < 1e-11
    ones = np.ones(shape)
    L1 = oracle.apply_minus_laplacian(ones, bcs)
    if oracle.is_singular(bcs):
        assert np.max(np.abs(L1)) == 0.0
    else:
        assert np.max(np.abs(L1)) > 0.0
    # positive semidefinite
    assert np.sum(Lx * x) >= -1e-12
