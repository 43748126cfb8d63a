"""Oracle pins: Algorithm 1 with the pseudoinverse preconditioner."""

import itertools
import os

import numpy as np
import pytest

import oracle
import synth
from pins import pin_solve_brute

ALL3 = list(itertools.product(oracle.BCS, repeat=3))
ALL2 = list(itertools.product(oracle.BCS, repeat=2))
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("bcs", ALL3)
@pytest.mark.parametrize("shape", [(3, 4, 5), (5, 4, 3), (4, 4, 4)])
def test_solve_vs_brute_force_3d(shape, bcs):
    pin_solve_brute(shape, bcs)


@pytest.mark.parametrize("bcs", ALL3[::7])
def test_solve_vs_brute_force_3d_765(bcs):
    pin_solve_brute((7, 6, 5), bcs)


@pytest.mark.parametrize("bcs", ALL2)
@pytest.mark.parametrize("shape", [(5, 7), (6, 4)])
def test_solve_vs_brute_force_2d(shape, bcs):
    pin_solve_brute(shape, bcs)


@pytest.mark.parametrize("bcs", [("D", "P", "N"), ("DN", "DN", "ND"), ("D", "D")])
def test_manufactured_solution(bcs):
    # non-singular: pick U, form H = L U, recover U
    rng = np.random.default_rng(11)
    shape = (9, 7, 6)[: len(bcs)]
    U = rng.standard_normal(shape)
    H = oracle.apply_minus_laplacian(U, bcs)
    res = oracle.solve(H, bcs)
    assert np.linalg.norm(res.u - U) / np.linalg.norm(U) < 1e-12


@pytest.mark.parametrize("bcs", [("P", "P", "P"), ("N", "N", "N"), ("P", "N", "N"), ("P", "P")])
def test_singular_invariants(bcs):
    rng = np.random.default_rng(12)
    shape = (8, 6, 5)[: len(bcs)]
    U = rng.standard_normal(shape)
    U -= U.mean()
    H = oracle.apply_minus_laplacian(U, bcs)
    # a constant added to H is projected out (eq. 3.6) and reported
    res = oracle.solve(H + 0.25, bcs)
    assert abs(res.removed_mean - 0.25) < 1e-12
    assert abs(res.u.mean()) < 1e-14
    assert np.linalg.norm(res.u - U) / np.linalg.norm(U) < 1e-12
    # the null-space direction alone gives the zero solution
    res0 = oracle.solve(np.full(shape, -2.0), bcs)
    assert np.max(np.abs(res0.u)) == 0.0 and res0.iterations == 0


def test_zero_rhs():
    res = oracle.solve(np.zeros((4, 5, 6)), ("D", "D", "D"))
    assert res.iterations == 0 and np.max(np.abs(res.u)) == 0.0


@pytest.mark.parametrize("shape,bcs,seed", [
    ((32, 32, 16), ("P", "P", "DN"), 2),
    ((24, 24, 24), ("N", "N", "N"), 3000),
    ((16, 16, 64), ("P", "P", "D"), 5),
])
def test_few_iterations_suffice(shape, bcs, seed):
    # Sec. 5.2 / Sec. 6: with the pseudoinverse preconditioner PCG is almost
    # done after one iteration and two or three iterations suffice
    H = synth.charge_field(shape[::-1], ncharges=200, seed=seed).T
    res = oracle.solve(H, bcs)
    assert res.true_rel_res[1] < 1e-12
    assert min(res.true_rel_res[:4]) < 1e-13
    # the recursive residual tracks the true one until it stagnates (Exp. 5.4)
    assert abs(res.rec_rel_res[1] - res.true_rel_res[1]) < 1e-13


def test_normalisation_of_initial_residual():
    # eq. (5.1) and the values printed in Experiment 5.6
    rows = []
    with open(os.path.join(HERE, "golden", "normalization.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                grid, value = line.split()
                rows.append((tuple(int(x) for x in grid.split("x")), float(value)))
    assert len(rows) == 2
    for dims, printed in rows:
        N = int(np.prod(dims))
        assert 1.0 / N == printed
        if N <= 100:
            rng = np.random.default_rng(5)
            H = rng.standard_normal(dims)
            H *= (1.0 / N) / np.linalg.norm(H)
            res = oracle.pcg(H, ("P", "P"), precond=oracle.PinvPreconditioner(dims, ("P", "P")),
                             fixed_iterations=1)
            # ||R_0|| = ||H|| since U_0 = 0 (Algorithm 1, W_0 = -Delta(0) = 0);
            # H is not centred here, so compare with the centred norm
            assert abs(res.rec_rel_res[0] * res.h_norm - np.linalg.norm(H - H.mean())) < 1e-18


def test_unpreconditioned_cg_converges():
    # M = I is plain CG (Experiment 5.5); it converges, just more slowly
    rng = np.random.default_rng(9)
    H = rng.standard_normal((10, 8, 6))
    res = oracle.pcg(H, ("D", "D", "D"), precond=None, max_iter=400, true_tol=1e-12)
    ref = oracle.dense_pinv_solve(H, ("D", "D", "D"))
    assert res.iterations > 5
    assert np.linalg.norm(res.u - ref) / np.linalg.norm(ref) < 1e-10
