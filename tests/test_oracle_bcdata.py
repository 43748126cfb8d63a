"""Pins of the boundary-data update (Sec. 3.4.2) and of the field eps = -grad u
(Sec. 1) in the oracle, against an independent ghost-layer construction,
closed-form linear profiles and the paper's mixed-BC problem setup."""

import itertools

import numpy as np
import pytest

import oracle
from oracle.bcdata import assemble_rhs, field, minus_laplacian_with_ghosts

ALL3 = list(itertools.product(oracle.BCS, repeat=3))


def _faces(bcs, rng):
    f = rng.standard_normal((len(bcs), 2))
    for a, bc in enumerate(bcs):
        if bc == "P":
            f[a] = 0.0
    return f


@pytest.mark.parametrize("bcs", ALL3)
def test_update_equals_ghost_operator(bcs):
    # moving the prescribed boundary values to the right-hand side: the
    # operator with ghost values is the homogeneous one minus the update
    rng = np.random.default_rng(ALL3.index(bcs))
    u = rng.standard_normal((3, 4, 5))
    f = _faces(bcs, rng)
    lhs = minus_laplacian_with_ghosts(u, bcs, f)
    rhs = oracle.apply_minus_laplacian(u, bcs) - assemble_rhs(np.zeros(u.shape), bcs, f)
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-13)


def test_homogeneous_data_changes_nothing():
    rng = np.random.default_rng(1)
    eta = rng.standard_normal((4, 5, 6))
    for bcs in ALL3[::7]:
        assert np.array_equal(assemble_rhs(eta, bcs, None), eta)
        assert np.allclose(minus_laplacian_with_ghosts(eta, bcs, None),
                           oracle.apply_minus_laplacian(eta, bcs), atol=1e-14)


@pytest.mark.parametrize("bc", ["D", "N", "DN", "ND"])
def test_linear_profile_is_exact(bc):
    # u_j = a + b j (j = 1..n) with boundary data read off the same line:
    # Dirichlet ends take the node values u_0 and u_{n+1}, Neumann ends the
    # outward differences u_0 - u_1 = -b and u_{n+1} - u_n = b; then the
    # discrete Laplacian vanishes and the field is -b everywhere
    n, a, b = 9, 0.7, -1.3
    j = np.arange(1, n + 1, dtype=float)
    u = a + b * j
    ends = {"D": ("D", "D"), "N": ("N", "N"), "DN": ("D", "N"), "ND": ("N", "D")}[bc]
    f = np.array([[a if ends[0] == "D" else -b, (a + b * (n + 1)) if ends[1] == "D" else b]])
    assert np.allclose(minus_laplacian_with_ghosts(u, (bc,), f), 0.0, atol=1e-13)
    assert np.allclose(field(u, (bc,), f)[0], -b, atol=1e-14)


def test_dirichlet_solve_gives_the_line():
    # L_D u = i_1 u_B + i_n u_E is solved by the straight line through the
    # two boundary nodes
    n, uB, uE = 12, 2.0, -1.0
    rhs = assemble_rhs(np.zeros(n), ("D",), [[uB, uE]])
    u = np.linalg.solve(oracle.laplacian_1d(n, "D"), rhs)
    j = np.arange(1, n + 1)
    assert np.allclose(u, uB + (uE - uB) * j / (n + 1), atol=1e-13)


def test_mixed_problem_setup_of_problem_5_2():
    # 40 x 120, zero potential on the left, outward derivative -1/2 on the
    # right, periodic vertically, no charge: the potential is u_i = -i/2 and
    # the field is 1/2 in x and 0 in y
    nx, ny = 40, 120
    faces = [[0.0, -0.5], [0.0, 0.0]]
    rhs = assemble_rhs(np.zeros((nx, ny)), ("DN", "P"), faces)
    res = oracle.solve(rhs, ("DN", "P"))
    i = np.arange(1, nx + 1, dtype=float)[:, None]
    assert np.allclose(res.u, -0.5 * i * np.ones((1, ny)), atol=1e-10)
    eps = field(res.u, ("DN", "P"), faces)
    assert np.allclose(eps[0], 0.5, atol=1e-10) and np.allclose(eps[1], 0.0, atol=1e-10)


def test_field_of_a_quadratic_and_periodic_wrap():
    # central differences are exact for quadratics away from the walls, and
    # a periodic axis wraps
    n = 8
    i = np.arange(1, n + 1, dtype=float)
    eps = field(i ** 2, ("D",), [[0.0, (n + 1) ** 2]])
    assert np.allclose(eps[0], -2.0 * i, atol=1e-12)
    u = np.sin(2 * np.pi * np.arange(n) / n)
    e = field(u, ("P",))[0]
    assert np.isclose(e[0], -(u[1] - u[-1]) / 2) and np.isclose(e[-1], -(u[0] - u[-2]) / 2)


def test_periodic_axis_rejects_data():
    with pytest.raises(ValueError):
        assemble_rhs(np.zeros((4, 4)), ("P", "D"), [[1.0, 0.0], [0.0, 0.0]])
