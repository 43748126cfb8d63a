"""Non-homogeneous boundary data (kp_assemble_rhs) and the field eps = -grad u
(kp_field) against the oracle, and a non-homogeneous solve end to end."""

import itertools

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_close, grid_dims, to_dev, to_host

pytestmark = pytest.mark.gpu

ALL3 = list(itertools.product(oracle.BCS, repeat=3))


def _plan(shape, bcs, prec="f64", max_batch=1):
    from paper_2501_03377_amd import Plan
    nx, ny, nz = grid_dims(shape)
    return Plan(nx, ny, nz, bcs, prec=prec, max_batch=max_batch)


def _faces(bcs, rng):
    f = rng.standard_normal((len(bcs), 2))
    for a, bc in enumerate(bcs):
        if bc == "P":
            f[a] = 0.0
    return f


def test_assemble_and_field_all_bc_triples():
    # element by element against the oracle (device arrays are the transpose
    # of the paper-indexed oracle arrays; face data is [axis][end] in both)
    shape = (5, 6, 7)
    rng = np.random.default_rng(70)
    for k, bcs in enumerate(ALL3):
        eta = rng.standard_normal(shape)
        u = rng.standard_normal(shape)
        f = _faces(bcs, rng)
        plan = _plan(shape, bcs)
        rhs = to_host(plan.assemble_rhs(to_dev(eta), f))
        assert np.array_equal(rhs, oracle.assemble_rhs(eta.T, bcs, f).T), bcs
        eps = to_host(plan.field(to_dev(u), f))
        ref = oracle.field(u.T, bcs, f)
        for a in range(3):
            assert np.array_equal(eps[a], ref[a].T), (bcs, a)
        plan.close()


@pytest.mark.parametrize("shape,bcs", [((33, 70, 129), ("DN", "P", "ND")),
                                       ((40, 64), ("N", "D")),
                                       ((64, 48, 20), ("D", "N", "P"))])
def test_assemble_and_field_batched_multi_tile(shape, bcs):
    rng = np.random.default_rng(71)
    dim = len(shape)
    batch = 3
    eta = rng.standard_normal((batch,) + shape)
    u = rng.standard_normal((batch,) + shape)
    faces = np.stack([_faces(bcs, rng) for _ in range(batch)])
    plan = _plan(shape, bcs, max_batch=batch)
    e = to_dev(eta)
    rhs = to_host(plan.assemble_rhs(e, faces, out=e))      # in place
    eps = to_host(plan.field(to_dev(u), faces))
    assert eps.shape == (batch, dim) + shape
    for b in range(batch):
        assert np.array_equal(rhs[b], oracle.assemble_rhs(eta[b].T, bcs, faces[b]).T)
        ref = oracle.field(u[b].T, bcs, faces[b])
        for a in range(dim):
            assert np.array_equal(eps[b, a], ref[a].T)


def test_mixed_boundary_problem_end_to_end():
    # the setup of the paper's mixed-BC problem (2D 40 x 120: zero potential
    # on the left, outward derivative -1/2 on the right, periodic vertically)
    # with a band of positive charge; the charge-free case has the exact
    # solution u_i = -i/2 with field (1/2, 0)
    nx, ny = 40, 120
    faces = np.array([[0.0, -0.5], [0.0, 0.0]])
    plan = _plan((ny, nx), ("DN", "P"))
    rhs = plan.assemble_rhs(to_dev(np.zeros((ny, nx))), faces)
    u, res, _, rc = plan.solve(rhs, tol=1e-12)
    i = np.arange(1, nx + 1, dtype=float)[None, :]
    assert rc == 0
    assert_close(to_host(u), -0.5 * i * np.ones((ny, 1)), 1e-10)
    eps = to_host(plan.field(u, faces))
    assert np.allclose(eps[0], 0.5, atol=1e-9) and np.allclose(eps[1], 0.0, atol=1e-9)
    # a band of charge: GPU potential and field against the oracle
    eta = np.zeros((ny, nx))
    eta[:, 15:20] = 1.0
    rhs = plan.assemble_rhs(to_dev(eta), faces)
    u, res, _, rc = plan.solve(rhs, tol=1e-12)
    ref = oracle.min_norm_solution(oracle.assemble_rhs(eta.T, ("DN", "P"), faces), ("DN", "P"))[0]
    assert rc == 0
    assert_close(to_host(u), ref.T, 1e-10)
    eps = to_host(plan.field(u, faces))
    ref_eps = oracle.field(ref, ("DN", "P"), faces)
    # the band is uniform in y, so the y-component is zero up to rounding:
    # compare it on the scale of the field
    scale = np.abs(ref_eps[0]).max()
    assert_close(eps[0], ref_eps[0].T, 1e-9)
    assert np.abs(eps[1] - ref_eps[1].T).max() <= 1e-9 * scale


def test_nonhomogeneous_3d_solve_in_mixed_precision():
    shape, bcs = (24, 36, 30), ("D", "N", "DN")
    rng = np.random.default_rng(72)
    faces = _faces(bcs, rng)
    eta = synth.charge_field(shape, ncharges=200, seed=73)
    plan = _plan(shape, bcs, prec="f32")
    u, res, _, rc = plan.solve(plan.assemble_rhs(to_dev(eta), faces), tol=1e-10)
    ref = oracle.min_norm_solution(oracle.assemble_rhs(eta.T, bcs, faces), bcs)[0].T
    assert rc == 0
    assert_close(to_host(u), ref, 1e-10)


def test_periodic_face_data_is_rejected():
    from paper_2501_03377_amd import KpError
    plan = _plan((8, 8, 8), ("P", "D", "N"))
    x = to_dev(np.zeros((8, 8, 8)))
    with pytest.raises(KpError):
        plan.assemble_rhs(x, [[1.0, 0.0], [0.0, 0.0], [0.0, 0.0]])
    with pytest.raises(KpError):
        plan.field(x, [[0.0, 0.0], [np.nan, 0.0], [0.0, 0.0]])


# ------------------------------------------------------------- Jacobi(p, w) ----
@pytest.mark.parametrize("shape,bcs,steps,omega", [((5, 6, 7), ("N", "DN", "P"), 1, 1.0),
                                                   ((33, 70, 67), ("D", "ND", "P"), 3, 1.3),
                                                   ((40, 64), ("N", "D"), 4, 1.7),
                                                   ((24, 20, 36), ("P", "P", "P"), 5, 2.0)])
def test_jacobi_preconditioner_parity(shape, bcs, steps, omega):
    from oracle.jacobi import jacobi_apply, jacobi_init
    rng = np.random.default_rng(80)
    r = rng.standard_normal(shape)
    plan = _plan(shape, bcs)
    plan.set_preconditioner("jacobi", steps, omega)
    z = to_host(plan.apply_preconditioner(to_dev(r)))
    O, Dinv = jacobi_init(r.T.shape, bcs, omega)
    ref = jacobi_apply(r.T, O, Dinv, steps).T
    assert_close(z, ref, 1e-14)


def test_jacobi_solves_match_the_oracle_and_rank_as_in_the_paper():
    # PCG with Jacobi(3, 1.3) reaches the oracle's solution; it needs more
    # iterations than the pseudoinverse and fewer than plain CG
    from paper_2501_03377_amd import KP_FLAG_NO_PRECOND
    shape, bcs = (16, 24, 20), ("D", "N", "P")
    eta = synth.charge_field(shape, ncharges=60, seed=4)
    ref = oracle.min_norm_solution(eta.T, bcs)[0].T
    plan = _plan(shape, bcs)
    u_p, res_p, _, rc = plan.solve(to_dev(eta), tol=1e-10)
    assert rc == 0
    u_cg, res_cg, _, rc = plan.solve(to_dev(eta), tol=1e-10, max_iter=1000, flags=KP_FLAG_NO_PRECOND)
    assert rc == 0
    plan.set_preconditioner("jacobi", 3, 1.3)
    u_j, res_j, _, rc = plan.solve(to_dev(eta), tol=1e-10, max_iter=1000)
    assert rc == 0
    # the pseudoinverse certifies the error; CG and Jacobi stop on the
    # residual alone (tol 1e-10, kappa about 5e2 here)
    assert_close(to_host(u_p), ref, 1e-10)
    for u in (u_cg, u_j):
        assert_close(to_host(u), ref, 1e-8)
    it = (res_p[0]["iterations"], res_j[0]["iterations"], res_cg[0]["iterations"])
    assert it[0] <= 3 < it[1] < it[2], it
    plan.set_preconditioner("pinv")
    u_p2, _, _, rc = plan.solve(to_dev(eta), tol=1e-10)
    assert rc == 0 and np.array_equal(to_host(u_p2), to_host(u_p))
