"""GPU parity of the FP64-accurate preconditioners on the int8 matrix cores
(I8X7: every value cut into seven truncated 7-bit digits, 28 exact digit
products; I8X6: six balanced base-256 digits, 21 products): the application
against the oracle's pseudoinverse (Algs. 6-7), and whole solves
(Algorithm 1) against the converged oracle solution."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_close, grid_dims, oracle_pinv, oracle_solve, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

# the FP64 preconditioner's bound in the other parity tests
PINV_TOL = 1e-12
INT8 = ["i8x7", "i8x6"]


def _plan(shape, bcs, prec="i8x7", max_batch=1):
    from paper_2501_03377_amd import Plan
    nx, ny, nz = grid_dims(shape)
    return Plan(nx, ny, nz, bcs, prec=prec, max_batch=max_batch)


@pytest.mark.parametrize("shape,bcs", [
    ((16, 16, 16), ("N", "N", "N")),      # one k-block of 64, 16 of it used
    ((32, 48, 80), ("P", "DN", "ND")),    # 80: a partial second k-block
    ((48, 64, 192), ("D", "P", "N")),     # 192: three k-blocks per wave
    ((16, 32, 512), ("P", "P", "D")),     # 512: k split over two waves
    ((16, 48, 320), ("N", "D", "DN")),    # 320: split, padded k-blocks
    ((320, 16, 32), ("D", "N", "P")),     # the Hadamard product on a split axis
    ((384, 32, 16), ("D", "N", "D")),     # split, three k-blocks per wave
    ((64, 80), ("P", "N")),               # 2D; 80 rows: a ragged row tile
    ((16, 16), ("D", "D")),
])
@pytest.mark.parametrize("prec", INT8)
def test_int8_pinv_parity(shape, bcs, prec):
    rng = np.random.default_rng(40)
    r = rng.standard_normal(shape)
    plan = _plan(shape, bcs, prec=prec)
    z = to_host(plan.apply_pinv(to_dev(r)))
    plan.close()
    err = assert_close(z, oracle_pinv(r, bcs), PINV_TOL, (shape, bcs))
    print(f"pinv {prec} {shape} {bcs}: rel err (2-norm, max) {err[0]:.3e} {err[1]:.3e}")


@pytest.mark.parametrize("prec", INT8)
def test_int8_pinv_small_eigenvalue(prec):
    # (P, N, D) with a long Dirichlet axis: the smallest eigenvalue sum is
    # the Dirichlet axis's own smallest eigenvalue, 6.7e-5 at n = 384, and the
    # output is dominated by its mode.  LAPACK's eigenvalues (the oracle's)
    # are backward stable, |d lambda| <= c eps ||L|| with ||L|| <= 4, so the
    # oracle's 1/lambda there is good to about 4 eps / lambda_min relative
    # (observed 2.9e-12 against the closed form 4 sin^2); the device's closed
    # forms do not have that error.  Parity with the oracle is asserted
    # within its own bound, and the int8 split agrees with the FP64 matrix
    # cores (the same closed-form eigenvalues) to 1e-12.
    shape, bcs = (384, 32, 16), ("P", "N", "D")
    r = np.random.default_rng(40).standard_normal(shape)
    _, lam, _ = oracle.pinv_init(r.T.shape, bcs)
    mu_min = lam[2][0]                      # lambda_x(0) = lambda_y(0) = 0
    z = {}
    for p in (prec, "f64"):
        plan = _plan(shape, bcs, prec=p)
        z[p] = to_host(plan.apply_pinv(to_dev(r)))
        plan.close()
    ref = oracle_pinv(r, bcs)
    bound = PINV_TOL + 12 * np.finfo(float).eps / mu_min
    for p in z:
        assert_close(z[p], ref, bound, p)
    assert_close(z[prec], z["f64"], PINV_TOL)


@pytest.mark.parametrize("prec", INT8)
def test_int8_is_as_accurate_as_fp64(prec):
    # the splits keep 47 to 49 bits of every row and column: their error to
    # the exact pseudoinverse is within a small factor of the FP64 matrix
    # cores'
    shape, bcs = (32, 64, 128), ("P", "P", "DN")
    rng = np.random.default_rng(41)
    r = rng.standard_normal(shape)
    ref = oracle_pinv(r, bcs)
    err = {}
    for p in ("f64", prec, "f32"):
        plan = _plan(shape, bcs, prec=p)
        err[p] = rel(to_host(plan.apply_pinv(to_dev(r))), ref)
        plan.close()
    print("pinv errors", err)
    assert err[prec] <= 10 * err["f64"] + 1e-14, err
    assert err[prec] * 1e6 <= err["f32"], err


# (the long axis is not the only nonsingular one: see the small-eigenvalue test)
@pytest.mark.parametrize("shape,bcs", [((16, 32, 64), ("D", "N", "P")),
                                       ((16, 16, 384), ("N", "D", "P"))])
@pytest.mark.parametrize("prec", INT8)
def test_int8_rows_of_any_magnitude(shape, bcs, prec):
    # every row gets its own power of two: right-hand sides from 1e-200 to
    # 1e200, and rows of one dominant entry, keep their relative accuracy;
    # each right-hand side of a batch equals its single application exactly
    rng = np.random.default_rng(42)
    r = rng.standard_normal((3,) + shape)
    r[0] *= 1e-200
    r[2] *= 1e200
    r[1, :, :, 5] *= 1e9
    plan = _plan(shape, bcs, prec=prec, max_batch=3)
    zb = to_host(plan.apply_pinv(to_dev(r)))
    for b in range(3):
        z1 = to_host(plan.apply_pinv(to_dev(r[b])))
        assert np.array_equal(zb[b], z1), b
        s = 1e200 if b == 0 else (1e-200 if b == 2 else 1.0)
        assert_close(zb[b] * s, oracle_pinv(r[b] * s, bcs), PINV_TOL, b)
    plan.close()


@pytest.mark.parametrize("shape", [(16, 16, 32), (16, 16, 320), (320, 16, 16)])
@pytest.mark.parametrize("prec", INT8)
def test_int8_nonfinite_input_gives_nonfinite_output(shape, prec):
    # a NaN in R reaches every output, as in FP64 arithmetic (the solver's
    # non-finite checks rely on it)
    bcs = ("P", "D", "N")
    r = np.random.default_rng(43).standard_normal(shape)
    r[3, 4, 5] = np.nan
    plan = _plan(shape, bcs, prec=prec)
    z = to_host(plan.apply_pinv(to_dev(r)))
    plan.close()
    assert np.isnan(z).all()


@pytest.mark.parametrize("shape,bcs", [
    ((32, 64, 128), ("P", "P", "DN")),
    ((48, 48, 48), ("N", "N", "N")),
    ((64, 32, 96), ("P", "P", "D")),
    ((64, 96), ("D", "N")),
])
@pytest.mark.parametrize("prec", INT8)
def test_int8_solve_one_iteration(shape, bcs, prec):
    # as with the FP64 pseudoinverse, one iteration reaches tol 1e-10
    from paper_2501_03377_amd import Plan
    eta = synth.charge_field(shape, ncharges=2000, seed=9)
    nx, ny, nz = grid_dims(shape)
    plan = Plan(nx, ny, nz, bcs, prec=prec)
    u, res, hist, rc = plan.solve(to_dev(eta), tol=1e-10, raise_on_error=False)
    u = to_host(u)
    plan.close()
    err = rel(u, oracle_solve(eta, bcs))
    print(f"{prec} {shape} {bcs}: iters {res[0]['iterations']} err {err:.3e} "
          f"rel_res {res[0]['rel_res']:.3e} true {res[0]['true_rel_res']:.3e}")
    assert rc == 0, res
    assert res[0]["iterations"] == 1, res
    assert_close(u, oracle_solve(eta, bcs), 1e-10, (shape, bcs))
    assert res[0]["true_rel_res"] <= 1e-10


@pytest.mark.parametrize("prec", INT8)
def test_int8_batch_solve_and_replay(prec):
    # a batch of 4 all-Neumann right-hand sides: each equals its single solve
    # bitwise, a repeated solve (graph replay) is bitwise identical, and all
    # match the oracle
    from paper_2501_03377_amd import Plan
    shape, bcs = (32, 32, 64), ("N", "N", "N")
    eta = np.stack([synth.charge_field(shape, ncharges=1000, seed=20 + b) for b in range(4)])
    plan = Plan(64, 32, 32, bcs, prec=prec, max_batch=4)
    ub, res, _, rc = plan.solve(to_dev(eta), tol=1e-10, raise_on_error=False)
    ub = to_host(ub)
    assert rc == 0, res
    ub2 = to_host(plan.solve(to_dev(eta), tol=1e-10)[0])
    assert np.array_equal(ub, ub2)
    for b in range(4):
        u1 = to_host(plan.solve(to_dev(eta[b]), tol=1e-10)[0])
        assert np.array_equal(ub[b], u1), b
        assert_close(ub[b], oracle_solve(eta[b], bcs), 1e-10, b)
    plan.close()


@pytest.mark.parametrize("shape,bcs", [
    ((48, 64, 192), ("D", "P", "N")),     # the first product on 192 (K <= 256 kernel)
    ((64, 32, 512), ("P", "P", "D")),     # the first product on 512 (split kernel)
    ((64, 80), ("P", "D")),               # 2D, a ragged row tile
])
@pytest.mark.parametrize("prec", INT8)
def test_int8_norm_from_first_product(shape, bcs, prec):
    # A nonsingular solve from U_0 = 0 takes ||eta||^2 from the first
    # preconditioner product, which reads eta; with KP_FLAG_DIAGNOSTICS it
    # comes from a pass of its own.  Only the rounding of that sum may differ:
    # the same u, bit for bit, and residuals relative to ||eta|| equal to
    # about the sum's rounding.
    from paper_2501_03377_amd.kpcg import KP_FLAG_DIAGNOSTICS
    eta = np.stack([synth.charge_field(shape, ncharges=800, seed=14),
                    np.zeros(shape)])
    plan = _plan(shape, bcs, prec=prec, max_batch=2)
    out = []
    for flags in (0, KP_FLAG_DIAGNOSTICS, 0):
        u, res, hist, rc = plan.solve(to_dev(eta), tol=1e-10, max_iter=20, flags=flags,
                                      raise_on_error=False)
        assert rc == 0, res
        out.append((to_host(u), res, hist))
    plan.close()
    (u0, r0, h0), (u1, r1, h1), (u2, r2, _) = out
    assert np.array_equal(u0, u1) and np.array_equal(u0, u2)
    assert np.array_equal(u0[1], np.zeros(shape)) and r0[1]["iterations"] == 0
    assert r0[0]["iterations"] == r1[0]["iterations"] >= 1
    assert h0[0, 0] == 1.0
    for key in ("rel_res", "true_rel_res"):
        assert abs(r0[0][key] - r1[0][key]) <= 1e-13 * r1[0][key], (key, r0[0], r1[0])
        assert r0[0][key] == r2[0][key]
