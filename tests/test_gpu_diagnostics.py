"""Convergence descriptors (KP_FLAG_DIAGNOSTICS, kp_plan_diagnostics)
against the oracle's definitions on the same iterate and against the
oracle's own runs."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import grid_dims, to_dev, to_host

pytestmark = pytest.mark.gpu


def _plan(shape, bcs, prec="f64", max_batch=1):
    from paper_2501_03377_amd import Plan
    nx, ny, nz = grid_dims(shape)
    return Plan(nx, ny, nz, bcs, prec=prec, max_batch=max_batch)


def _flags(*names):
    import paper_2501_03377_amd as kp
    f = kp.KP_FLAG_DIAGNOSTICS
    for n in names:
        f |= getattr(kp, n)
    return f


@pytest.mark.parametrize("bcs", [("D", "N", "DN"), ("N", "P", "N")])
def test_row_s_describes_the_returned_iterate(bcs):
    # plain CG stopped after s iterations returns U_s; row s must be the
    # oracle's descriptors of that iterate (the exit centring of a singular
    # problem changes neither kappa nor the residual, since L1 = 0 and eta_c
    # sums to zero)
    shape = (20, 24, 28)
    eta = synth.charge_field(shape, ncharges=80, seed=21)
    plan = _plan(shape, bcs)
    e = to_dev(eta)
    H = eta.T - eta.mean() if oracle.is_singular(bcs) else eta.T
    for s in (1, 4, 9):
        u, res, hist, rc = plan.solve(e, tol=1e-14, max_iter=s, flags=_flags("KP_FLAG_NO_PRECOND"),
                                      raise_on_error=False)
        assert res[0]["iterations"] == s
        d = plan.diagnostics()[0]
        true_rel, kappa, null = oracle.iterate_descriptors(to_host(u).T, H, bcs)
        assert abs(d[s, 0] - true_rel) <= 1e-12 * true_rel
        assert abs(d[s, 1] - hist[0, s]) == 0.0
        assert abs(d[s, 2] - kappa) <= 1e-12 * abs(kappa)
        if oracle.is_singular(bcs):
            # the iterate is mean-free in exact arithmetic: rounding only
            assert d[s, 4] <= 1e-12 * np.linalg.norm(to_host(u))
        else:
            assert d[s, 4] == 0.0
        assert np.isnan(d[s + 1:]).all()


@pytest.mark.parametrize("bcs,flags", [(("D", "N", "P"), ()), (("P", "N", "N"), ()),
                                       (("D", "D", "N"), ("KP_FLAG_NO_PRECOND",))])
def test_series_matches_the_oracle_run(bcs, flags):
    # FP64 runs follow the oracle's iterates up to rounding order
    shape = (16, 20, 24)
    eta = synth.charge_field(shape, ncharges=50, seed=22)
    plan = _plan(shape, bcs)
    n = 25 if flags else 2
    u, res, hist, rc = plan.solve(to_dev(eta), tol=1e-30, max_iter=n, flags=_flags(*flags),
                                  raise_on_error=False)
    d = plan.diagnostics()[0]
    M = None if flags else oracle.PinvPreconditioner(eta.T.shape, bcs)
    ref = np.array(oracle.pcg(eta.T, bcs, precond=M, fixed_iterations=res[0]["iterations"])
                   .diagnostics)
    k = len(ref)
    assert np.isfinite(d[:k]).all() and np.isnan(d[k:]).all()
    scale = abs(ref[:, 1]).max()
    tol = 1e-9 if flags else 1e-12
    assert np.allclose(d[:k, 2], ref[:, 1], rtol=0, atol=tol * scale)          # kappa
    assert np.allclose(d[:k, 5], ref[:, 3], rtol=0, atol=tol * scale)          # alpha rho
    big = ref[:, 0] > 1e-8
    assert np.allclose(d[:k, 0][big], ref[:, 0][big], rtol=1e-6 if flags else 1e-10)
    # the derived columns from their definitions
    kmin = d[:k, 2].min()
    assert np.allclose(d[:k, 3], np.sqrt(np.maximum(d[:k, 2] - kmin, 0.0)), rtol=1e-14, atol=0)
    est = np.array([np.sqrt(max(d[s + 1:min(s + 4, k - 1) + 1, 5].sum(), 0.0)) for s in range(k)])
    assert np.allclose(d[:k, 6], est, rtol=1e-14, atol=0)


def test_batched_rows_and_a_zero_rhs():
    shape, bcs = (24, 20, 16), ("N", "D", "P")
    eta = np.stack([synth.charge_field(shape, ncharges=40, seed=23),
                    np.zeros(shape),
                    synth.charge_field(shape, ncharges=5, seed=24)])
    plan = _plan(shape, bcs, max_batch=3)
    u, res, hist, rc = plan.solve(to_dev(eta), tol=1e-10, max_iter=30, flags=_flags())
    assert rc == 0
    d = plan.diagnostics(delay=2)
    for b in range(3):
        it = res[b]["iterations"]
        assert np.isfinite(d[b, :it + 1]).all() and np.isnan(d[b, it + 1:]).all()
        if b != 1:
            single = _plan(shape, bcs)
            single.solve(to_dev(eta[b]), tol=1e-10, max_iter=30, flags=_flags())
            assert np.array_equal(single.diagnostics(delay=2)[0], d[b], equal_nan=True)
    assert d[1, 0, 0] == 0.0 and d[1, 0, 2] == 0.0 and res[1]["iterations"] == 0


def test_recording_changes_nothing_and_replays_alike():
    from paper_2501_03377_amd import KpError
    shape, bcs = (32, 40, 36), ("DN", "P", "D")
    eta = synth.charge_field(shape, ncharges=100, seed=25)
    plan = _plan(shape, bcs, prec="f32")
    e = to_dev(eta)
    u0, r0, h0, _ = plan.solve(e, tol=1e-10)
    u0 = to_host(u0)
    with pytest.raises(KpError):
        plan.diagnostics()                       # that solve recorded nothing
    tables = []
    for _ in range(3):                           # first run, then whole-solve graph replays
        u1, r1, h1, _ = plan.solve(e, tol=1e-10, flags=_flags())
        assert np.array_equal(to_host(u1), u0) and np.array_equal(h1, h0)
        assert r1[0]["iterations"] == r0[0]["iterations"]
        tables.append(plan.diagnostics())
    assert all(np.array_equal(t, tables[0], equal_nan=True) for t in tables)


def test_mixed_precision_kappa_falls_by_the_hs_terms():
    # with the FP32 pseudoinverse the L-norm of the error still falls
    # monotonically, by the Hestenes-Stiefel terms up to the preconditioner's
    # rounding
    shape, bcs = (48, 64, 64), ("P", "P", "DN")
    eta = synth.charge_field(shape, ncharges=300, seed=26)
    plan = _plan(shape, bcs, prec="f32")
    u, res, hist, rc = plan.solve(to_dev(eta), tol=1e-12, flags=_flags())
    assert rc == 0
    d = plan.diagnostics()[0]
    k = res[0]["iterations"] + 1
    scale = abs(d[:k, 2]).max()
    for s in range(1, k):
        assert d[s, 2] <= d[s - 1, 2] + 1e-13 * scale
        assert abs((d[s - 1, 2] - d[s, 2]) - d[s, 5]) <= 1e-6 * scale
    assert d[k - 1, 0] <= 1e-11


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_anorm_stop_matches_the_oracle_rule(precond):
    # the device stops at the first iteration where the Hestenes-Stiefel rule
    # holds on its own terms, which is the oracle's stopping iteration, and
    # the returned iterate meets the tolerance in the L-norm
    from oracle.diagnostics import hs_stop_iteration
    from oracle.jacobi import JacobiPreconditioner
    shape, bcs = (16, 20, 24), ("D", "N", "D")
    eta = synth.charge_field(shape, ncharges=50, seed=27)
    tol = 1e-7
    plan = _plan(shape, bcs)
    extra = ("KP_FLAG_ANORM_STOP",)
    if precond == "jacobi":
        plan.set_preconditioner("jacobi", 3, 1.3)
        M = JacobiPreconditioner(eta.T.shape, bcs, 3, 1.3)
    else:
        extra += ("KP_FLAG_NO_PRECOND",)
        M = None
    u, res, hist, rc = plan.solve(to_dev(eta), tol=tol, max_iter=400, flags=_flags(*extra))
    assert rc == 0
    s = res[0]["iterations"]
    d = plan.diagnostics()[0]
    assert hs_stop_iteration(d[:, 5], tol) == s
    ref = oracle.pcg(eta.T, bcs, precond=M, max_iter=400, stall=10**6, true_tol=0.0)
    t = np.array(ref.diagnostics)[:, 3]
    assert hs_stop_iteration(t, tol) == s
    ustar = oracle.min_norm_solution(eta.T, bcs)[0]
    e = to_host(u).T - ustar
    lnorm = lambda x: np.sqrt(np.sum(x * oracle.apply_minus_laplacian(x, bcs)))
    assert lnorm(e) <= tol * lnorm(ustar)
