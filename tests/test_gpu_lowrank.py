"""The 2D low-Kronecker-rank preconditioner (Sec. 4.3.2) on the device
against the oracle's sum of Kronecker pairs, and PCG with it."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_close, grid_dims, to_dev, to_host
from oracle.lowrank import lowrank_apply, lowrank_init

pytestmark = pytest.mark.gpu

PREC_TOL = {"f64": 1e-12, "f32": 2e-4, "bf16x6": 2e-4, "i8x7": 1e-12, "i8x6": 1e-12}


def _plan(shape, bcs, prec="f64", max_batch=1):
    from paper_2501_03377_amd import Plan
    nx, ny, nz = grid_dims(shape)
    return Plan(nx, ny, nz, bcs, prec=prec, max_batch=max_batch)


@pytest.mark.parametrize("shape,bcs,rank,prec", [((40, 64), ("D", "N"), 1, "f64"),
                                                 ((40, 64), ("D", "N"), 3, "f64"),
                                                 ((100, 50), ("N", "P"), 3, "f64"),
                                                 ((120, 40), ("DN", "P"), 16, "f64"),
                                                 ((70, 36), ("P", "ND"), 2, "f32"),
                                                 ((64, 64), ("D", "D"), 3, "bf16x6"),
                                                 # the int8 split carries the G_r table too
                                                 ((48, 64), ("D", "N"), 3, "i8x7"),
                                                 ((80, 32), ("N", "P"), 5, "i8x7"),
                                                 # the table on a split axis (K > 256)
                                                 ((320, 32), ("D", "N"), 3, "i8x7"),
                                                 ((48, 64), ("D", "N"), 3, "i8x6"),
                                                 ((320, 32), ("D", "N"), 3, "i8x6")])
def test_apply_parity(shape, bcs, rank, prec):
    rng = np.random.default_rng(90)
    batch = 2
    r = rng.standard_normal((batch,) + shape)
    plan = _plan(shape, bcs, prec=prec, max_batch=batch)
    plan.set_preconditioner("lowrank", rank)
    z = to_host(plan.apply_preconditioner(to_dev(r)))
    pairs = lowrank_init(shape[::-1], bcs, rank)
    for b in range(batch):
        ref = lowrank_apply(r[b].T, pairs).T
        assert_close(z[b], ref, PREC_TOL[prec], b)


def test_full_rank_is_the_pseudoinverse():
    shape, bcs = (9, 12), ("DN", "D")
    r = np.random.default_rng(91).standard_normal(shape)
    plan = _plan(shape, bcs)
    z_pinv = to_host(plan.apply_preconditioner(to_dev(r)))
    plan.set_preconditioner("lowrank", 9)
    z_lr = to_host(plan.apply_preconditioner(to_dev(r)))
    assert_close(z_lr, z_pinv, 1e-13)
    plan.set_preconditioner("pinv")
    assert np.array_equal(to_host(plan.apply_preconditioner(to_dev(r))), z_pinv)


def test_solves_rank_as_in_experiment_5_5():
    from paper_2501_03377_amd import KP_FLAG_NO_PRECOND
    shape, bcs = (64, 64), ("D", "D")
    eta = synth.gaussian_blobs_2d(64, 64, 16, 2.0, seed=1)
    ref = oracle.min_norm_solution(eta.T, bcs)[0].T
    plan = _plan(shape, bcs)
    its = {}
    for name, setup, flags in [("pinv", ("pinv",), 0), ("lowrank", ("lowrank", 3), 0),
                               ("jacobi", ("jacobi", 3, 1.3), 0), ("cg", ("pinv",), KP_FLAG_NO_PRECOND)]:
        plan.set_preconditioner(*setup)
        u, res, _, rc = plan.solve(to_dev(eta), tol=1e-10, max_iter=2000, flags=flags)
        assert rc == 0, name
        assert_close(to_host(u), ref, 1e-8, name)
        its[name] = res[0]["iterations"]
    assert its["pinv"] <= 3 < its["lowrank"] < its["jacobi"] < its["cg"], its


def test_rejections():
    from paper_2501_03377_amd import KpError
    with pytest.raises(KpError):
        _plan((8, 8, 8), ("D", "D", "D")).set_preconditioner("lowrank", 2)   # 3D
    plan = _plan((10, 12), ("D", "N"))
    for rank in (0, 11, 17):
        with pytest.raises(KpError):
            plan.set_preconditioner("lowrank", rank)
