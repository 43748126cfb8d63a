"""GPU parity of the individual operators against the oracle: the minus
Laplacian of eq. (3.2) and the pseudoinverse preconditioner of Algs. 6-7."""

import itertools

import numpy as np
import pytest

import oracle
from gpu_util import (assert_close, grid_dims, oracle_laplacian, oracle_pinv, rel, to_dev,
                      to_host)

pytestmark = pytest.mark.gpu

ALL3 = list(itertools.product(oracle.BCS, repeat=3))
ALL2 = list(itertools.product(oracle.BCS, repeat=2))


def _plan(shape, bcs, prec="f64", max_batch=1):
    from paper_2501_03377_amd import Plan
    nx, ny, nz = grid_dims(shape)
    return Plan(nx, ny, nz, bcs, prec=prec, max_batch=max_batch)


def test_stencil_all_bc_triples_exact_on_integers():
    # integer data: the stencil has integer coefficients, so results are exact
    import torch
    rng = np.random.default_rng(0)
    shape = (5, 6, 7)
    p = rng.integers(-50, 50, size=shape).astype(np.float64)
    for bcs in ALL3:
        plan = _plan(shape, bcs)
        w = to_host(plan.apply_laplacian(to_dev(p)))
        torch.cuda.synchronize()
        assert np.array_equal(w, oracle_laplacian(p, bcs)), bcs
        plan.close()


def test_stencil_all_bc_pairs_2d():
    import torch
    rng = np.random.default_rng(1)
    shape = (9, 13)
    p = rng.integers(-50, 50, size=shape).astype(np.float64)
    for bcs in ALL2:
        plan = _plan(shape, bcs)
        w = to_host(plan.apply_laplacian(to_dev(p)))
        torch.cuda.synchronize()
        assert np.array_equal(w, oracle_laplacian(p, bcs)), bcs


@pytest.mark.parametrize("shape,bcs", [((33, 67, 130), ("P", "P", "DN")),
                                       ((128, 256, 256), ("P", "P", "DN"))])
def test_stencil_random_large(shape, bcs):
    rng = np.random.default_rng(2)
    p = rng.standard_normal(shape)
    plan = _plan(shape, bcs, max_batch=2)
    w = to_host(plan.apply_laplacian(to_dev(np.stack([p, 2 * p]))))
    ref = oracle_laplacian(p, bcs)
    assert np.max(np.abs(w[0] - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.max(np.abs(w[1] - 2 * ref)) <= 2e-13 * np.max(np.abs(ref))


PINV_TOL = {"f64": 1e-12, "f32": 2e-4, "bf16": 5e-2, "bf16x6": 2e-4}
PRECS = ["f64", "f32", "bf16", "bf16x6"]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape,bcs", [
    ((5, 4, 3), ("D", "N", "P")),
    ((7, 70, 67), ("P", "DN", "ND")),
    ((33, 65, 130), ("P", "P", "DN")),
    ((20, 17), ("D", "D")),
    ((64, 64), ("P", "N")),
])
def test_pinv_parity(shape, bcs, prec):
    rng = np.random.default_rng(3)
    r = rng.standard_normal(shape)
    plan = _plan(shape, bcs, prec=prec)
    z = to_host(plan.apply_pinv(to_dev(r)))
    ref = oracle_pinv(r, bcs)
    err = assert_close(z, ref, PINV_TOL[prec])
    print(f"pinv {prec} {shape} {bcs}: rel err (2-norm, max) {err[0]:.3e} {err[1]:.3e}")


@pytest.mark.parametrize("prec", PRECS)
def test_pinv_all_bc_triples_small(prec):
    rng = np.random.default_rng(4)
    shape = (4, 5, 6)
    r = rng.standard_normal(shape)
    for bcs in ALL3:
        plan = _plan(shape, bcs, prec=prec)
        z = to_host(plan.apply_pinv(to_dev(r)))
        assert_close(z, oracle_pinv(r, bcs), PINV_TOL[prec], bcs)
        plan.close()


@pytest.mark.parametrize("shape,bcs", [((33, 65, 130), ("P", "P", "DN")), ((64, 64), ("P", "N")),
                                       ((40, 48, 64), ("N", "D", "P"))])
def test_bf16x6_is_as_accurate_as_fp32(shape, bcs):
    # three-term BF16 splits on the BF16 matrix cores reach FP32 accuracy: the
    # error to the exact pseudoinverse is within a small factor of the FP32
    # matrix-core result's and far below the plain BF16 one's
    rng = np.random.default_rng(31)
    r = rng.standard_normal(shape)
    ref = oracle_pinv(r, bcs)
    err = {}
    for prec in ("f32", "bf16x6", "bf16"):
        plan = _plan(shape, bcs, prec=prec)
        err[prec] = rel(to_host(plan.apply_pinv(to_dev(r))), ref)
        plan.close()
    print("pinv errors", err)
    assert err["bf16x6"] <= 4 * err["f32"] + 1e-12, err
    assert err["bf16x6"] * 100 <= err["bf16"], err


def test_pinv_batch_matches_single():
    import torch
    rng = np.random.default_rng(5)
    shape = (12, 40, 33)
    r = rng.standard_normal((3,) + shape)
    plan = _plan(shape, ("P", "D", "N"), prec="f64", max_batch=3)
    zb = to_host(plan.apply_pinv(to_dev(r)))
    for b in range(3):
        z1 = to_host(plan.apply_pinv(to_dev(r[b])))
        assert np.array_equal(zb[b], z1)


# tile configurations compiled per precision (the others would spill)
# 20 and 21: the operator-resident tiles (contractions of at most 128)
TILE_CONFIGS = {"f64": [c for c in range(22) if c not in (3, 7, 11, 15, 16, 17)],
                "f32": list(range(22)),
                "bf16": [c for c in range(22) if c != 16],
                "bf16x6": [c for c in range(22) if c not in (3, 7, 11, 15, 16, 17)]}


@pytest.mark.parametrize("shape", [(20, 36, 70), (24, 40, 72)])
@pytest.mark.parametrize("prec", PRECS)
def test_tile_shapes_are_bitwise_identical(prec, shape):
    # every tile shape sums over k in the same order, so the result does not
    # depend on the autotuner's choice; (20, 36, 70) has rows too ragged for
    # 16-byte loads, (24, 40, 72) takes the vector path with ragged k-blocks
    from paper_2501_03377_amd.kpcg import kp_plan_set_tuning
    rng = np.random.default_rng(6)
    r = to_dev(rng.standard_normal((2,) + shape))
    plan = _plan(shape, ("P", "D", "N"), prec=prec, max_batch=2)
    ref = to_host(plan.apply_pinv(r))
    rh = to_host(r)
    for b in range(2):
        assert_close(ref[b], oracle_pinv(rh[b], ("P", "D", "N")), PINV_TOL[prec], b)
    for cfg in range(23):
        rc = kp_plan_set_tuning(plan._h, [cfg] * 6)
        if cfg not in TILE_CONFIGS[prec]:
            assert rc != 0, cfg
            continue
        assert rc == 0, cfg
        z = to_host(plan.apply_pinv(r))
        assert np.array_equal(z, ref), cfg


def test_autotune_keeps_results():
    rng = np.random.default_rng(8)
    shape = (16, 48, 96)
    r = rng.standard_normal(shape)
    plan = _plan(shape, ("P", "P", "DN"), prec="f32")
    before = to_host(plan.apply_pinv(to_dev(r)))
    cfg = plan.autotune(batch=1, reps=2)
    assert len(cfg) == 6
    after = to_host(plan.apply_pinv(to_dev(r)))
    assert np.array_equal(before, after)
    assert_close(after, oracle_pinv(r, ("P", "P", "DN")), PINV_TOL["f32"])


@pytest.mark.parametrize("shape,bcs,prec", [((16, 48, 96), ("P", "P", "DN"), "f32"),
                                            ((40, 64), ("N", "D"), "bf16")])
def test_kernel_timing_call(shape, bcs, prec):
    # every supported class times, unsupported ones are rejected, and the
    # call leaves the caller's buffers and later solves untouched
    from paper_2501_03377_amd import KpError, KP_FLAG_FLEX_BETA
    from paper_2501_03377_amd.kpcg import KERNEL_CLASSES, kp_kernel_class_name
    import synth
    eta = synth.charge_field(shape, ncharges=30, seed=9)
    plan = _plan(shape, bcs, prec=prec, max_batch=2)
    e = to_dev(eta)
    flags = KP_FLAG_FLEX_BETA if prec == "bf16" else 0
    u1, _, _, rc = plan.solve(e, tol=1e-10, flags=flags)
    assert rc == 0
    u1 = to_host(u1)
    dim = len(shape)
    timed = set()
    for c in range(KERNEL_CLASSES):
        name = kp_kernel_class_name(c)
        ok = (name.startswith("modeprod") and (dim == 3 or "_z_" not in name)) or \
            name in ("stencil_dot", "update_ur", "dot_rz", "update_p")
        if ok:
            ms = plan.time_kernel(c, batch=2, flags=flags, reps=3)
            assert 0.0 < ms < 100.0, (name, ms)
            timed.add(name)
        else:
            with pytest.raises(KpError):
                plan.time_kernel(c, batch=1, reps=1)
    assert len(timed) == 2 * dim + 4
    with pytest.raises(KpError):
        plan.time_kernel("update_ur", batch=3)          # beyond max_batch
    with pytest.raises(KpError):
        plan.time_kernel("update_ur", flags=1)          # only the flexible-beta flag
    assert np.array_equal(to_host(e), eta)
    u2, _, _, rc = plan.solve(e, tol=1e-10, flags=flags)
    assert rc == 0 and np.array_equal(to_host(u2), u1)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_resident_tiles_only_for_short_contractions(prec):
    # the operator-resident tiles hold a 128 x 128 operator at most: refused
    # for a product along a longer axis, accepted (and bitwise the same as the
    # default tiles) where every axis fits, including a batch
    from paper_2501_03377_amd.kpcg import kp_plan_set_tuning
    plan = _plan((16, 24, 160), ("P", "D", "N"), prec=prec)
    assert kp_plan_set_tuning(plan._h, [20] * 6) != 0
    plan.close()
    rng = np.random.default_rng(22)
    shape = (32, 64, 128)
    r = to_dev(rng.standard_normal((3,) + shape))
    plan = _plan(shape, ("N", "DN", "P"), prec=prec, max_batch=3)
    ref = to_host(plan.apply_pinv(r))
    for cfg in (20, 21):
        assert kp_plan_set_tuning(plan._h, [cfg] * 6) == 0
        assert np.array_equal(to_host(plan.apply_pinv(r)), ref), cfg
    plan.close()
