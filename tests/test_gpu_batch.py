"""GPU parity of batched mixed-precision solves: 64 right-hand sides on one
128^3 all-Neumann grid with the BF16 preconditioner (the batched workload at
full shape) against the oracle, every right-hand side bitwise equal to its
single solve, and the power-of-two input scaling of the reduced-precision
products shown to be bitwise neutral."""

import numpy as np
import pytest

import synth
from gpu_util import assert_close, oracle_solve, to_dev, to_host

pytestmark = pytest.mark.gpu

NNN = ("N", "N", "N")
_CFG = {}
CHECKED = (0, 7, 13, 21, 34, 42, 55, 63)   # right-hand sides compared with the oracle


def _batch64():
    if not _CFG:
        # right-hand side b: 10^4 random-sign unit charges + N(0, 1e-3) noise,
        # zero mean, seed 3000 + b
        etas = np.stack([synth.charge_field((128, 128, 128), ncharges=10_000, seed=3000 + b)
                         for b in range(64)])
        _CFG["eta"] = etas
        _CFG["ref"] = {b: oracle_solve(etas[b], NNN) for b in CHECKED}
    return _CFG


@pytest.mark.parametrize("tiles", ["autotuned", "resident20", "resident21"])
def test_bf16_batch64_128cube_nnn(tiles):
    # flexible beta, tol 1e-10; the operator-resident tiles sweep their row
    # tiles here (64 right-hand sides: many tiles per persistent block)
    from paper_2501_03377_amd import KP_FLAG_FLEX_BETA, Plan
    d = _batch64()
    plan = Plan(128, 128, 128, NNN, prec="bf16", max_batch=64)
    if tiles == "autotuned":
        cfg = plan.autotune(batch=64, reps=2)
    else:
        cfg = [int(tiles[-2:])] * 6
        plan.tuning = cfg
    eta_d = to_dev(d["eta"])
    u, res, hist, rc = plan.solve(eta_d, tol=1e-10, max_iter=60, flags=KP_FLAG_FLEX_BETA)
    assert rc == 0, res
    uh = to_host(u)
    print(tiles, cfg, "iterations", sorted({r["iterations"] for r in res}))
    for b in CHECKED:
        e = assert_close(uh[b], d["ref"][b], 1e-10, (tiles, b))
        print(f"  rhs {b}: errors {e[0]:.2e} {e[1]:.2e}")
    for b, r in enumerate(res):
        assert r["true_rel_res"] <= 1e-10 and r["err_est"] <= 1e-10, (b, r)
        assert abs(float(uh[b].mean())) <= 1e-14 * float(np.abs(uh[b]).max()), b
    # each right-hand side alone, on the same plan and tile choices
    for b in range(64):
        u1, r1, _, rc1 = plan.solve(eta_d[b], tol=1e-10, max_iter=60, flags=KP_FLAG_FLEX_BETA)
        assert rc1 == 0
        assert np.array_equal(to_host(u1), uh[b]), (tiles, b)
        assert r1[0]["iterations"] == res[b]["iterations"], b
    plan.close()


@pytest.mark.parametrize("prec", ["bf16", "f32", "bf16x6"])
def test_input_scaling_is_bitwise_neutral(prec):
    # The preconditioner input of every right-hand side is scaled by a power
    # of two (its RMS brought to [1, 2)) and unscaled at the output.  Powers
    # of two commute with round-to-nearest and with FP32 and FP64 sums as long
    # as nothing over- or underflows, so a right-hand side multiplied by 2^k
    # must give exactly 2^k times the solution, also where unscaled BF16
    # products would overflow (k = 120) or flush to zero (k = -120).
    from paper_2501_03377_amd import KP_FLAG_FLEX_BETA, Plan
    shape = (24, 40, 48)
    eta = synth.charge_field(shape, ncharges=300, seed=31)
    fl = KP_FLAG_FLEX_BETA if prec == "bf16" else 0
    plan = Plan(48, 40, 24, ("P", "N", "DN"), prec=prec, max_batch=3)
    stack = np.stack([eta, np.ldexp(eta, 120), np.ldexp(eta, -120)])
    u, res, _, rc = plan.solve(to_dev(stack), tol=1e-10, max_iter=60, flags=fl)
    assert rc == 0, res
    uh = to_host(u)
    assert np.array_equal(uh[1], np.ldexp(uh[0], 120))
    assert np.array_equal(uh[2], np.ldexp(uh[0], -120))
    assert res[0]["iterations"] == res[1]["iterations"] == res[2]["iterations"]
    assert_close(uh[0], oracle_solve(eta, ("P", "N", "DN")), 1e-10, prec)
    plan.close()
