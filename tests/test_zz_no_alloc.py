"""The allocation-free pseudoinverse entry point, kp_apply_pinv_noalloc, through
the C ABI: the same output as kp_apply_pinv (same kernels) on two calls in a
row, the second with a smaller input, in every precision; the oracle's
pseudoinverse to each precision's bound; and an input beyond the static
scratch refused before any work."""

import numpy as np
import pytest

from gpu_util import oracle_pinv, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

# relative error of one application against the exact L^+ (as the pinv parity
# tests use)
PINV_TOL = {"f64": 1e-12, "f32": 2e-4, "bf16": 5e-2, "i8x7": 1e-12, "i8x6": 1e-12}


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "i8x7", "i8x6"])
def test_noalloc_pinv_matches_apply_pinv(prec):
    import torch
    from paper_2501_03377_amd import Plan, kpcg
    cases = [((64, 96, 128), ("P", "N", "DN"), 2),    # (nz, ny, nx), batch: the larger input
             ((32, 48, 16), ("D", "P", "N"), 1)]      # then a smaller one
    for k, (shape, bcs, batch) in enumerate(cases):
        nz, ny, nx = shape
        plan = Plan(nx, ny, nz, bcs, prec=prec, max_batch=batch)
        r = np.random.default_rng(60 + k).standard_normal((batch,) + shape)
        R = to_dev(r)
        Z = torch.full_like(R, float("nan"))
        print(f"kp_apply_pinv_noalloc {prec} {shape} batch {batch}", flush=True)
        rc = kpcg.kp_apply_pinv_noalloc(plan._h, R.data_ptr(), Z.data_ptr(), batch)
        assert rc == kpcg.KP_OK, kpcg.kp_strerror(rc)
        torch.cuda.synchronize()
        got = to_host(Z)
        ref = to_host(plan.apply_pinv(R))
        torch.cuda.synchronize()
        assert np.array_equal(got, ref), (prec, shape)
        for b in range(batch):
            assert rel(got[b], oracle_pinv(r[b], bcs)) <= PINV_TOL[prec], (prec, shape, b)
        plan.close()


def test_noalloc_pinv_refuses_inputs_beyond_the_scratch():
    import torch
    from paper_2501_03377_amd import Plan, kpcg
    # 256 x 256 x 128 in FP64: two intermediate grids of 64 MiB each, twice
    # what the static scratch holds
    plan = Plan(256, 256, 128, ("P", "P", "DN"), prec="f64")
    R = torch.zeros((128, 256, 256), dtype=torch.float64, device="cuda")
    Z = torch.full_like(R, 7.0)
    rc = kpcg.kp_apply_pinv_noalloc(plan._h, R.data_ptr(), Z.data_ptr(), 1)
    assert rc == kpcg.KP_ENOMEM
    assert "scratch" in kpcg.kp_last_error()
    torch.cuda.synchronize()
    assert bool((Z == 7.0).all())
    plan.close()
