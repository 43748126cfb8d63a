"""The request server (kp_server_*): results against the oracle, bitwise
equality of batched and solo solves, HBM admission with eviction, and
rejection of requests the budget cannot hold."""

import numpy as np
import pytest

import synth
from gpu_util import assert_close, oracle_solve, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


def _drain(srv, n, timeout=60.0):
    import time
    done, t0 = {}, time.time()
    while len(done) < n:
        for c in srv.poll(max_n=64, timeout=0.5):
            done[c["id"]] = c
        assert time.time() - t0 < timeout, f"only {len(done)} of {n} completions"
    return done


def test_server_results_match_oracle():
    import torch
    from paper_2501_03377_amd import Server
    cases = [((12, 20, 24), ("P", "P", "DN"), "f64", 1e-10, "dev"),
             ((16, 18, 20), ("N", "N", "N"), "f32", 1e-10, "host"),
             ((20, 16), ("D", "N"), "f64", 1e-12, "dev"),
             ((10, 12, 14), ("D", "ND", "P"), "bf16", 1e-8, "host"),
             ((24, 24, 24), ("DN", "D", "N"), "f32", 1e-8, "dev")]
    srv = Server(hbm_budget=0, workers=2, max_batch=4)
    try:
        outs, etas = {}, {}
        for k, (shape, bcs, prec, tol, where) in enumerate(cases):
            eta = synth.charge_field(shape, ncharges=50, seed=900 + k)
            etas[k] = eta
            if where == "dev":
                e, u = to_dev(eta), torch.empty(shape, dtype=torch.float64, device="cuda")
            else:
                e, u = eta, np.empty(shape)
            outs[k] = u
            srv.submit(k, e, bcs, tol=tol, prec=prec, u=u,
                       flags=2 if prec == "bf16" else 0)   # flexible beta for BF16
        done = _drain(srv, len(cases))
        for k, (shape, bcs, prec, tol, where) in enumerate(cases):
            c = done[k]
            assert c["status"] == 0, c
            u = to_host(outs[k]) if where == "dev" else outs[k]
            assert_close(u, oracle_solve(etas[k], bcs), 1e-10 if prec == "f64" else tol, (k, c))
            assert c["t_submit"] <= c["t_start"] <= c["t_end"]
        st = srv.stats()
        assert st["completed"] == len(cases) and st["plans_created"] == len(cases)
    finally:
        srv.close()


def test_server_batches_match_solo_bitwise():
    # one worker, requests queued while it is busy: they are solved in
    # batches; the same requests solved one at a time give identical bits
    import torch
    from paper_2501_03377_amd import Server
    shape, bcs = (16, 20, 24), ("P", "N", "D")
    etas = [synth.charge_field(shape, ncharges=80, seed=1200 + k) for k in range(7)]

    def run(together):
        srv = Server(hbm_budget=0, workers=1, max_batch=4)
        us, batches = [], []
        try:
            for k, eta in enumerate(etas):
                u = torch.empty(shape, dtype=torch.float64, device="cuda")
                us.append(u)
                srv.submit(k, to_dev(eta), bcs, tol=1e-10, prec="f32", u=u)
                if not together:
                    batches.append(_drain(srv, 1)[k]["batch"])
            if together:
                batches = [c["batch"] for c in _drain(srv, len(etas)).values()]
            return [to_host(u) for u in us], batches
        finally:
            srv.close()

    mixed, b_mixed = run(True)
    solo, b_solo = run(False)
    assert max(b_mixed) > 1 and max(b_solo) == 1
    for a, b in zip(mixed, solo):
        assert np.array_equal(a, b)


def test_server_evicts_idle_plans_and_rejects_oversize():
    from paper_2501_03377_amd import Server
    from paper_2501_03377_amd import Plan
    shape = (24, 24, 24)
    probe = Plan(24, 24, 24, ("P", "P", "P"), prec="f32", max_batch=2)
    resident = probe.resident_bytes
    one = resident + probe.workspace_bytes + 2 * 2 * 8 * 24 ** 3
    probe.close()
    # the worker's workspace and staging plus one plan's operators fit, a
    # second plan's operators do not
    srv = Server(hbm_budget=one + resident // 2, workers=1, max_batch=2)
    try:
        keys = [("P", "P", "P"), ("D", "D", "D"), ("N", "N", "N"), ("P", "P", "P")]
        for k, bcs in enumerate(keys):
            srv.submit(k, synth.charge_field(shape, ncharges=40, seed=1300 + k), bcs, tol=1e-8)
            c = _drain(srv, 1)[k]
            assert c["status"] == 0, c
        st = srv.stats()
        assert st["plans_evicted"] >= 3 and st["plans_cached"] == 1
        assert st["hbm_high_water"] <= st["hbm_budget"]
        # a grid whose plan alone exceeds the budget completes with KP_ENOMEM
        srv.submit(99, synth.charge_field((96, 96, 96), ncharges=40, seed=1399), ("P",) * 3)
        c = _drain(srv, 1)[99]
        assert c["status"] == -2 and srv.stats()["rejected"] == 1
    finally:
        srv.close()


@pytest.mark.parametrize("prec", ["i8x7", "i8x6"])
def test_server_int8_split_requests(prec):
    # int8 split requests are served like the others, in one iteration, and
    # match the oracle; a grid the int8 split cannot take (an axis not a
    # multiple of 16) is refused at submission, before any work is queued
    from paper_2501_03377_amd import Server
    from paper_2501_03377_amd.kpcg import KpError
    srv = Server(hbm_budget=0, workers=2, max_batch=4)
    try:
        cases = [((32, 32, 48), ("P", "P", "DN")), ((16, 32, 32), ("N", "N", "N")),
                 ((48, 64), ("D", "N"))]
        etas, outs = {}, {}
        for k, (shape, bcs) in enumerate(cases):
            etas[k] = synth.charge_field(shape, ncharges=60, seed=1500 + k)
            outs[k] = np.empty(shape)
            srv.submit(k, etas[k], bcs, tol=1e-10, prec=prec, u=outs[k])
        with pytest.raises(KpError):
            srv.submit(99, synth.charge_field((20, 32, 32), ncharges=10, seed=1599),
                       ("P", "P", "D"), prec=prec)
        done = _drain(srv, len(cases))
        for k, (shape, bcs) in enumerate(cases):
            c = done[k]
            assert c["status"] == 0 and c["iterations"] == 1, c
            assert_close(outs[k], oracle_solve(etas[k], bcs), 1e-10, (k, c))
        assert srv.stats()["completed"] == len(cases)
    finally:
        srv.close()


def test_requests_join_a_running_batch_and_leave_on_their_own():
    # continuous batching: plain CG (hundreds of iterations); requests of the
    # same kind submitted while the first is being solved take free slots at
    # the next iteration boundary, before the first has finished, and each
    # leaves when its own solve ends.  Every result is bitwise that of the
    # same request alone and matches the oracle.
    import time
    import torch
    from paper_2501_03377_amd import KP_FLAG_NO_PRECOND, Server
    shape, bcs = (32, 32, 32), ("D", "N", "D")
    etas = [synth.charge_field(shape, ncharges=60, seed=1700 + k) for k in range(3)]
    kw = dict(tol=1e-12, prec="f64", flags=KP_FLAG_NO_PRECOND, max_iter=3000)
    srv = Server(hbm_budget=0, workers=1, max_batch=4)
    try:
        us = [torch.empty(shape, dtype=torch.float64, device="cuda") for _ in range(3)]
        srv.submit(0, to_dev(etas[0]), bcs, u=us[0], **kw)
        time.sleep(0.005)
        for k in (1, 2):
            srv.submit(k, to_dev(etas[k]), bcs, u=us[k], **kw)
        done = _drain(srv, 3)
        first = done[0]
        assert first["status"] == 0 and first["iterations"] > 100, first
        for k in (1, 2):
            c = done[k]
            assert c["status"] == 0, c
            assert c["worker"] == first["worker"]
            assert first["t_start"] < c["t_start"] < first["t_end"], (first, c)
        assert max(c["batch"] for c in done.values()) >= 2
        mix = [to_host(u) for u in us]
        for k in range(3):
            u = torch.empty(shape, dtype=torch.float64, device="cuda")
            srv.submit(10 + k, to_dev(etas[k]), bcs, u=u, **kw)
            c = _drain(srv, 1)[10 + k]
            assert c["batch"] == 1 and c["iterations"] == done[k]["iterations"], (c, done[k])
            assert np.array_equal(to_host(u), mix[k]), k
            # stopped on the residual alone (1e-12), kappa about 10^3
            assert_close(mix[k], oracle_solve(etas[k], bcs), 1e-8, k)
    finally:
        srv.close()


def test_two_workers_mixed_plans_alone_equals_mix():
    # two workers serve three kinds of request (grid, boundary conditions,
    # precision) at once, each in its own continuous batch; every result is
    # bitwise that of the same request served alone, and within its
    # tolerance of the oracle
    import torch
    from paper_2501_03377_amd import KP_FLAG_FLEX_BETA, Server
    kinds = [((32, 32, 48), ("P", "P", "DN"), "i8x7", 0, 1e-10),
             ((20, 24, 28), ("N", "N", "N"), "bf16", KP_FLAG_FLEX_BETA, 1e-10),
             ((16, 20, 24), ("D", "P", "N"), "f64", 0, 1e-10),
             ((24, 24, 24), ("DN", "D", "P"), "f32", 0, 1e-8),
             ((16, 32, 32), ("N", "D", "P"), "i8x6", 0, 1e-10)]
    reqs = [(k % len(kinds), 1800 + k) for k in range(16)]
    # every input is on the device before the first submission, so that the
    # requests queue up together.  Plans belong to a worker, and making one
    # (and capturing its first graph) holds a lock that the other worker's
    # set-up needs too, so on a cold server one worker may still be setting
    # up while the other finishes its short solves: the mix is served again,
    # on warm plans, until two kinds have run at the same time (at most three
    # rounds).  Every round's results are checked.
    etas, devs = {}, {}
    for rid, (kind, seed) in enumerate(reqs):
        etas[rid] = synth.charge_field(kinds[kind][0], ncharges=100, seed=seed)
        devs[rid] = to_dev(etas[rid])
    torch.cuda.synchronize()
    srv = Server(hbm_budget=0, workers=2, max_batch=3)
    try:
        mixes, overlap = [], False
        for rnd in range(3):
            outs = {rid: torch.empty(kinds[kind][0], dtype=torch.float64, device="cuda")
                    for rid, (kind, _) in enumerate(reqs)}
            for rid, (kind, seed) in enumerate(reqs):
                shape, bcs, prec, fl, tol = kinds[kind]
                srv.submit(100 * rnd + rid, devs[rid], bcs, tol=tol, prec=prec, flags=fl,
                           u=outs[rid])
            got = _drain(srv, len(reqs))
            done = {c - 100 * rnd: v for c, v in got.items()}
            assert all(c["status"] == 0 for c in done.values()), done
            mixes.append(({rid: to_host(u) for rid, u in outs.items()}, done))
            # some requests of different kinds ran at the same time on the two workers
            ivs = [(c["t_start"], c["t_end"], c["worker"], reqs[i][0]) for i, c in done.items()]
            if any(a[2] != b[2] and a[3] != b[3] and a[0] < b[1] and b[0] < a[1]
                   for a in ivs for b in ivs):
                overlap = True
                break
        assert overlap, "no two kinds ran at the same time in three rounds"
        assert len({c["worker"] for _, d in mixes for c in d.values()}) == 2
        for rid, (kind, seed) in enumerate(reqs):
            shape, bcs, prec, fl, tol = kinds[kind]
            u = torch.empty(shape, dtype=torch.float64, device="cuda")
            srv.submit(1000 + rid, devs[rid], bcs, tol=tol, prec=prec, flags=fl, u=u)
            c = _drain(srv, 1)[1000 + rid]
            alone = to_host(u)
            for mix, done in mixes:
                assert c["batch"] == 1 and c["iterations"] == done[rid]["iterations"]
                assert np.array_equal(alone, mix[rid]), (rid, prec)
            assert_close(alone, oracle_solve(etas[rid], bcs), tol, (rid, prec))
    finally:
        srv.close()


def test_step_length_does_not_change_results():
    # a continuous batch steps one iteration at a time while a request of its
    # kind waits for a slot (here max_batch = 1 with two queued behind the
    # first), and up to four at a time otherwise (the last request, and every
    # request served alone): plain CG, tens of iterations, bitwise equal
    # either way; an iteration cap that is not a multiple of four is met
    # exactly
    import torch
    from paper_2501_03377_amd import KP_FLAG_NO_PRECOND, KP_NOT_CONVERGED, Server
    shape, bcs = (16, 20, 24), ("D", "N", "P")
    etas = [synth.charge_field(shape, ncharges=50, seed=1900 + k) for k in range(3)]
    kw = dict(tol=1e-10, prec="f64", flags=KP_FLAG_NO_PRECOND, max_iter=500)
    srv = Server(hbm_budget=0, workers=1, max_batch=1)
    try:
        outs = [torch.empty(shape, dtype=torch.float64, device="cuda") for _ in range(3)]
        for k in range(3):
            srv.submit(k, to_dev(etas[k]), bcs, u=outs[k], **kw)
        done = _drain(srv, 3)
        assert all(c["status"] == 0 and c["iterations"] > 20 for c in done.values()), done
        for k in range(3):
            u = torch.empty(shape, dtype=torch.float64, device="cuda")
            srv.submit(10 + k, to_dev(etas[k]), bcs, u=u, **kw)
            c = _drain(srv, 1)[10 + k]
            assert c["iterations"] == done[k]["iterations"], (c, done[k])
            assert np.array_equal(to_host(u), to_host(outs[k])), k
        u = torch.empty(shape, dtype=torch.float64, device="cuda")
        srv.submit(99, to_dev(etas[0]), bcs, u=u, **dict(kw, max_iter=7))
        c = _drain(srv, 1)[99]
        assert c["status"] == KP_NOT_CONVERGED and c["iterations"] == 7, c
    finally:
        srv.close()
