"""The solve server (continuous batching) through the C ABI: requests that
arrive while others run are admitted as device memory frees up, and each
result is the same as the request solved alone (pcdn_solve on its own
context) and as the FP64 oracle's, within the parity bar."""
import numpy as np
import pytest

import oracle
import synth

from tests.test_gpu_batch import RTOL, _assert_oracle, _assert_same_run, pc  # noqa: F401

pytestmark = pytest.mark.gpu


def _requests():
    """(data, loss, C, P, eps) of a mixed stream: both losses, both
    schedules, uneven sizes."""
    c1 = synth.c1()
    return [
        (c1, "lr", 1.0, 32, 1e-4),
        (synth.bernoulli_csc(41, 1500, 4000, 0.01), "lr", 0.5, 800, 1e-4),
        (synth.sparse_random(42, 900, 2500, 0.004, binary=True), "svm", 0.3, 125, 1e-3),
        (c1, "svm", 2.0, 100, 1e-4),
        (synth.bernoulli_csc(43, 300, 9000, 0.02), "lr", 4.0, 0, 1e-4),
        (synth.tiny(44, n=40, p=12, density=0.4), "lr", 1.0, 3, 1e-6),
        (synth.bernoulli_csc(45, 2500, 1200, 0.015), "svm", 1.0, 240, 1e-4),
        (synth.bernoulli_csc(46, 700, 20000, 0.003), "lr", 2.0, 4000, 1e-4),
    ]


def _alone(pc, d, loss, C, P, eps, seed):
    s = pc.Solver(device=0).load_data(d)
    out = s.solve(C, P, eps, loss, seed=seed)
    s.close()
    return out


def _staggered(pc, srv, reqs, seed):
    """Submit the requests a few at a time with steps in between (later
    requests arrive while earlier ones run); return id -> result."""
    ids, results = [], {}
    pending = list(enumerate(reqs))
    steps = 0
    while pending or len(results) < len(reqs):
        for _ in range(2):
            if pending:
                i, (d, loss, C, P, eps) = pending.pop(0)
                ids.append((i, srv.submit(d, C, P, eps, loss, seed=seed)))
        srv.step()
        steps += 1
        for i, rid in ids:
            if i not in results:
                r = srv.take(rid)
                if r is not None:
                    results[i] = r
                    if r[0] < 0:
                        print(f"request {i} failed: {srv.last_error()}", flush=True)
        assert steps < 5000
    return results


def test_server_same_alone_and_in_mix(pc):
    reqs = _requests()
    srv = pc.Server(device=0, budget_bytes=8 << 30)
    results = _staggered(pc, srv, reqs, seed=7)
    for i, (d, loss, C, P, eps) in enumerate(reqs):
        Pe = P if P else max(1, int(np.floor(0.05 * d.p + 0.5)))
        alone = _alone(pc, d, loss, C, Pe, eps, seed=7)
        print(f"request {i}: status {results[i][0]} outer {results[i][2]['outer_iters']} "
              f"F {results[i][2]['objective']:.15g}", flush=True)
        _assert_same_run(results[i], alone)
        if d.nnz <= 200000:
            w_o, io, _ = oracle.solve(oracle.Problem.from_data(d), oracle.Params(loss=loss, C=C),
                                      P=Pe, eps=eps, seed=7)
            _assert_oracle(results[i], (w_o, io), d.p > 20)
    assert srv.status() == (0, 0, 0)
    srv.close()


def test_server_admission_by_footprint(pc):
    """A budget that holds about two of these problems: the queue drains in
    order, never more state is admitted than fits, and every result still
    equals its solve alone."""
    data = [synth.bernoulli_csc(60 + i, 2000, 6000, 0.01) for i in range(6)]
    srv = pc.Server(device=0, budget_bytes=1 << 40)
    one = None
    # measure one request's footprint through the status call
    rid = srv.submit(data[0], 1.0, 300, 1e-4, "lr", seed=3)
    srv.step()
    one = srv.status()[2]
    while srv.take(rid) is None:
        srv.step()
    srv.close()
    assert one > 0
    srv = pc.Server(device=0, budget_bytes=int(2.5 * one))
    ids = [srv.submit(d, 1.0, 300, 1e-4, "lr", seed=3) for d in data]
    res, peak = {}, 0
    while len(res) < len(ids):
        srv.step()
        waiting, running, used = srv.status()
        assert used <= int(2.5 * one) and running <= 2
        peak = max(peak, running)
        for k, rid in enumerate(ids):
            if k not in res:
                r = srv.take(rid)
                if r is not None:
                    res[k] = r
    assert peak == 2
    for k, d in enumerate(data):
        _assert_same_run(res[k], _alone(pc, d, "lr", 1.0, 300, 1e-4, seed=3))
    srv.close()


def test_server_errors(pc):
    from paper_1306_4080_amd import PcdnError
    d = synth.c1()
    srv = pc.Server(device=0, budget_bytes=1 << 30)
    with pytest.raises(PcdnError, match="E_ARG"):
        srv.submit(d, -1.0, 32, 1e-4, "lr")
    with pytest.raises(PcdnError, match="E_ARG"):
        srv.submit(d, 1.0, d.p + 1, 1e-4, "lr")
    tiny_srv = pc.Server(device=0, budget_bytes=1 << 20)
    with pytest.raises(PcdnError, match="E_OOM"):
        tiny_srv.submit(d, 1.0, 32, 1e-4, "lr")
    tiny_srv.close()
    # a request whose data fails the CSC checks finishes with that error
    bad = synth.Data(n=d.n, p=d.p, col_ptr=d.col_ptr, row_idx=d.row_idx.copy(), val=d.val, y=d.y)
    bad.row_idx[0] = d.n
    rid_bad = srv.submit(bad, 1.0, 32, 1e-4, "lr")
    rid_ok = srv.submit(d, 1.0, 32, 1e-4, "lr")
    assert srv.take(rid_ok) is None                 # not finished yet
    while True:
        srv.step()
        r = srv.take(rid_bad)
        if r is not None:
            break
    assert r[0] == -2                                # PCDN_E_CSC
    while srv.take(rid_ok) is None:
        srv.step()
    with pytest.raises(PcdnError, match="E_ARG"):
        srv.take(12345)
    srv.close()
