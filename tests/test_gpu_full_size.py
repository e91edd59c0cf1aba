"""Full-size configurations, in the launch configurations the bench times,
checked where the oracle cannot follow every problem in seconds.

The checks recompute the stopping rule and the objective in FP64 from X
with scipy.sparse at the returned w: an evaluation independent of the
oracle and of the GPU's retained quantities (a property that holds at any
size).  Where a problem is small enough, the oracle is run too.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.special

import oracle
import synth

from tests.test_gpu_batch import _assert_oracle, _assert_same_run, pc  # noqa: F401

pytestmark = pytest.mark.gpu


def _np_check(d, loss, C, w):
    """(F(w), ||grad^S F(w)||_1, ||grad^S F(0)||_1) for eq. (1) in FP64 from X."""
    X = sp.csc_matrix((d.val.astype(np.float64), d.row_idx, d.col_ptr), shape=(d.n, d.p))
    y = d.y.astype(np.float64)
    z = X @ w
    if loss == "lr":
        F = np.abs(w).sum() + C * np.logaddexp(0.0, -y * z).sum()
        g = -C * (X.T @ (y * scipy.special.expit(-y * z)))
        g0 = -0.5 * C * (X.T @ y)
    else:
        b = 1.0 - y * z
        F = np.abs(w).sum() + C * np.sum(np.where(b > 0, b * b, 0.0))
        g = -2.0 * C * (X.T @ (y * np.where(b > 0, b, 0.0)))
        g0 = -2.0 * C * (X.T @ y)
    sub = np.where(w > 0, g + 1.0, np.where(w < 0, g - 1.0,
                                             np.sign(g) * np.maximum(np.abs(g) - 1.0, 0.0)))
    G = np.abs(sub).sum()
    G0 = np.maximum(np.abs(g0) - 1.0, 0.0).sum()
    return float(F), float(G), float(G0)


def _assert_properties(info, d, loss, C, eps, w):
    F, G, G0 = _np_check(d, loss, C, w)
    assert info["objective"] == pytest.approx(F, rel=1e-9)
    assert info["subgrad0"] == pytest.approx(G0, rel=1e-9)
    # the GPU's norm (from its retained quantities) against the recomputed one
    assert abs(info["subgrad"] - G) <= 1e-6 * G0
    if info["converged"]:
        assert G <= eps * G0 * (1.0 + 1e-6) + 1e-6 * G0


def test_full_size_batched_problems(pc):
    """The 64 batched independent LR problems (334M nonzeros, n up to 20,000,
    p up to 100,000) in one pcdn_solve_batch call with P = 5% of the features:
    every result satisfies the stopping rule and reports F(w); the three
    smallest also give the oracle's trajectory."""
    data = synth.c4b(scale=1.0)
    assert sum(d.nnz for d in data) > 3e8
    solvers = [pc.Solver(device=0).load_data(d) for d in data]
    Ps = [max(1, int(np.floor(0.05 * d.p + 0.5))) for d in data]
    out = pc.solve_batch([s.job(1.0, P, 1e-4, "lr", seed=7) for s, P in zip(solvers, Ps)])
    for s in solvers:
        s.close()
    for d, b in zip(data, out):
        _assert_properties(b[2], d, "lr", 1.0, 1e-4, b[1])
    assert all(b[0] == 0 for b in out)
    for i in sorted(range(len(data)), key=lambda i: data[i].nnz)[:3]:
        d = data[i]
        w_o, io, _ = oracle.solve(oracle.Problem.from_data(d), oracle.Params(loss="lr", C=1.0),
                                  P=Ps[i], eps=1e-4, seed=7)
        _assert_oracle(out[i], (w_o, io), True)


def test_full_size_served_requests(pc):
    """Requests from the full-size serving pool (n up to 2e5, p up to 2e6,
    both losses) through the server together: each equals the request
    solved alone and satisfies the stopping rule recomputed from X."""
    pool = synth.c5_pool(scale=1.0)
    picks = [(0, 1.0), (15, 0.5), (3, 2.0), (12, 0.3), (1, 1.0)]  # LR 4.6M, LR 6.2M, LR, SVM, SVM
    eps = {"lr": 1e-4, "svm": 1e-3}
    srv = pc.Server(device=0)
    ids = [srv.submit(pool[i][0], C, 0, eps[pool[i][1]], pool[i][1], seed=3) for i, C in picks]
    results, steps = {}, 0
    while len(results) < len(ids):
        srv.step()
        steps += 1
        for k, rid in enumerate(ids):
            if k not in results:
                r = srv.take(rid)
                if r is not None:
                    results[k] = r
        assert steps < 20000
    srv.close()
    results = [results[k] for k in range(len(ids))]
    for (i, C), res in zip(picks, results):
        d, loss = pool[i]
        print(f"pool {i} {loss} n={d.n} p={d.p} nnz={d.nnz} C={C}: status={res[0]} "
              f"outer={res[2]['outer_iters']}", flush=True)
        s = pc.Solver(device=0).load_data(d)
        alone = s.solve(C, max(1, int(np.floor(0.05 * d.p + 0.5))), eps[loss], loss, seed=3)
        s.close()
        _assert_same_run(res, alone)
        _assert_properties(res[2], d, loss, C, eps[loss], res[1])
