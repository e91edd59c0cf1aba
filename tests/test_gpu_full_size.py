"""Full-size configurations, in the launch configurations the bench times:
the 64 batched problems, the 32-C regularisation path and the full-size
served requests, each against the FP64 oracle's result stored in
tests/golden/ (written by tests/golden/make_goldens.py, which runs only the
oracle): the same trajectory (outer iterations, bundles, line-search steps
and failures, nonzeros swept) and F within 1e-6 relative.

A trajectory may differ from the oracle's only where rounding decides it:
either one of its decisions sat at the rounding floor (an Armijo or
stopping test within 1e-9 of its threshold on the scale of its rounding
errors, in the oracle's run or the GPU's), or the oracle's own trajectory
changes when C moves by one or two units in the last place (the stored
`ulp_runs`: the solve amplifies rounding, as the squared-hinge solves at
eps = 1e-4 do over their 100-300 outer iterations).  Such a flip is
reported, and F must then lie within 1e-6 relative or within twice the
spread of F over the oracle's own ulp-moved runs, whichever is larger.

The stopping rule and the objective are also recomputed in FP64 from X
with scipy.sparse at the returned w: an evaluation independent of the
oracle and of the GPU's retained quantities.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.special

import synth

from tests.test_gpu_batch import _assert_same_run, pc  # noqa: F401

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
RTOL = 1e-6
FLOOR = 1e-9
COUNTS = ("outer_iters", "converged", "bundles", "ls_steps", "ls_fail", "nnz_swept")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)["records"]


def _data_sha(d):
    import hashlib
    h = hashlib.sha256()
    for a in (d.col_ptr, d.row_idx, d.val, d.y):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


def _margin(x):
    return np.inf if x is None else x


def _assert_golden(tag, info, rec):
    """The GPU solve against the oracle's stored result (see the module
    docstring for when a different trajectory is accepted)."""
    same = all(info[k] == rec[k] for k in COUNTS)
    rel = abs(info["objective"] - rec["objective"]) / abs(rec["objective"])
    if same:
        assert rel <= RTOL, (tag, info["objective"], rec["objective"])
        return rel
    floor = min(_margin(rec["min_armijo_margin"]), _margin(rec["min_stop_margin"]),
                info["min_armijo_margin"], info["min_stop_margin"])
    ulp = rec.get("ulp_runs", [])
    moved = [u for u in ulp if any(u[k] != rec[k] for k in COUNTS)]
    spread = max([abs(u["objective"] - rec["objective"]) / abs(rec["objective"]) for u in ulp],
                 default=0.0)
    report = (f"ROUNDING-FLIP {tag}: gpu " + ", ".join(f"{k}={info[k]}" for k in COUNTS) +
              " oracle " + ", ".join(f"{k}={rec[k]}" for k in COUNTS) +
              f"; smallest decision margin {floor:.3g}; {len(moved)} of {len(ulp)} ulp-moved "
              f"oracle runs change trajectory (F spread {spread:.2e}); F rel {rel:.2e}")
    print(report, flush=True)
    assert floor < FLOOR or moved, (report, "the flip is not explained by rounding")
    assert rel <= max(RTOL, 2.0 * spread), (report, "F outside the oracle's rounding spread")
    return rel
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
    p up to 100,000) in one pcdn_solve_batch call with P = 5% of the
    features: every job against the oracle's stored result, and the stopping
    rule and F recomputed from X."""
    recs = _golden("c4b_batched_problems.json")
    data = synth.c4b(scale=1.0)
    assert len(recs) == len(data) == 64 and sum(d.nnz for d in data) > 3e8
    for d, r in zip(data, recs):
        assert _data_sha(d) == r["sha"]
    solvers = [pc.Solver(device=0).load_data(d) for d in data]
    out = pc.solve_batch([s.job(r["C"], r["P"], r["eps"], "lr", seed=r["seed"])
                          for s, r in zip(solvers, recs)])
    for s in solvers:
        s.close()
    flips, worst = 0, 0.0
    for i, (d, b, r) in enumerate(zip(data, out, recs)):
        assert b[0] == 0
        worst = max(worst, _assert_golden(f"batched {i}", b[2], r))
        flips += any(b[2][k] != r[k] for k in COUNTS)
        _assert_properties(b[2], d, "lr", r["C"], r["eps"], b[1])
    print(f"{flips} of 64 batched problems differ from the oracle's trajectory; "
          f"largest F difference {worst:.2e} relative", flush=True)


def test_full_size_regularisation_path(pc):
    """The 32-C warm-started path on the text-like matrix (C = 2^-4 .. 2^6,
    P = 2,500, eps = 1e-4) through pcdn_solve_path: every point against the
    oracle's stored chain."""
    recs = _golden("c4a_path.json")
    d = synth.c2()
    assert _data_sha(d) == recs[0]["sha"]
    Cs = [r["C"] for r in recs]
    np.testing.assert_array_equal(Cs, synth.c4_path_Cs())
    s = pc.Solver(device=0).load_data(d)
    rc, W, infos = s.solve_path(Cs, recs[0]["P"], recs[0]["eps"], "lr", seed=recs[0]["seed"])
    s.close()
    assert rc == 0
    for k, (info, r) in enumerate(zip(infos, recs)):
        _assert_golden(f"path C={r['C']:.4g}", info, r)


def test_full_size_path_over_lanes(pc):
    """The same 32-C path over 8 contexts (pcdn_solve_path_lanes, as the
    bench times it): every point against the oracle's chain over its run."""
    recs = _golden("c4a_path_lanes.json")
    d = synth.c2()
    assert _data_sha(d) == recs[0]["sha"]
    Cs = synth.c4_path_Cs()
    np.testing.assert_array_equal([r["C"] for r in recs], Cs)
    solvers = [pc.Solver(device=0).load_data(d) for _ in range(8)]
    rc, W, infos = pc.pcdn_solve_path_lanes([s.ctx for s in solvers], Cs, recs[0]["P"],
                                            recs[0]["eps"], "lr", d.p, seed=recs[0]["seed"])
    for s in solvers:
        s.close()
    assert rc == 0
    for k, (info, r) in enumerate(zip(infos, recs)):
        _assert_golden(f"lanes path C={r['C']:.4g}", info, r)


def test_full_size_served_requests(pc):
    """Requests from the full-size serving pool (n up to 2e5, p up to 2e6,
    both losses) through the server together: each equals the request
    solved alone, the oracle's stored result, and satisfies the stopping rule
    recomputed from X."""
    recs = _golden("c5_served_requests.json")
    pool = synth.c5_pool(scale=1.0)
    srv = pc.Server(device=0)
    ids = [srv.submit(pool[r["pool_index"]][0], r["C"], r["P"], r["eps"], r["loss"],
                      seed=r["seed"]) for r in recs]
    results, steps = {}, 0
    while len(results) < len(ids):
        srv.step()
        steps += 1
        for k, rid in enumerate(ids):
            if k not in results:
                res = srv.take(rid)
                if res is not None:
                    results[k] = res
        assert steps < 20000
    srv.close()
    for k, r in enumerate(recs):
        d, loss = pool[r["pool_index"]]
        assert _data_sha(d) == r["sha"] and loss == r["loss"]
        res = results[k]
        print(f"pool {r['pool_index']} {loss} n={d.n} p={d.p} nnz={d.nnz} C={r['C']}: "
              f"status={res[0]} outer={res[2]['outer_iters']}/{r['outer_iters']}", flush=True)
        s = pc.Solver(device=0).load_data(d)
        alone = s.solve(r["C"], r["P"], r["eps"], loss, seed=r["seed"])
        s.close()
        _assert_same_run(res, alone)
        _assert_golden(f"served pool {r['pool_index']}", res[2], r)
        _assert_properties(res[2], d, loss, r["C"], r["eps"], res[1])
