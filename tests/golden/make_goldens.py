"""Write the FP64 oracle's results for the full-size batched, path and served
configurations into tests/golden/*.json.

    python tests/golden/make_goldens.py [--jobs 7] [--only c4b|path|lanes|c5]

Only the oracle (oracle/) and the seeded input generators (synth/) run here;
nothing reads the GPU library.  Each record holds the inputs' checksum, the
solve's settings and the oracle's result: trajectory counts, F, the stopping
norm and reference, and how close its Armijo and stopping decisions came to
their thresholds.  The GPU tests (tests/test_gpu_full_size.py) compare with
these records.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

# the settings the GPU tests use
C4B_SEED, C4B_EPS, C4B_C = 7, 1e-4, 1.0
PATH_SEED, PATH_EPS, PATH_P = 1, 1e-4, 2500
C5_SEED = 3
C5_EPS = {"lr": 1e-4, "svm": 1e-4}  # the serving configuration: eps = 1e-4
# (pool index, C): the full-size served requests of the GPU test
C5_PICKS = [(0, 1.0), (15, 0.5), (3, 2.0), (12, 0.3), (1, 1.0), (6, 0.5), (11, 0.2), (13, 1.0)]
COUNTS = ("outer_iters", "converged", "bundles", "ls_steps", "ls_fail", "nnz_swept")
FIELDS = ("outer_iters", "converged", "bundles", "ls_steps", "ls_fail", "nnz_swept", "objective",
          "subgrad", "subgrad0", "min_armijo_margin", "min_stop_margin")


def data_sha(d) -> str:
    h = hashlib.sha256()
    for a in (d.col_ptr, d.row_idx, d.val, d.y):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


def five_percent(p: int) -> int:
    """The bundle size the tests use: 5% of the features (the paper's starting
    point for its bundle-size search), at least 1."""
    return max(1, int(np.floor(0.05 * p + 0.5)))


def _record(d, loss, C, P, eps, seed, info) -> dict:
    r = {"n": d.n, "p": d.p, "nnz": d.nnz, "sha": data_sha(d), "loss": loss, "C": C, "P": P,
         "eps": eps, "seed": seed}
    for f in FIELDS:
        v = info[f]
        r[f] = None if isinstance(v, float) and not np.isfinite(v) else v
    return r


def _c4b_one(i: int) -> dict:
    d = synth.c4b_problem(i)
    P = five_percent(d.p)
    t0 = time.time()
    _, info, _ = oracle.solve(oracle.Problem.from_data(d), oracle.Params(loss="lr", C=C4B_C),
                              P=P, eps=C4B_EPS, seed=C4B_SEED)
    r = _record(d, "lr", C4B_C, P, C4B_EPS, C4B_SEED, info)
    r["index"] = i
    print(f"c4b {i}: n={d.n} p={d.p} nnz={d.nnz} outer={info['outer_iters']} "
          f"{time.time() - t0:.1f}s", flush=True)
    return r


# C moved by one and two units in the last place either way: solves whose
# arithmetic differs from the unperturbed one only at the rounding level
ULP_STEPS = (1, -1, 2, -2)


def _ulp_moved(C: float, k: int) -> float:
    for _ in range(abs(k)):
        C = float(np.nextafter(C, np.inf if k > 0 else 0.0))
    return C


def _c5_one(task) -> dict:
    """One served request (task = (pick, ulp step)): the solve at the pick's C,
    or at C moved by the step."""
    k, step = task
    i, C = C5_PICKS[k]
    d, loss = synth.c5_pool(scale=1.0)[i]
    P = five_percent(d.p)
    Cr = _ulp_moved(C, step)
    t0 = time.time()
    _, info, _ = oracle.solve(oracle.Problem.from_data(d), oracle.Params(loss=loss, C=Cr), P=P,
                              eps=C5_EPS[loss], seed=C5_SEED)
    r = _record(d, loss, Cr, P, C5_EPS[loss], C5_SEED, info)
    r["pool_index"] = i
    print(f"c5 pool {i} {loss} C={C} ulp {step:+d}: nnz={d.nnz} outer={info['outer_iters']} "
          f"{time.time() - t0:.1f}s", flush=True)
    return r


def _c5_records(pool) -> list:
    """The served requests, each with the oracle's runs at C moved by a few
    ulps (`ulp_runs`: their trajectory counts and F), which show whether the
    trajectory at this eps is decided by rounding."""
    tasks = [(k, step) for k in range(len(C5_PICKS)) for step in (0,) + ULP_STEPS]
    # longest (most nonzeros) first
    nnz = [synth.c5_pool(scale=1.0)[i][0].nnz for i, _ in C5_PICKS]
    tasks.sort(key=lambda t: -nnz[t[0]])
    runs = dict(zip(tasks, pool.map(_c5_one, tasks, chunksize=1)))
    recs = []
    for k in range(len(C5_PICKS)):
        r = runs[(k, 0)]
        r["ulp_runs"] = [{"ulp": s, "C": runs[(k, s)]["C"],
                          **{f: runs[(k, s)][f] for f in COUNTS + ("objective",)}}
                         for s in ULP_STEPS]
        recs.append(r)
    return recs


def _path() -> list:
    d = synth.c2()
    prob = oracle.Problem.from_data(d)
    out, w = [], None
    for C in synth.c4_path_Cs():
        t0 = time.time()
        w, info, _ = oracle.solve(prob, oracle.Params(loss="lr", C=float(C)), P=PATH_P,
                                  eps=PATH_EPS, seed=PATH_SEED, w0=w)
        out.append(_record(d, "lr", float(C), PATH_P, PATH_EPS, PATH_SEED, info))
        print(f"path C={C:.4g}: outer={info['outer_iters']} {time.time() - t0:.1f}s", flush=True)
    return out


PATH_LANES = 8


def _lane_runs(count: int, lanes: int) -> list:
    """The contiguous runs pcdn_solve_path_lanes cuts count C values into."""
    L = min(lanes, count)
    first = [(i * count) // L for i in range(L + 1)]
    return [(first[i], first[i + 1]) for i in range(L)]


def _path_run(run) -> list:
    """One run of the path over lanes: a warm-started chain from w = 0."""
    lo, hi = run
    d = synth.c2()
    prob = oracle.Problem.from_data(d)
    Cs = synth.c4_path_Cs()
    out, w = [], None
    for k in range(lo, hi):
        w, info, _ = oracle.solve(prob, oracle.Params(loss="lr", C=float(Cs[k])), P=PATH_P,
                                  eps=PATH_EPS, seed=PATH_SEED, w0=w)
        r = _record(d, "lr", float(Cs[k]), PATH_P, PATH_EPS, PATH_SEED, info)
        r["lane_run"] = [lo, hi]
        out.append(r)
        print(f"path lanes run {lo}-{hi} C={Cs[k]:.4g}: outer={info['outer_iters']}", flush=True)
    return out


def _write(name: str, payload) -> None:
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(payload, f, indent=1)
        f.write("\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    ap.add_argument("--only", choices=("c4b", "path", "lanes", "c5"), action="append")
    args = ap.parse_args()
    todo = args.only or ["c5", "path", "lanes", "c4b"]
    oracle.build()
    with mp.get_context("fork").Pool(args.jobs) as pool:
        if "c5" in todo:
            recs = _c5_records(pool)
            _write("c5_served_requests.json", {"note": "oracle results of the full-size served "
                                               "requests (pool index, C; P = 5% of p), each "
                                               "with the oracle's runs at C moved by 1 and 2 "
                                               "ulps either way", "records": recs})
        if "c4b" in todo:
            n = len(synth.c4b_shapes(scale=1.0))
            # largest first, so that the long ones start early
            order = sorted(range(n), key=lambda i: -np.prod(synth.c4b_shapes(scale=1.0)[i]))
            recs = sorted(pool.map(_c4b_one, order, chunksize=1), key=lambda r: r["index"])
            _write("c4b_batched_problems.json", {"note": "oracle results of the 64 batched LR "
                                                 "problems (P = 5% of p)", "records": recs})
        if "lanes" in todo:
            runs = _lane_runs(len(synth.c4_path_Cs()), PATH_LANES)
            recs = [r for chunk in pool.map(_path_run, runs, chunksize=1) for r in chunk]
            _write("c4a_path_lanes.json", {"note": "oracle results of the 32-C path cut into "
                                           f"{PATH_LANES} warm-started runs (each run's first C "
                                           "from w = 0)", "records": recs})
    if "path" in todo:
        _write("c4a_path.json", {"note": "oracle results of the 32-C warm-started path on the "
                                 "text-like matrix", "records": _path()})


if __name__ == "__main__":
    main()
