#!/usr/bin/env python3
"""PCDN bundle-sweep benchmark on one MI355X.

Workload (the headline): the huge sparse binary L1-regularised L2-loss SVM
problem (n = 100,000 samples, p = 1,000,000 features, ~12M binary fp32
nonzeros, ~120 per row, Zipf(1.05) column frequencies with columns capped at
50,000 nonzeros), C = 1, bundle size P = 16,384; synthetic, seeded, generated
in-process.  It is the largest configuration that the method's benchmark
set runs on one GPU.

A step is one pass of the whole hot path: one outer iteration of Algorithm 3
(seeded partition, every bundle's gradient/Hessian sweep, direction, d^T x,
line search and apply, then the full-gradient stopping test), continuing the
trajectory from w = 0 (the warmup steps are the first iterations).  value =
bundle-sweep nonzeros processed per second over the timed steps (nnz(X) per
step), with X resident in HBM before timing.

Region A (value) replays the captured outer iteration on the library's
stream.  Region B runs the next steps of the same solve with every kernel
launch bracketed by HIP events on that stream (direct launches, same kernels
and launch shapes); the roofline object reports the kernel class with the
most time there (algorithmic bytes per launch / average launch duration),
beside a device-to-device copy measured in the same process.
The FP64 CPU oracle is timed on a bounded sample of the same workload.

More objects on the same line:
- "text_like": the text-like L1-LR problem (20,000 x 50,000, ~1.6M nonzeros)
  at its six settings C in {0.5, 4} x P in {64, 1024, 8192}, one outer
  iteration of each per step, run concurrently through pcdn_iterate_batch
  and one after another;
- "batched" (skipped with --no-batched): 64 independent LR problems (n
  U[500,20000], p U[1000,100000], density U[0.001,0.02]) solved to
  eps = 1e-4 one pcdn_solve after another and in one pcdn_solve_batch call
  (bundle size, schedule and range width from the autotuner, tuned before
  timing);
- "path": 32 C values on the text-like matrix with warm starts,
  pcdn_solve_path against the same chain of pcdn_solve calls, against the
  32 solves one at a time from w = 0, and the path cut into 8 warm-started
  runs advanced together (pcdn_solve_path_lanes, every solve to the same
  stopping rule);
- "serving" (skipped with --no-serving): a Poisson stream of mixed LR/SVM
  solves through the solve server against one solve after another.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "bundle-sweep nnz/s (HBM GB/s %peak); batched solves/s + p99 latency vs plain"
HBM_PEAK_GBS = 8000.0
KERNEL_CLASSES = ("sweep", "sweep_finish", "dtx_linesearch", "apply", "stopping_sweep", "narrow")
KERNEL_NAMES = ("k_sweep_ranges (gradient/Hessian sweep and direction over the bundle's "
                "nonzeros in partition order, 256 per wavefront)",
                "k_sweep_finish (slots crossing a range boundary, and empty slots)",
                "k_rows_dtx (d^T x by row and the first line-search candidates)",
                "k_rows_apply (Armijo decision, w and retained-quantity update)",
                "k_stop_tiles+k_stop_finish (full-gradient subgradient norm)",
                "k_narrow (one workgroup runs every bundle of an outer iteration)")
C3 = dict(C=1.0, P=16384, eps=1e-3, loss="svm")
SETTINGS = [(0.5, 64), (0.5, 1024), (0.5, 8192), (4.0, 64), (4.0, 1024), (4.0, 8192)]
SEED = 1
PATH_LANES = 8


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time budget of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-text-like", action="store_true",
                    help="skip the text-like six-setting measurement")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-mebibyte device buffer three times (the plain copy "
                         "kernel that scales the rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-solve and regularisation-path measurements")
    ap.add_argument("--batched-scale", type=float, default=1.0,
                    help="shrink n and p of the 64 batched problems (1.0: full size)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--serving-scale", type=float, default=1.0,
                    help="shrink the served problems' n and p ranges (1.0: full size)")
    ap.add_argument("--serving-requests", type=int, default=500)
    ap.add_argument("--source-hash", action="store_true",
                    help="print the hash of the kernel sources that traffic records are keyed by")
    return ap.parse_args()


def copy_calibration(mib: int) -> None:
    import torch
    nbytes = mib << 20
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copies": 3}),
          flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("pcdn_kernels.hip", "pcdn_device.h"):
        with open(os.path.join(ROOT, "paper_1306_4080_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_class: str):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel_class}_c3_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(d, budget_s: float) -> dict:
    """The FP64 oracle on a bounded sample of the headline workload: the
    first outer iterations of the solve from w = 0, as many as fit the
    budget (one probe iteration sets the count).  `value` is its multicore
    build (OpenMP over the features of a bundle and over the samples of the
    line search and update, the loops the paper runs in parallel; the d^T x
    scatter stays serial) on every host core the process may use; the
    single-threaded parity build is reported beside it on half the budget."""
    import oracle
    prob = oracle.Problem.from_data(d)
    par = oracle.Params(loss=C3["loss"], C=C3["C"])
    want = int(os.environ.get("OMP_NUM_THREADS") or 0) or len(os.sched_getaffinity(0))
    cores = oracle.threads_available(want)

    def timed(budget, threads):
        t0 = time.perf_counter()
        oracle.solve(prob, par, P=C3["P"], eps=0.0, seed=SEED, max_outer=1, threads=threads)
        probe = time.perf_counter() - t0
        m = max(1, int(budget / max(probe, 1e-3)))
        t0 = time.perf_counter()
        _, info, _ = oracle.solve(prob, par, P=C3["P"], eps=0.0, seed=SEED, max_outer=m,
                                  threads=threads)
        return m, info["nnz_swept"], time.perf_counter() - t0

    m, nz, dt = timed(0.5 * budget_s, cores)
    m1, nz1, dt1 = timed(0.5 * budget_s, 0)
    return {"value": nz / dt, "unit": "nnz/s", "cores": cores, "kind": "oracle",
            "sample": f"first {m} outer iterations of the solve from w = 0 ({nz} bundle "
                      f"nonzeros, {dt:.1f} s) with the OpenMP build on {cores} threads",
            "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(),
            "single_thread": {"value": nz1 / dt1, "unit": "nnz/s", "cores": 1,
                              "sample": f"first {m1} outer iterations ({nz1} bundle nonzeros, "
                                        f"{dt1:.1f} s)"}}


def _chosen_pilot(t: dict) -> dict:
    """The autotuner's pilot that ran with the chosen configuration."""
    for x in t["tried"]:
        if (x["P"], x["schedule"], x["chunk"]) == (t["P"], t["schedule"], t["chunk"]):
            return x
    return {"narrow": 0}


def batched_measurement(pc, synth, scale: float) -> dict:
    """64 independent LR problems (C = 1, eps = 1e-4), bundle size, schedule
    and range width (pcdn_opts.chunk) from the autotuner (not timed): one pcdn_solve after
    another ("plain") against one pcdn_solve_batch call; both give the same
    results."""
    import torch
    data = synth.c4b(scale=scale)
    solvers = [pc.Solver(device=0).load_data(d) for d in data]
    t0 = time.perf_counter()
    tunes = [s.autotune(1.0, 1e-4, "lr", seed=SEED) for s in solvers]
    t_tune = time.perf_counter() - t0
    # the tuned bundle size, schedule and range width of each problem
    cfg = [dict(P=t["P"], schedule=t["schedule"], chunk=t["chunk"]) for t in tunes]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [s.solve(1.0, c["P"], 1e-4, "lr", seed=SEED, schedule=c["schedule"], chunk=c["chunk"])
             for s, c in zip(solvers, cfg)]
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    batch = pc.solve_batch([s.job(1.0, c["P"], 1e-4, "lr", seed=SEED, schedule=c["schedule"],
                                  chunk=c["chunk"]) for s, c in zip(solvers, cfg)])
    t_batch = time.perf_counter() - t0
    same = all(a[2]["outer_iters"] == b[2]["outer_iters"] and
               abs(a[2]["objective"] - b[2]["objective"]) <= 1e-12 * abs(a[2]["objective"])
               for a, b in zip(plain, batch))
    nnz_swept = sum(b[2]["nnz_swept"] for b in batch)
    for s in solvers:
        s.close()
    n = len(data)
    return {"workload": f"{n} independent L1-LR problems, n U[500,20000], p U[1000,100000], "
                        f"density U[0.001,0.02] (scale {scale}), C=1, eps=1e-4, "
                        "autotuned P, schedule and chunk",
            "nnz_total": int(sum(d.nnz for d in data)),
            "plain_solves_per_s": n / t_plain, "batched_solves_per_s": n / t_batch,
            "speedup": t_plain / t_batch, "plain_s": t_plain, "batched_s": t_batch,
            "batched_nnz_per_s": nnz_swept / t_batch,
            "autotune_s": t_tune, "same_results": same,
            "narrow_jobs": sum(_chosen_pilot(t)["narrow"] for t in tunes),
            "tuned": {"schedules": {str(k): sum(t["schedule"] == k for t in tunes)
                                    for k in (0, 1, 2)},
                      "chunks": {str(k): sum(t["chunk"] == k for t in tunes)
                                 for k in (64, 128, 256, 512)}},
            "outer_iters_total": int(sum(b[2]["outer_iters"] for b in batch))}


def path_measurement(pc, d) -> dict:
    """Regularisation path: 32 C values log-spaced over [2^-4, 2^6] on the
    text-like matrix, each warm-started from the previous solution; P from
    the autotuner at the middle C.  pcdn_solve_path against the same chain
    of pcdn_solve calls with the warm start passed through the host."""
    import synth
    Cs = synth.c4_path_Cs()
    s = pc.Solver(device=0).load_data(d)
    P = s.autotune(float(Cs[len(Cs) // 2]), 1e-4, "lr", seed=SEED)["P"]
    t0 = time.perf_counter()
    rc, W, infos = s.solve_path(Cs, P, 1e-4, "lr", seed=SEED)
    t_path = time.perf_counter() - t0
    t0 = time.perf_counter()
    w = None
    outer = 0
    for C in Cs:
        _, w, info = s.solve(float(C), P, 1e-4, "lr", seed=SEED, w0=w)
        outer += info["outer_iters"]
    t_plain = time.perf_counter() - t0
    # one solve at a time, each from w = 0
    t0 = time.perf_counter()
    cold_outer = 0
    for C in Cs:
        cold_outer += s.solve(float(C), P, 1e-4, "lr", seed=SEED)[2]["outer_iters"]
    t_cold = time.perf_counter() - t0
    # the path cut into runs on 8 contexts (loaded before the timed region)
    lanes = [s] + [pc.Solver(device=0).load_data(d) for _ in range(PATH_LANES - 1)]
    t0 = time.perf_counter()
    rl, Wl, il = pc.pcdn_solve_path_lanes([x.ctx for x in lanes], Cs, P, 1e-4, "lr", d.p,
                                          seed=SEED)
    t_lanes = time.perf_counter() - t0
    for x in lanes:
        x.close()
    n = len(Cs)
    return {"workload": "32 C values 2^-4..2^6 (log-spaced, ascending) on the text-like "
                        "L1-LR matrix, warm starts, eps=1e-4",
            "P": int(P), "path_s": t_path, "plain_chain_s": t_plain,
            "path_solves_per_s": n / t_path, "plain_solves_per_s": n / t_plain,
            "path_outer_iters": int(sum(i["outer_iters"] for i in infos)),
            "plain_outer_iters": int(outer),
            "cold_solves_per_s": n / t_cold, "cold_outer_iters": int(cold_outer),
            "lanes": PATH_LANES, "lanes_s": t_lanes, "lanes_solves_per_s": n / t_lanes,
            "lanes_outer_iters": int(sum(i["outer_iters"] for i in il)),
            "lanes_all_converged": bool(rl == 0 and all(i["converged"] for i in il)),
            "lanes_speedup_vs_plain_chain": t_plain / t_lanes,
            "path_speedup_vs_plain_chain": t_plain / t_path}


def _percentiles(lat):
    lat = sorted(lat)
    pick = lambda q: lat[min(len(lat) - 1, int(np.ceil(q * len(lat))) - 1)]
    return {"p50_s": pick(0.50), "p99_s": pick(0.99), "max_s": lat[-1],
            "mean_s": float(np.mean(lat))}


def serving_measurement(pc, synth, scale: float, n_req: int) -> dict:
    """A Poisson stream (50 requests/s) of mixed LR/SVM solves drawn from a
    pool of 16 problems, replayed by arrival time through the solve server
    (continuous batching, 64 GiB budget) and through one pcdn_load_csc +
    pcdn_solve after another in arrival order ("plain"); latency = finish
    time - arrival time.  P, schedule and chunk per pool problem from the autotuner, chosen
    before the stream starts."""
    pool = synth.c5_pool(scale=scale)
    stream = synth.c5_stream(count=n_req, pool=len(pool))
    Ps = []
    for d, loss in pool:
        s = pc.Solver(device=0).load_data(d)
        t = s.autotune(1.0, 1e-4, loss, seed=SEED)
        Ps.append(dict(P=t["P"], schedule=t["schedule"], chunk=t["chunk"]))
        s.close()
    # served
    srv = pc.Server(device=0, budget_bytes=64 << 30)
    arrival, finish, F_srv, st_srv = {}, {}, {}, {}
    out = {}
    k = 0
    t0 = time.perf_counter()
    while len(finish) < len(stream):
        now = time.perf_counter() - t0
        while k < len(stream) and stream[k][0] <= now:
            t_arr, i, C = stream[k]
            d, loss = pool[i]
            rid = srv.submit(d, C, Ps[i]["P"], 1e-4, loss, seed=SEED, schedule=Ps[i]["schedule"],
                             chunk=Ps[i]["chunk"])
            out[rid] = k
            arrival[k] = t_arr
            k += 1
        waiting, running, _ = srv.status()
        if waiting + running == 0:
            if k < len(stream):
                time.sleep(max(0.0, stream[k][0] - (time.perf_counter() - t0)))
            continue
        srv.step()
        for rid in [r for r in out if out[r] not in finish]:
            r = srv.take(rid)
            if r is not None:
                finish[out[rid]] = time.perf_counter() - t0
                F_srv[out[rid]] = r[2]["objective"]
                st_srv[out[rid]] = r[0]
    srv.close()
    lat_srv = [finish[q] - arrival[q] for q in range(len(stream))]
    span_srv = max(finish.values()) - stream[0][0]
    # plain: one request at a time, in arrival order
    s = pc.Solver(device=0)
    F_plain, st_plain, lat_plain = {}, {}, []
    t0 = time.perf_counter()
    for q, (t_arr, i, C) in enumerate(stream):
        now = time.perf_counter() - t0
        if now < t_arr:
            time.sleep(t_arr - now)
        d, loss = pool[i]
        s.load_data(d)
        st_plain[q], _, info = s.solve(C, Ps[i]["P"], 1e-4, loss, seed=SEED,
                                       schedule=Ps[i]["schedule"], chunk=Ps[i]["chunk"])
        F_plain[q] = info["objective"]
        lat_plain.append(time.perf_counter() - t0 - t_arr)
    span_plain = time.perf_counter() - t0 - stream[0][0]
    s.close()
    both = [q for q in range(len(stream)) if st_srv[q] == 0 and st_plain[q] == 0]
    gap = lambda qs: max((abs(F_srv[q] - F_plain[q]) / abs(F_plain[q]) for q in qs), default=0.0)
    return {"workload": f"{len(stream)} requests, Poisson 50/s, pool of {len(pool)} problems "
                        f"(LR/SVM 1:1, n log-U[1e3, {2e5 * scale:.0f}], p log-U[1e3, "
                        f"{2e6 * scale:.0f}], U{{20..150}} nnz/row, Zipf(1.1) columns), "
                        "C log-U[0.1, 10], eps=1e-4, autotuned P, schedule and chunk per pool "
                        "problem",
            "served": dict(_percentiles(lat_srv), solves_per_s=len(stream) / span_srv),
            "plain": dict(_percentiles(lat_plain), solves_per_s=len(stream) / span_plain),
            "converged": {"served": sum(v == 0 for v in st_srv.values()),
                          "plain": sum(v == 0 for v in st_plain.values())},
            "max_rel_objective_gap_converged": gap(both),
            "max_rel_objective_gap_all": gap(range(len(stream))),
            "nnz_mean": float(np.mean([d.nnz for d, _ in pool]))}


def copy_peak() -> dict:
    """Device-to-device copy of 1 GiB (torch's copy kernel), best of five:
    bytes read + written per second."""
    import torch
    nbytes = 1 << 30
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    y = torch.empty_like(x)
    best = float("inf")
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    del x, y
    return {"copy_GBps": 2 * nbytes / best / 1e9, "bytes": 2 * nbytes,
            "measured": "1 GiB device-to-device copy, HIP events, best of 5"}


def headline(pc, d, steps: int, warmup: int) -> dict:
    """The huge sparse L2-SVM problem: region A (value) and region B (kernel
    classes with HIP events), one solve continued step by step."""
    import torch
    s = pc.Solver(device=0).load_data(d)
    C, P = C3["C"], C3["P"]
    s.reset(C3["loss"], C)
    opts = dict(seed=SEED)
    for k in range(warmup):
        s.iterate(P, k, 1, want_subgrad=True, **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G = s.iterate(P, warmup, steps, want_subgrad=True, **opts)
    elapsed = time.perf_counter() - t0
    # region B: the next steps, every kernel class bracketed by events
    pc.pcdn_profile(s.ctx, (1 << len(KERNEL_CLASSES)) - 1)
    tb0 = time.perf_counter()
    s.iterate(P, warmup + steps, steps, want_subgrad=True, **opts)
    tb1 = time.perf_counter()
    kernels, totals = {}, {}
    for cls, name in enumerate(KERNEL_CLASSES):
        ms, n, b = pc.pcdn_profile_read(s.ctx, cls)
        totals[cls] = (ms, n, b)
        kernels[name] = {"launches": int(n), "ms_total": round(ms, 4),
                         "us_per_launch": round(1e3 * ms / max(n, 1), 3),
                         "alg_bytes_per_launch": round(b / max(n, 1)),
                         "alg_GBps": round(b / (ms / 1e3) / 1e9, 1) if ms > 0 and b > 0 else None}
    pc.pcdn_profile(s.ctx, 0)
    F, Gs = s.evaluate()
    s.close()
    return {"value": d.nnz * steps / elapsed, "ms_per_step": 1e3 * elapsed / steps,
            "subgrad_after_region_a": G, "objective_after": F, "subgrad_after": Gs,
            "region_b_ms_per_step": 1e3 * (tb1 - tb0) / steps,
            "kernels": kernels, "totals": totals}


def text_like(pc, d, steps: int, warmup: int) -> dict:
    """The text-like LR problem at its six (C, P) settings: one outer
    iteration of each per step, concurrently (one round of the batch engine
    per step) and one setting after another."""
    import torch
    solvers = []
    for C, P in SETTINGS:
        s = pc.Solver(device=0).load_data(d)
        s.reset("lr", C)
        solvers.append((s, C, P))
    for k in range(warmup):
        for s, C, P in solvers:
            s.iterate(P, k, 1, want_subgrad=True, seed=SEED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pc.iterate_batch([s for s, _, _ in solvers], [P for _, _, P in solvers], warmup, steps,
                     seed=SEED)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    per_setting = {f"C={C},P={P}": 0.0 for _, C, P in solvers}
    t0 = time.perf_counter()
    for step in range(steps):
        for s, C, P in solvers:
            ts = time.perf_counter()
            s.iterate(P, warmup + steps + step, 1, want_subgrad=True, seed=SEED)
            per_setting[f"C={C},P={P}"] += time.perf_counter() - ts
    torch.cuda.synchronize()
    elapsed_seq = time.perf_counter() - t0
    F = {f"C={C},P={P}": s.evaluate()[0] for s, C, P in solvers}
    for s, _, _ in solvers:
        s.close()
    nnz_total = d.nnz * len(SETTINGS) * steps
    return {"workload": "text-like L1-LR 20000x50000, Zipf(1.1) columns, "
                        "C in {0.5,4} x P in {64,1024,8192}, one outer iteration of each per step",
            "n": d.n, "p": d.p, "nnz": d.nnz,
            "value": nnz_total / elapsed, "unit": "nnz/s", "ms_per_step": 1e3 * elapsed / steps,
            "measured": "six settings concurrently, one pcdn_iterate_batch round per step",
            "sequential": {"value": nnz_total / elapsed_seq,
                           "ms_per_step": 1e3 * elapsed_seq / steps},
            "per_setting_ms_per_iter": {k: 1e3 * v / steps for k, v in per_setting.items()},
            "objective_after": F}


def main():
    args = parse()
    if args.source_hash:
        print(kernel_source_hash())
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU PCDN is a design "
              "(row sharding with two all-reduces per bundle), not built", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import paper_1306_4080_amd as pc

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    pc.ensure_built()
    print("bench: generating the huge sparse L2-SVM problem", file=sys.stderr, flush=True)
    d3 = synth.c3()
    print("bench: headline", file=sys.stderr, flush=True)
    h = headline(pc, d3, args.steps, args.warmup)
    cp = copy_peak()
    totals = h.pop("totals")
    dominant = max(totals, key=lambda k: totals[k][0])
    dom_ms, dom_n, dom_bytes = totals[dominant]
    avg_launch_s = dom_ms / 1e3 / max(dom_n, 1)
    bytes_per_launch = dom_bytes / max(dom_n, 1)
    achieved = bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    path_ms = sum(v[0] for v in totals.values())
    path_gbps = sum(v[2] for v in totals.values()) / (path_ms / 1e3) / 1e9 if path_ms > 0 else 0.0
    line = {
        "metric": METRIC,
        "value": h["value"],
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "huge sparse binary L1-regularised L2-SVM 100000x1000000, "
                               "~120 nonzeros per row, Zipf(1.05) columns capped at 50000, "
                               "C=1, P=16384, one outer iteration per step",
                   "n": d3.n, "p": d3.p, "nnz": d3.nnz, "loss": "l2svm", "C": C3["C"],
                   "P": C3["P"], "seed": SEED},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(KERNEL_CLASSES[dominant]),
                     "kernel": KERNEL_NAMES[dominant],
                     "alg_bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": avg_launch_s * 1e6, "launches": int(dom_n),
                     "copy_GBps": cp["copy_GBps"],
                     "frac_of_copy": achieved / cp["copy_GBps"],
                     "measured": "HIP events around each launch on the library's stream in "
                                 "region B (the next steps of the same solve)",
                     "region_b_ms_per_step": h["region_b_ms_per_step"],
                     # the whole path's kernels together: every class's algorithmic
                     # bytes over every class's event time in region B
                     "path_alg_GBps": path_gbps,
                     "path_frac": path_gbps / HBM_PEAK_GBS},
        "kernels": h["kernels"],
        "objective_after": h["objective_after"],
        "subgrad_after": h["subgrad_after"],
    }
    del d3
    d2 = synth.c2()
    if not args.no_text_like:
        print("bench: text-like settings", file=sys.stderr, flush=True)
        line["text_like"] = text_like(pc, d2, args.steps, args.warmup)
    if not args.no_batched:
        print("bench: batched problems and path", file=sys.stderr, flush=True)
        line["batched"] = batched_measurement(pc, synth, args.batched_scale)
        line["path"] = path_measurement(pc, d2)
    if not args.no_serving:
        print("bench: serving", file=sys.stderr, flush=True)
        line["serving"] = serving_measurement(pc, synth, args.serving_scale,
                                              args.serving_requests)
    if not args.no_cpu_baseline:
        print("bench: CPU oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(synth.c3(), args.cpu_seconds)
    print(json.dumps(line), flush=True)
    # every batched and served solve must equal its plain run (the kernels'
    # sums have fixed orders); a difference is a defect, not noise
    bad = []
    if "batched" in line and not line["batched"]["same_results"]:
        bad.append("batched solves differ from the plain ones")
    if "serving" in line and line["serving"]["max_rel_objective_gap_converged"] > 1e-6:
        bad.append("served objectives differ from the plain ones by more than 1e-6")
    if bad:
        print("bench.py: " + "; ".join(bad), file=sys.stderr)
        sys.exit(3)


if __name__ == "__main__":
    main()
