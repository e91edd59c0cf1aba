"""Several solves per call, through the C ABI: pcdn_solve_batch (independent
problems advanced together, the single-workgroup ones in one launch) and
pcdn_solve_path (a regularisation path with warm starts).

Bars:
- every batched job against the same solve run alone with pcdn_solve:
  bit-identical (the same outer iterations, bundles, line-search steps and
  failures, the same F, stopping norm and w);
- every job and every path point against the FP64 oracle: F within 1e-6
  relative and the same trajectory on the non-degenerate problems.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-6


@pytest.fixture(scope="module")
def pc():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_4080_amd as pc
    pc.ensure_built()
    return pc


def _empty(n, p):
    return synth.Data(n=n, p=p, col_ptr=np.zeros(p + 1, np.int64), row_idx=np.zeros(0, np.int32),
                      val=np.zeros(0, np.float32), y=np.where(np.arange(n) % 2, 1, -1).astype(np.int8))


def _mixed_jobs():
    """(name, data, loss, C, P, eps, opts, strict) of a mixed batch: both
    losses, both schedules, sizes from 3x4 to 2,000x3,000, one job that is
    optimal at w = 0 and one that stops at max_outer."""
    c1 = synth.c1()
    return [
        ("c1-lr-narrow", c1, "lr", 1.0, 32, 1e-4, {}, True),
        ("c1-svm-narrow", c1, "svm", 0.5, 32, 1e-4, {}, True),
        ("c1-lr-wide", c1, "lr", 2.0, 64, 1e-4, {"schedule": "wide"}, True),
        ("rand-lr", synth.sparse_random(11, 2000, 3000, 0.004), "lr", 1.0, 96, 1e-4, {}, True),
        ("rand-svm-wide", synth.sparse_random(12, 800, 5000, 0.002, binary=True), "svm", 0.3, 512,
         1e-3, {"schedule": "wide"}, True),
        ("tiny-lr-p1", synth.tiny(70, n=50, p=13, density=0.3, empty_cols=(0, 5)), "lr", 1.0, 1,
         1e-6, {"max_outer": 500}, False),
        ("empty", _empty(3, 4), "svm", 1.0, 2, 1e-6, {}, False),
        ("c1-lr-maxouter", c1, "lr", 1.0, 32, 1e-12, {"max_outer": 3}, True),
    ]


def _assert_same_run(a, b):
    """Batched or served vs alone on the GPU: bit-identical.  Every sum of
    the library runs in an order fixed by the problem and the launch shape
    (d^T x included: fixed-order row sums on the multi-kernel schedule,
    integer fixed point in the single workgroup), and the batch engine keeps
    each problem's launch shapes, so the same solve gives the same bits
    alone, in a batch and in the server."""
    (ra, wa, ia), (rb, wb, ib) = a, b
    keys = ("outer_iters", "converged", "bundles", "ls_steps", "ls_fail", "nnz_swept")
    assert ra == rb
    for k in keys:
        assert ia[k] == ib[k], (k, ia[k], ib[k])
    assert ia["objective"] == ib["objective"]
    assert ia["subgrad"] == ib["subgrad"]
    np.testing.assert_array_equal(wa, wb)


def _assert_same_trajectory(a, b):
    """Two schedules of one solve (the single workgroup against the
    multi-kernel path): the same arithmetic summed in different orders (g_j
    and h_j by segmented scans against chunk sums; the line-search sums over
    512 threads against G blocks), so the same trajectory with F and w equal
    up to the last bits."""
    (ra, wa, ia), (rb, wb, ib) = a, b
    assert ra == rb
    for k in ("outer_iters", "converged", "bundles", "ls_steps", "ls_fail", "nnz_swept"):
        assert ia[k] == ib[k], (k, ia[k], ib[k])
    assert ia["objective"] == pytest.approx(ib["objective"], rel=1e-10)
    np.testing.assert_allclose(wa, wb, rtol=1e-6, atol=1e-8 * max(1.0, np.max(np.abs(wb))))


def _assert_oracle(g, o, strict):
    rc, w_g, ig = g
    w_o, io = o
    assert ig["objective"] == pytest.approx(io["objective"], rel=RTOL)
    assert ig["converged"] == io["converged"]
    if strict:
        for k in ("outer_iters", "bundles", "ls_steps", "ls_fail", "nnz_swept"):
            assert ig[k] == io[k], (k, ig[k], io[k])


def test_batch_matches_alone_and_oracle(pc):
    jobs = _mixed_jobs()
    solvers = [pc.Solver(device=0).load_data(d) for _, d, *_ in jobs]
    specs = [s.job(C, P, eps, loss, seed=5, **opts)
             for s, (_, d, loss, C, P, eps, opts, _) in zip(solvers, jobs)]
    batched = pc.solve_batch(specs)
    for s, (name, d, loss, C, P, eps, opts, strict), b in zip(solvers, jobs, batched):
        print(f"{name}: status={b[0]} outer={b[2]['outer_iters']} F={b[2]['objective']:.15g}",
              flush=True)
        alone = s.solve(C, P, eps, loss, seed=5, **opts)
        _assert_same_run(b, alone)
        w_o, io, _ = oracle.solve(oracle.Problem.from_data(d), oracle.Params(loss=loss, C=C),
                                  P=P, eps=eps, seed=5, max_outer=opts.get("max_outer", 1000))
        _assert_oracle(b, (w_o, io), strict)
    assert batched[-1][0] == 1           # stopped at max_outer
    assert batched[-2][2]["outer_iters"] == 0 and np.all(batched[-2][1] == 0)
    for s in solvers:
        s.close()


def test_batch_many_small_problems(pc):
    """32 heterogeneous LR problems (the batched recipe at small sizes) in one
    call, every other one forced onto the multi-kernel schedule (so both the
    single-workgroup launch and the lock-step executor carry 16 problems):
    every job equals its solve alone."""
    rng = np.random.default_rng(4)
    data = []
    for i in range(32):
        n = int(rng.integers(200, 1500))
        p = int(rng.integers(300, 3000))
        dens = float(rng.uniform(0.002, 0.02))
        data.append(synth.sparse_random(100 + i, n, p, dens))
    sched = ["wide" if i % 2 else "auto" for i in range(32)]
    solvers = [pc.Solver(device=0).load_data(d) for d in data]
    specs = [s.job(1.0, max(1, d.p // 20), 1e-4, "lr", seed=9, schedule=sc)
             for s, d, sc in zip(solvers, data, sched)]
    batched = pc.solve_batch(specs)
    for s, d, b, sc in zip(solvers, data, batched, sched):
        alone = s.solve(1.0, max(1, d.p // 20), 1e-4, "lr", seed=9, schedule=sc)
        _assert_same_run(b, alone)
        assert b[0] == 0
    # spot-check three of them against the oracle
    for i in (0, 13, 31):
        d = data[i]
        w_o, io, _ = oracle.solve(oracle.Problem.from_data(d), oracle.Params(loss="lr", C=1.0),
                                  P=max(1, d.p // 20), eps=1e-4, seed=9)
        _assert_oracle(batched[i], (w_o, io), True)
    for s in solvers:
        s.close()


def test_executor_partition_with_multiblock_scans(pc):
    """Multi-kernel jobs run their partition as executor tasks, whose scans
    take several blocks once p > 4,096 (chunk counts) and p > 16,384 (the
    radix histograms), also with shrinking (active features keyed first).
    A few outer iterations of such jobs (a different permutation would move
    w and F far beyond the bars) equal the solve alone, and w equals the
    oracle's, which draws the same seeded permutation, to the parity bar."""
    data = [synth.sparse_random(120, 3000, 20000, 0.002),
            synth.sparse_random(121, 2000, 70000, 0.001),
            synth.sparse_random(122, 1500, 3000, 0.004),
            synth.sparse_random(123, 3000, 30000, 0.002)]
    solvers = [pc.Solver(device=0).load_data(d) for d in data]
    Ps = [d.p // 10 for d in data]
    # the last job shrinks: its keys put the active features first
    opts = [dict(seed=3, schedule="wide", max_outer=m, shrink=sh)
            for m, sh in ((2, False), (2, False), (2, False), (4, True))]
    batched = pc.solve_batch([s.job(1.0, P, 1e-12, "lr", **o)
                              for s, P, o in zip(solvers, Ps, opts)])
    for s, d, P, o, b in zip(solvers, data, Ps, opts, batched):
        print(f"p={d.p} shrink={o['shrink']}: status={b[0]} outer={b[2]['outer_iters']} "
              f"F={b[2]['objective']:.15g}", flush=True)
        assert b[0] == 1 and b[2]["outer_iters"] == o["max_outer"]
        _assert_same_run(b, s.solve(1.0, P, 1e-12, "lr", **o))
        w_o, io, _ = oracle.solve(oracle.Problem.from_data(d),
                                  oracle.Params(loss="lr", C=1.0, shrink=o["shrink"]),
                                  P=P, eps=1e-12, seed=3, max_outer=o["max_outer"])
        _assert_oracle(b, (w_o, io), True)
        np.testing.assert_allclose(b[1], w_o, rtol=RTOL, atol=RTOL * max(1.0, np.max(np.abs(w_o))))
    for s in solvers:
        s.close()


def test_executor_split_line_search(pc):
    """Enough multi-kernel jobs with n = 20,000 that the executor runs the
    later line-search candidate groups as a task of its own (which stops at
    once when the first group of four holds the accepted step).  Bundles of
    all features at C = 16 need q = 4 (the second group) in most outer
    iterations, so both ways out of that task run.  Every job equals its
    solve alone and the oracle."""
    specs = []
    for i in range(8):
        lr = i % 2 == 0
        d = synth.sparse_random(130 + i, 20000, 1500, 0.02 if lr else 0.01, binary=True)
        specs.append((d, "lr" if lr else "svm", 16.0 if lr else 4.0, d.p if i < 4 else d.p // 6))
    solvers = [pc.Solver(device=0).load_data(d) for d, *_ in specs]
    opts = dict(seed=3, schedule="wide", max_outer=8)
    batched = pc.solve_batch([s.job(C, P, 1e-12, loss, **opts)
                              for s, (d, loss, C, P) in zip(solvers, specs)])
    long_searches = 0
    for s, (d, loss, C, P), b in zip(solvers, specs, batched):
        ib = b[2]
        print(f"{loss} C={C} P={P}: outer={ib['outer_iters']} bundles={ib['bundles']} "
              f"ls_steps={ib['ls_steps']} F={ib['objective']:.15g}", flush=True)
        _assert_same_run(b, s.solve(C, P, 1e-12, loss, **opts))
        w_o, io, _ = oracle.solve(oracle.Problem.from_data(d), oracle.Params(loss=loss, C=C),
                                  P=P, eps=1e-12, seed=3, max_outer=8)
        _assert_oracle(b, (w_o, io), True)
        long_searches += ib["ls_steps"] > 4 * ib["bundles"]
    assert long_searches >= 1
    for s in solvers:
        s.close()


def test_batch_errors_run_nothing(pc):
    from paper_1306_4080_amd import PcdnError
    d = synth.c1()
    a = pc.Solver(device=0).load_data(d)
    b = pc.Solver(device=0).load_data(d)
    assert pc.solve_batch([]) == []
    with pytest.raises(PcdnError, match="E_ARG"):
        pc.solve_batch([a.job(1.0, 32, 1e-4, "lr"), b.job(-1.0, 32, 1e-4, "lr")])
    with pytest.raises(PcdnError, match="E_ARG"):
        pc.solve_batch([a.job(1.0, 32, 1e-4, "lr"), a.job(1.0, 32, 1e-4, "lr")])
    with pytest.raises(PcdnError, match="E_ARG"):
        pc.solve_batch([a.job(1.0, -1, 1e-4, "lr")])
    with pytest.raises(PcdnError, match="E_ARG"):
        pc.solve_batch([a.job(1.0, 0, 1e-4, "lr"), b.job(1.0, d.p + 1, 1e-4, "lr")])
    # nothing ran: a has no state yet
    with pytest.raises(PcdnError, match="E_STATE"):
        a.evaluate()
    a.close()
    b.close()


def test_path_matches_oracle_chain(pc):
    """C log-spaced, ascending, each solve warm-started from the previous
    solution; the oracle runs the same chain."""
    d = synth.c1()
    Cs = 2.0 ** np.linspace(-4, 2, 6)
    s = pc.Solver(device=0).load_data(d)
    rc, W, infos = s.solve_path(Cs, 32, 1e-4, "lr", seed=3)
    assert rc == 0
    prob = oracle.Problem.from_data(d)
    w_prev = None
    for k, C in enumerate(Cs):
        w_o, io, _ = oracle.solve(prob, oracle.Params(loss="lr", C=float(C)), P=32, eps=1e-4,
                                  seed=3, w0=w_prev)
        print(f"C={C:.4g}: outer {infos[k]['outer_iters']}/{io['outer_iters']} "
              f"F {infos[k]['objective']:.15g}/{io['objective']:.15g}", flush=True)
        _assert_oracle((rc, W[k], infos[k]), (w_o, io), True)
        w_prev = w_o
    # the path equals solves chained through the host-side warm start
    w_prev = None
    for k, C in enumerate(Cs):
        r2, w2, i2 = s.solve(float(C), 32, 1e-4, "lr", seed=3, w0=w_prev)
        _assert_same_run((rc, W[k], infos[k]), (r2, w2, i2))
        w_prev = w2
    s.close()


@pytest.mark.parametrize("schedule", ["wide", "narrow"])
def test_path_lanes_match_runs_alone_and_oracle(pc, schedule):
    """Seven C values over three contexts holding the same data: runs
    Cs[0:2], Cs[2:4], Cs[4:7] advance together, and each run equals
    pcdn_solve_path over that run alone (bit for bit) and the oracle's
    warm-started chain over it (first C from w = 0)."""
    d = synth.c1()
    Cs = 2.0 ** np.linspace(-4, 2, 7)
    solvers = [pc.Solver(device=0).load_data(d) for _ in range(3)]
    rc, W, infos = pc.pcdn_solve_path_lanes([s.ctx for s in solvers], Cs, 32, 1e-4, "lr", d.p,
                                            seed=3, schedule=schedule)
    assert rc == 0
    prob = oracle.Problem.from_data(d)
    alone = pc.Solver(device=0).load_data(d)
    for lo, hi in ((0, 2), (2, 4), (4, 7)):
        ra, Wa, ia = alone.solve_path(Cs[lo:hi], 32, 1e-4, "lr", seed=3, schedule=schedule)
        w_prev = None
        for k in range(lo, hi):
            _assert_same_run((rc, W[k], infos[k]), (ra, Wa[k - lo], ia[k - lo]))
            w_o, io, _ = oracle.solve(prob, oracle.Params(loss="lr", C=float(Cs[k])), P=32,
                                      eps=1e-4, seed=3, w0=w_prev)
            _assert_oracle((rc, W[k], infos[k]), (w_o, io), True)
            w_prev = w_o
    # more lanes than C values: one C per lane
    r1, W1, i1 = pc.pcdn_solve_path_lanes([s.ctx for s in solvers], Cs[:2], 32, 1e-4, "lr", d.p,
                                          seed=3, schedule=schedule)
    for k in range(2):
        single = alone.solve(float(Cs[k]), 32, 1e-4, "lr", seed=3, schedule=schedule)
        _assert_same_run((r1, W1[k], i1[k]), single)
    alone.close()
    for s in solvers:
        s.close()


def test_path_lanes_reject_different_data(pc):
    from paper_1306_4080_amd import PcdnError
    d = synth.c1()
    e = synth.tiny(3, n=d.n, p=d.p, density=0.1)
    a, b = pc.Solver(device=0).load_data(d), pc.Solver(device=0).load_data(e)
    with pytest.raises(PcdnError, match="E_ARG"):
        pc.pcdn_solve_path_lanes([a.ctx, b.ctx], [0.5, 1.0], 32, 1e-4, "lr", d.p)
    with pytest.raises(PcdnError, match="E_ARG"):
        pc.pcdn_solve_path_lanes([a.ctx, a.ctx], [0.5, 1.0], 32, 1e-4, "lr", d.p)
    a.close()
    b.close()


def test_heavy_bundles_beyond_the_list_cap(pc):
    """Every bundle heavy (1,000 bundles of ~6,000 nonzeros, more than the
    256 the list holds, each with more distinct rows than the LDS holds):
    the first 256 run on the multi-kernel path, the rest in the single
    workgroup's global-memory path; the trajectory is the oracle's."""
    d = synth.bernoulli_csc(91, 20000, 64000, 0.0047)
    s = pc.Solver(device=0).load_data(d)
    g = s.solve(1.0, 64, 1e-3, "lr", seed=5)
    s.close()
    w_o, io, _ = oracle.solve(oracle.Problem.from_data(d), oracle.Params(loss="lr", C=1.0),
                              P=64, eps=1e-3, seed=5)
    _assert_oracle(g, (w_o, io), True)


def test_path_heavy_bundles(pc):
    """A path on the text-like matrix at P = 64 (automatic schedule: the
    engine's heavy-bundle path, one job per C): the oracle's warm-started
    chain, and the chain forced onto the plain single-workgroup schedule."""
    d = synth.c2()
    Cs = [0.25, 0.5, 1.0]
    s = pc.Solver(device=0).load_data(d)
    rc, W, infos = s.solve_path(Cs, 64, 1e-4, "lr", seed=2)
    rn, Wn, infn = s.solve_path(Cs, 64, 1e-4, "lr", seed=2, schedule="narrow")
    prob = oracle.Problem.from_data(d)
    w_prev = None
    for k, C in enumerate(Cs):
        w_o, io, _ = oracle.solve(prob, oracle.Params(loss="lr", C=C), P=64, eps=1e-4, seed=2,
                                  w0=w_prev)
        print(f"C={C}: outer {infos[k]['outer_iters']}/{io['outer_iters']}", flush=True)
        _assert_oracle((rc, W[k], infos[k]), (w_o, io), True)
        _assert_same_trajectory((rc, W[k], infos[k]), (rn, Wn[k], infn[k]))
        w_prev = w_o
    s.close()


def test_path_svm_wide(pc):
    d = synth.sparse_random(21, 1500, 4000, 0.003, binary=True)
    Cs = [0.05, 0.2, 0.8]
    s = pc.Solver(device=0).load_data(d)
    rc, W, infos = s.solve_path(Cs, 1024, 1e-3, "svm", seed=2, schedule="wide")
    prob = oracle.Problem.from_data(d)
    w_prev = None
    for k, C in enumerate(Cs):
        w_o, io, _ = oracle.solve(prob, oracle.Params(loss="svm", C=C), P=1024, eps=1e-3, seed=2,
                                  w0=w_prev)
        _assert_oracle((rc, W[k], infos[k]), (w_o, io), True)
        w_prev = w_o
    s.close()


def test_autotune_ladder_and_choice(pc):
    """The candidates are the paper's pilot start (5% of the features) and
    its factor-4 neighbours, nearest first; then, at the best of those, the
    schedule the automatic choice did not take, and the other sweep range
    widths (pcdn_opts.chunk) when multi-kernel bundles won.  The choice is the fastest finished pilot;
    solving with it matches the oracle at that P."""
    d = synth.c1()
    s = pc.Solver(device=0).load_data(d)
    t = s.autotune(1.0, 1e-4, "lr", seed=1)
    P0 = round(0.05 * d.p)
    ladder = []
    for k in (0, -1, 1, -2, 2, -3):
        P = min(d.p, max(1, int(np.floor(P0 * 4.0 ** k + 0.5))))
        if P not in ladder:
            ladder.append(P)
    tried = t["tried"]
    print("tuned:", {k: t[k] for k in ("P", "schedule", "chunk", "predicted_seconds")}, flush=True)
    for x in tried:
        print("  ", x, flush=True)
    assert [x["P"] for x in tried[:len(ladder)]] == ladder
    assert all(x["schedule"] == 0 and x["chunk"] == 256 for x in tried[:len(ladder)])
    first = [x for x in tried[:len(ladder)] if np.isfinite(x["predicted_seconds"])]
    assert first
    Pb = min(first, key=lambda x: x["predicted_seconds"])["P"]
    rest = tried[len(ladder):]
    assert rest and all(x["P"] == Pb for x in rest)
    assert rest[0]["schedule"] in (1, 2) and rest[0]["narrow"] == (rest[0]["schedule"] == 2)
    assert {x["chunk"] for x in rest[1:]} <= {64, 128, 512}
    done = [x for x in tried if np.isfinite(x["predicted_seconds"])]
    best = min(done, key=lambda x: x["predicted_seconds"])
    assert t["predicted_seconds"] == best["predicted_seconds"]
    assert (t["P"], t["schedule"], t["chunk"]) == (best["P"], best["schedule"], best["chunk"])
    assert all(x["outer"] > 0 for x in tried)
    g = s.solve(1.0, t["P"], 1e-4, "lr", seed=1, schedule=t["schedule"], chunk=t["chunk"])
    w_o, io, _ = oracle.solve(oracle.Problem.from_data(d), oracle.Params(loss="lr", C=1.0),
                              P=t["P"], eps=1e-4, seed=1)
    _assert_oracle(g, (w_o, io), True)
    s.close()


def test_batch_autotuned_jobs(pc):
    """P = 0 in a job: the batch tunes it first, writes it back, and the job
    equals its solve alone at that P."""
    data = [synth.bernoulli_csc(300 + i, 600 + 200 * i, 2000 + 500 * i, 0.01) for i in range(3)]
    solvers = [pc.Solver(device=0).load_data(d) for d in data]
    out = pc.solve_batch([s.job(1.0, 0, 1e-4, "lr", seed=4) for s in solvers])
    for s, b in zip(solvers, out):
        assert b[2]["P"] >= 1
        # the tuner's schedule and chunk, which fix the summation order
        alone = s.solve(1.0, b[2]["P"], 1e-4, "lr", seed=4, schedule=b[2]["schedule"],
                        chunk=b[2]["chunk"])
        _assert_same_run(b, alone)
    for s in solvers:
        s.close()


def test_iterate_batch_matches_sequential_and_oracle(pc):
    """pcdn_iterate_batch continues several contexts' states together (both
    schedules, both losses); each ends where pcdn_iterate alone ends, and
    where the oracle's first outer iterations end."""
    c1 = synth.c1()
    rnd = synth.bernoulli_csc(77, 1200, 3000, 0.01)
    cases = [(c1, "lr", 1.0, 32), (c1, "svm", 0.5, 100), (rnd, "lr", 2.0, 600),
             (rnd, "svm", 1.0, 64)]
    iters = 5
    a = [pc.Solver(device=0).load_data(d) for d, *_ in cases]
    b = [pc.Solver(device=0).load_data(d) for d, *_ in cases]
    for s, (d, loss, C, P) in zip(a + b, cases + cases):
        s.reset(loss, C)
    G_batch = pc.iterate_batch(a, [P for *_, P in cases], 0, iters, seed=11)
    for sa, sb, (d, loss, C, P), g in zip(a, b, cases, G_batch):
        g_alone = sb.iterate(P, 0, iters, seed=11)
        assert g == g_alone
        np.testing.assert_array_equal(sa.w(), sb.w())
        w_o, io, _ = oracle.solve(oracle.Problem.from_data(d), oracle.Params(loss=loss, C=C),
                                  P=P, eps=0.0, seed=11, max_outer=iters)
        F, G = sa.evaluate()
        assert F == pytest.approx(io["objective"], rel=RTOL)
        assert G == pytest.approx(io["subgrad"], rel=1e-5)
    for s in a + b:
        s.close()


def test_batch_shrink_jobs(pc):
    """Shrinking jobs beside plain ones, on both schedules: each batched job
    equals its solve alone and the oracle's shrinking solve."""
    c1 = synth.c1()
    rnd = synth.bernoulli_csc(78, 1500, 4000, 0.008)
    jobs = [(c1, "lr", 1.0, 32, 1e-4, {"shrink": True}),
            (c1, "svm", 1.0, 32, 1e-3, {"shrink": True, "schedule": "wide"}),
            (rnd, "lr", 2.0, 200, 1e-4, {"shrink": True}),
            (rnd, "lr", 2.0, 200, 1e-4, {}),
            (rnd, "svm", 0.5, 400, 1e-3, {"shrink": True, "schedule": "wide"})]
    solvers = [pc.Solver(device=0).load_data(d) for d, *_ in jobs]
    specs = [s.job(C, P, eps, loss, seed=3, **o) for s, (d, loss, C, P, eps, o) in zip(solvers, jobs)]
    batched = pc.solve_batch(specs)
    for s, (d, loss, C, P, eps, o), b in zip(solvers, jobs, batched):
        print(f"{loss} C={C} P={P} {o}: outer={b[2]['outer_iters']} swept={b[2]['nnz_swept']}",
              flush=True)
        _assert_same_run(b, s.solve(C, P, eps, loss, seed=3, **o))
        w_o, io, _ = oracle.solve(oracle.Problem.from_data(d),
                                  oracle.Params(loss=loss, C=C, shrink=o.get("shrink", False)),
                                  P=P, eps=eps, seed=3)
        _assert_oracle(b, (w_o, io), True)
    assert batched[2][2]["nnz_swept"] < batched[3][2]["nnz_swept"]
    for s in solvers:
        s.close()


def test_iterate_batch_shrink(pc):
    """pcdn_iterate_batch with shrinking, continued over two calls: the active
    set carries over inside each context, as in the oracle's run."""
    c1 = synth.c1()
    rnd = synth.bernoulli_csc(79, 1200, 3000, 0.01)
    cases = [(c1, "lr", 1.0, 32), (rnd, "svm", 1.0, 600)]
    a = [pc.Solver(device=0).load_data(d) for d, *_ in cases]
    for s, (d, loss, C, P) in zip(a, cases):
        s.reset(loss, C)
    Ps = [P for *_, P in cases]
    pc.iterate_batch(a, Ps, 0, 3, seed=13, shrink=True)
    pc.iterate_batch(a, Ps, 3, 3, seed=13, shrink=True)
    for s, (d, loss, C, P) in zip(a, cases):
        w_o, io, _ = oracle.solve(oracle.Problem.from_data(d),
                                  oracle.Params(loss=loss, C=C, shrink=True),
                                  P=P, eps=0.0, seed=13, max_outer=6)
        F, G = s.evaluate()
        assert F == pytest.approx(io["objective"], rel=RTOL)
        np.testing.assert_allclose(s.w(), w_o, rtol=RTOL, atol=RTOL * np.max(np.abs(w_o)))
        s.close()


def test_batch_regularised_jobs(pc):
    """Elastic-net and ridge jobs beside an L1 job in one batch (both
    schedules, one with shrinking): each equals its solve alone and the
    oracle's."""
    c1 = synth.c1()
    rnd = synth.bernoulli_csc(80, 1500, 4000, 0.008)
    jobs = [(c1, "lr", 1.0, 32, 1e-4, {"penalty": "elastic", "l2": 0.5}),
            (c1, "svm", 1.0, 32, 1e-3, {"penalty": "l2", "l2": 0.7, "schedule": "wide"}),
            (rnd, "lr", 2.0, 200, 1e-4, {"penalty": "elastic", "l2": 1.0, "shrink": True}),
            (rnd, "lr", 2.0, 200, 1e-4, {})]
    solvers = [pc.Solver(device=0).load_data(d) for d, *_ in jobs]
    specs = [s.job(C, P, eps, loss, seed=4, **o) for s, (d, loss, C, P, eps, o) in zip(solvers, jobs)]
    batched = pc.solve_batch(specs)
    for s, (d, loss, C, P, eps, o), b in zip(solvers, jobs, batched):
        print(f"{loss} C={C} P={P} {o}: outer={b[2]['outer_iters']} F={b[2]['objective']:.15g}",
              flush=True)
        _assert_same_run(b, s.solve(C, P, eps, loss, seed=4, **o))
        reg = {k: o[k] for k in ("penalty", "l2", "shrink") if k in o}
        w_o, io, _ = oracle.solve(oracle.Problem.from_data(d), oracle.Params(loss=loss, C=C, **reg),
                                  P=P, eps=eps, seed=4)
        _assert_oracle(b, (w_o, io), True)
    for s in solvers:
        s.close()


def test_batch_heavy_bundles_on_multi_kernel_path(pc):
    """The text-like matrix at P = 64 (automatic schedule) in the batch engine:
    bundles of at least 4,096 nonzeros (those holding Zipf-head columns) run
    on the multi-kernel path between single-workgroup segments.  Each job
    equals the plain single-workgroup solve alone and the oracle's, with and
    without shrinking, and for an elastic-net L2-SVM job; pcdn_iterate_batch on the same jobs ends where
    pcdn_iterate does (the plain runs forced onto the single-workgroup
    schedule; pcdn_solve and pcdn_iterate take the engine's path under the
    automatic one)."""
    d = synth.c2()
    prob = oracle.Problem.from_data(d)
    jobs = [(0.5, 64, {}, "lr", 1e-4), (4.0, 64, {}, "lr", 1e-4),
            (0.5, 64, {"shrink": True}, "lr", 1e-4),
            (0.5, 64, {"penalty": "elastic", "l2": 0.5}, "svm", 1e-3)]
    solvers = [pc.Solver(device=0).load_data(d) for _ in jobs]
    specs = [s.job(C, P, eps, loss, seed=1, **o) for s, (C, P, o, loss, eps) in zip(solvers, jobs)]
    batched = pc.solve_batch(specs)
    for s, (C, P, o, loss, eps), b in zip(solvers, jobs, batched):
        print(f"{loss} C={C} P={P} {o}: outer={b[2]['outer_iters']} F={b[2]['objective']:.15g}",
              flush=True)
        _assert_same_trajectory(b, s.solve(C, P, eps, loss, seed=1, schedule="narrow", **o))
        _assert_same_run(b, s.solve(C, P, eps, loss, seed=1, **o))
        w_o, io, _ = oracle.solve(prob, oracle.Params(loss=loss, C=C, **o), P=P, eps=eps, seed=1)
        _assert_oracle(b, (w_o, io), True)
    # a few outer iterations continued together vs one context at a time
    other = [pc.Solver(device=0).load_data(d) for _ in jobs[:2]]
    for s, t, (C, P, o, loss, eps) in zip(solvers[:2], other, jobs[:2]):
        s.reset("lr", C)
        t.reset("lr", C)
    G = pc.iterate_batch(solvers[:2], [64, 64], 0, 4, seed=2)
    for s, t, g in zip(solvers[:2], other, G):
        assert g == pytest.approx(t.iterate(64, 0, 4, seed=2, schedule="narrow"), rel=1e-10)
        np.testing.assert_allclose(s.w(), t.w(), rtol=1e-9, atol=1e-12)
    for s in solvers + other:
        s.close()
