"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (the build's target): g, h, d, d^T x at 1e-6 relative with the
absolute floors 1e-6 * C * sum_i |x_ij| for g_j and 1e-6 * max|.| for d and
d^T x; the accepted step alpha and index q exactly (powers of two); final
objective at 1e-6 relative.  The permutation is integer work: bit-exact.
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


def _solver(pc, d):
    return pc.Solver(device=0).load_data(d)


def _colabs(d):
    return np.array([np.abs(d.val[d.col_ptr[j]:d.col_ptr[j + 1]].astype(float)).sum()
                     for j in range(d.p)])


def _compare_step(d, s_gpu, s_orc, bundle, C):
    colabs = _colabs(d)[bundle]
    g_floor = RTOL * C * colabs + 1e-300
    np.testing.assert_array_less(np.abs(s_gpu["g"] - s_orc["g"]), RTOL * np.abs(s_orc["g"]) + g_floor + 1e-15)
    np.testing.assert_allclose(s_gpu["h"], s_orc["h"], rtol=RTOL, atol=1e-15)
    dmax = np.max(np.abs(s_orc["d"])) if len(bundle) else 0.0
    np.testing.assert_allclose(s_gpu["d"], s_orc["d"], rtol=RTOL, atol=RTOL * dmax + 1e-300)
    xmax = np.max(np.abs(s_orc["dtx"]))
    np.testing.assert_allclose(s_gpu["dtx"], s_orc["dtx"], rtol=RTOL, atol=RTOL * xmax + 1e-300)
    assert s_gpu["q"] == s_orc["q"], (s_gpu["q"], s_orc["q"], s_gpu["dF"], s_orc["dF"])
    assert s_gpu["alpha"] == s_orc["alpha"]
    assert s_gpu["delta"] == pytest.approx(s_orc["delta"], rel=RTOL, abs=1e-12)
    assert s_gpu["dF"] == pytest.approx(s_orc["dF"], rel=RTOL, abs=1e-12)


# --------------------------------------------------------------------------
# a1: the partition
# --------------------------------------------------------------------------
@pytest.mark.parametrize("p", [1, 7, 4096, 4097, 50000, 1000000])
def test_permutation_bitexact(pc, p):
    d = synth.tiny(1, n=3, p=p, density=0.0) if p < 100 else None
    if d is None:
        # a matrix with p columns is needed only to size the context
        col_ptr = np.zeros(p + 1, dtype=np.int64)
        d = synth.Data(n=1, p=p, col_ptr=col_ptr, row_idx=np.zeros(0, np.int32),
                       val=np.zeros(0, np.float32), y=np.ones(1, np.int8))
    s = _solver(pc, d)
    for seed, k in ((0, 0), (20130616, 3), (2**64 - 1, 11)):
        assert np.array_equal(s.permutation(seed, k), oracle.permutation(seed, k, p)), (seed, k)
    s.close()


# --------------------------------------------------------------------------
# a2-a6: one inner iteration on the same w and bundle
# --------------------------------------------------------------------------
def _random_w(rng, p, frac=0.5, scale=0.3):
    return rng.normal(0, scale, p) * (rng.random(p) < frac)


SCHEDULES = ["wide", "narrow"]


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("loss", ["lr", "svm"])
def test_step_parity_c1(pc, loss, schedule):
    d = synth.c1()
    prob = oracle.Problem.from_data(d)
    C = 1.0
    par = oracle.Params(loss=loss, C=C)
    s = _solver(pc, d)
    rng = np.random.default_rng(5)
    for trial in range(6):
        w = _random_w(rng, d.p) if trial else np.zeros(d.p)
        s.reset(loss, C, w)
        cache = oracle.cache_from_w(prob, loss, w)
        # z = X w is summed with atomics in no fixed order, so the SVM slack
        # b = 1 - y z carries a few ulps of max(1, |z|) in absolute terms
        # (relative bounds fail where b is near 0 after the cancellation)
        atol = 1e-13 if loss == "svm" else 0.0
        np.testing.assert_allclose(s.cache(), cache, rtol=1e-12, atol=atol)
        perm = oracle.permutation(3, trial, d.p)
        P = [32, 1, 500, 77, 32, 250][trial]
        bundle = perm[:P]
        w_o = w.copy()
        s_orc = oracle.step(prob, par, w_o, cache, bundle)
        s_gpu = s.step(bundle, schedule=schedule)
        _compare_step(d, s_gpu, s_orc, bundle, C)
        np.testing.assert_allclose(s.w(), w_o, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(s.cache(), cache, rtol=1e-10, atol=10 * atol)
    s.close()


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("loss", ["lr", "svm"])
def test_step_parity_long_columns_c2(pc, loss, schedule):
    """C2 has columns of up to 20,000 nonzeros (split over many wavefronts)."""
    d = synth.c2()
    prob = oracle.Problem.from_data(d)
    C = 4.0
    par = oracle.Params(loss=loss, C=C)
    s = _solver(pc, d)
    rng = np.random.default_rng(8)
    lens = d.col_lengths()
    heavy = np.argsort(lens)[::-1][:40]
    for trial in range(3):
        w = _random_w(rng, d.p, frac=0.05, scale=0.2) if trial else np.zeros(d.p)
        s.reset(loss, C, w)
        cache = oracle.cache_from_w(prob, loss, w)
        perm = oracle.permutation(9, trial, d.p)
        bundle = np.concatenate([heavy[trial::3], perm[:1024]])
        bundle = bundle[np.sort(np.unique(bundle, return_index=True)[1])]
        w_o = w.copy()
        s_orc = oracle.step(prob, par, w_o, cache, bundle)
        s_gpu = s.step(bundle, schedule=schedule)
        _compare_step(d, s_gpu, s_orc, bundle, C)
        np.testing.assert_allclose(s.w(), w_o, rtol=1e-12, atol=1e-15)
    s.close()


@pytest.mark.parametrize("width", [64, 128, 512])
@pytest.mark.parametrize("loss", ["lr", "svm"])
def test_step_parity_range_widths_c2(pc, loss, width):
    """Every range width of the bundle sweep (pcdn_opts.chunk): g, h, d,
    d^T x and the step against the oracle on bundles with C2's longest
    columns (a column then spans up to 300 ranges of 64 nonzeros)."""
    d = synth.c2()
    prob = oracle.Problem.from_data(d)
    C = 4.0
    par = oracle.Params(loss=loss, C=C)
    s = _solver(pc, d)
    rng = np.random.default_rng(11)
    heavy = np.argsort(d.col_lengths())[::-1][:30]
    for trial in range(2):
        w = _random_w(rng, d.p, frac=0.05, scale=0.2) if trial else np.zeros(d.p)
        s.reset(loss, C, w)
        cache = oracle.cache_from_w(prob, loss, w)
        perm = oracle.permutation(13, trial, d.p)
        bundle = np.concatenate([heavy[trial::2], perm[:2048]])
        bundle = bundle[np.sort(np.unique(bundle, return_index=True)[1])]
        w_o = w.copy()
        s_orc = oracle.step(prob, par, w_o, cache, bundle)
        s_gpu = s.step(bundle, schedule="wide", chunk=width)
        _compare_step(d, s_gpu, s_orc, bundle, C)
        np.testing.assert_allclose(s.w(), w_o, rtol=1e-12, atol=1e-15)
    s.close()


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("loss", ["lr", "svm"])
@pytest.mark.parametrize("zmax", [50.0, 700.0])
def test_step_parity_extreme_margins(pc, loss, schedule, zmax):
    """w scaled so that max_i |x_i^T w| = zmax: e^{w^T x} spans e^{+-50} and
    e^{+-700} (near both ends of the normal doubles), so the logistic
    weights come within one rounding of 0 and 1, h_j falls to the floor nu on
    columns whose rows all sit far out, directions and d^T x grow to ~1e10
    and the line search backtracks 20-odd times (the candidates past the
    first group, both branches of the loss change).  Three empty columns with
    nonzero weights (g = 0, h = nu, d = -w_j) join the bundles.

    Tolerances: g, h, d, d^T x as in every step test; w and the retained
    quantities then inherit them through the update, accumulated over the
    three bundles (w_j + alpha d_j; e^{w^T x_i} e^{alpha d^T x_i}, whose
    relative error is the absolute error of alpha d^T x_i; b_i - y_i alpha
    d^T x_i)."""
    base = synth.c1()
    d = synth.Data(n=base.n, p=base.p + 3,
                   col_ptr=np.concatenate([base.col_ptr, [base.nnz] * 3]).astype(np.int64),
                   row_idx=base.row_idx, val=base.val, y=base.y)
    prob = oracle.Problem.from_data(d)
    C = 1.0
    par = oracle.Params(loss=loss, C=C)
    rng = np.random.default_rng(11)
    w = _random_w(rng, d.p)
    z = oracle.margins(prob, w)
    w *= zmax / np.max(np.abs(z))
    w[-3:] = [0.5, -0.25, 0.0]
    s = _solver(pc, d)
    s.reset(loss, C, w)
    cache = oracle.cache_from_w(prob, loss, w)
    if loss == "lr" and zmax == 700.0:
        assert np.min(cache) < 1e-300 and np.max(cache) > 1e290
    # the retained quantities from w: z_i = x_i^T w in another summation order
    # (error within a few ulps of sum_j |x_ij w_j|), then e^z or 1 - y z
    ulp = np.finfo(float).eps
    tol_c = 4 * ulp * (_abs_X(d) @ np.abs(w) + 1.0)
    _assert_retained(loss, s.cache(), cache, tol_c)
    tol_w = np.zeros(d.p)
    perm = oracle.permutation(21, 0, base.p)
    bundles = [np.concatenate([[d.p - 3, d.p - 2, d.p - 1], perm[:61]]), perm[61:261], perm[261:262]]
    qs = []
    for B in bundles:
        B = np.asarray(B, dtype=np.int32)
        w_o = w.copy()
        s_orc = oracle.step(prob, par, w_o, cache, B)
        s_gpu = s.step(B, schedule=schedule)
        _compare_step(d, s_gpu, s_orc, B, C)
        al = s_orc["alpha"]
        dmax = np.max(np.abs(s_orc["d"]))
        xmax = np.max(np.abs(s_orc["dtx"]))
        tol_w[B] += al * (RTOL * np.abs(s_orc["d"]) + RTOL * dmax)
        tol_c = tol_c + al * (RTOL * np.abs(s_orc["dtx"]) + RTOL * xmax) + 4 * ulp
        assert np.all(np.abs(s.w() - w_o) <= tol_w + 4 * ulp * np.abs(w_o)), B[:3]
        _assert_retained(loss, s.cache(), cache, tol_c)
        qs.append(s_orc["q"])
        w = w_o
    s.close()
    if loss == "lr" and zmax == 700.0:
        assert max(qs) >= 8  # candidates past the first group were taken


def _abs_X(d):
    import scipy.sparse as sp
    return sp.csc_matrix((np.abs(d.val.astype(np.float64)), d.row_idx, d.col_ptr),
                         shape=(d.n, d.p)).tocsr()


def _assert_retained(loss, got, want, tol):
    """Retained quantities within tol: relative for e^{w^T x} (an absolute
    error in w^T x), absolute for b (plus rounding at |b|)."""
    assert np.all(np.isfinite(got)) and np.all(np.isfinite(want))
    if loss == "lr":
        assert np.all(got > 0) and np.all(want > 0)
        err = np.abs(np.log(got) - np.log(want))
        assert np.all(err <= tol), np.max(err - tol)
    else:
        err = np.abs(got - want)
        assert np.all(err <= tol + 4 * np.finfo(float).eps * np.abs(want)), np.max(err - tol)


@pytest.mark.parametrize("zmax", [745.0, 800.0])
def test_reset_rejects_margins_outside_the_doubles(pc, zmax):
    """e^{w^T x_i} past the normal doubles (|w^T x_i| > ~708: 0, a subnormal
    or inf) no longer determines w^T x_i, and the logistic loss of such a
    sample is not representable from it: pcdn_reset reports a numeric error
    rather than run from it.  The squared hinge's b_i stays finite there."""
    from paper_1306_4080_amd import PcdnError
    d = synth.c1()
    prob = oracle.Problem.from_data(d)
    w = _random_w(np.random.default_rng(11), d.p)
    w *= zmax / np.max(np.abs(oracle.margins(prob, w)))
    cache = oracle.cache_from_w(prob, "lr", w)
    assert np.min(cache) < 2.2250738585072014e-308 or np.max(cache) == np.inf
    s = _solver(pc, d)
    with pytest.raises(PcdnError, match="E_NUMERIC"):
        s.reset("lr", 1.0, w)
    s.reset("svm", 1.0, w)  # fine for the SVM
    s.reset("lr", 1.0, 0.5 * w)  # and the context stays usable
    s.close()


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_step_backtracking_and_failure(pc, schedule):
    """Duplicated columns force q > 0; max_ls = 1 forces a failed search."""
    base = synth.tiny(12, n=40, p=4, density=0.8)
    X = base.dense()
    X = np.hstack([X, X[:, :2], 0.5 * X[:, 2:3]])
    d = synth.from_dense(X, base.y)
    prob = oracle.Problem.from_data(d)
    s = _solver(pc, d)
    for loss in ("lr", "svm"):
        for max_ls in (30, 1):
            par = oracle.Params(loss=loss, C=3.0, max_ls=max_ls)
            w = np.zeros(d.p)
            s.reset(loss, 3.0, w)
            cache = oracle.cache_from_w(prob, loss, w)
            qs = []
            for k in range(5):
                B = oracle.permutation(77, k, d.p)
                s_orc = oracle.step(prob, par, w, cache, B)
                s_gpu = s.step(B, max_ls=max_ls, schedule=schedule)
                _compare_step(d, s_gpu, s_orc, B, 3.0)
                np.testing.assert_allclose(s.w(), w, rtol=1e-12, atol=1e-15)
                qs.append(s_orc["q"])
            assert (max(qs) > 0) if max_ls == 30 else (min(qs) == -1)
    s.close()


# --------------------------------------------------------------------------
# whole solves: final objective
# --------------------------------------------------------------------------
def _solve_both(pc, d, loss, C, P, eps, seed=1, max_outer=1000, w0=None, s=None,
                schedule="auto", shrink=False, **reg):
    prob = oracle.Problem.from_data(d)
    w_o, info_o, _ = oracle.solve(prob, oracle.Params(loss=loss, C=C, shrink=shrink, **reg), P=P,
                                  eps=eps, seed=seed, max_outer=max_outer, w0=w0)
    own = s is None
    if own:
        s = _solver(pc, d)
    rc, w_g, info_g = s.solve(C, P, eps, loss, seed=seed, max_outer=max_outer, w0=w0,
                              schedule=schedule, shrink=shrink, **reg)
    if own:
        s.close()
    return (rc, w_g, info_g), (w_o, info_o)


FLOOR = 1e-9  # a decision this close to its threshold (relative) is at the rounding floor


def _assert_solve_parity(g, o, strict=True):
    """Final objective within 1e-6 relative and the same trajectory step for
    step (outer iterations, bundles, nonzeros swept, line-search steps and
    failures).  strict=False (tiny problems, single-coordinate bundles or eps
    near the FP64 rounding floor) admits a different trajectory only where a
    decision sat at the rounding floor: an Armijo or stopping test within
    1e-9 relative of its threshold, in the oracle's run or the GPU's, where
    the two sides' summation orders can decide differently.  Such a flip is
    reported; one with no decision at the floor fails."""
    rc, w_g, ig = g
    w_o, io = o
    print(f"F_gpu={ig['objective']:.15g} F_orc={io['objective']:.15g} outer={ig['outer_iters']}/"
          f"{io['outer_iters']} ls={ig['ls_steps']}/{io['ls_steps']}", flush=True)
    assert ig["objective"] == pytest.approx(io["objective"], rel=RTOL)
    assert ig["converged"] == io["converged"]
    assert ig["subgrad0"] == pytest.approx(io["subgrad0"], rel=1e-12)
    keys = ("outer_iters", "nnz_swept", "bundles", "ls_steps", "ls_fail")
    if all(ig[k] == io[k] for k in keys):
        return
    floor = min(io["min_armijo_margin"], io["min_stop_margin"], ig["min_armijo_margin"],
                ig["min_stop_margin"])
    print(f"ROUNDING-FLIP: outer {ig['outer_iters']} vs {io['outer_iters']}, line-search steps "
          f"{ig['ls_steps']} vs {io['ls_steps']}; smallest decision margin {floor:.3g}",
          flush=True)
    assert not strict, "trajectory differs from the oracle's"
    assert floor < FLOOR, "trajectory differs with no decision at the rounding floor"


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_solve_parity_c1(pc, schedule):
    d = synth.c1()
    g, o = _solve_both(pc, d, "lr", 1.0, 32, 1e-4, schedule=schedule)
    _assert_solve_parity(g, o)
    assert g[0] == 0


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("C,P", [(0.5, 64), (0.5, 1024), (0.5, 8192),
                                 (4.0, 64), (4.0, 1024), (4.0, 8192)])
def test_solve_parity_c2(pc, C, P, schedule):
    d = _c2_cached()
    g, o = _solve_both(pc, d, "lr", C, P, 1e-4, schedule=schedule)
    _assert_solve_parity(g, o)


_C2 = {}


def _c2_cached():
    if "d" not in _C2:
        _C2["d"] = synth.c2()
    return _C2["d"]


def test_solve_parity_c3(pc):
    """Full-size SVM configuration (100,000 x 1,000,000, 12M nonzeros)."""
    d = synth.c3()
    g, o = _solve_both(pc, d, "svm", 1.0, 16384, 1e-3)
    _assert_solve_parity(g, o)


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("loss", ["lr", "svm"])
def test_solve_edge_cases(pc, loss, schedule):
    # empty columns, P = 1, P = p, ragged last bundle
    d = synth.tiny(70, n=50, p=13, density=0.3, empty_cols=(0, 5))
    for P in (1, 4, 13):
        for eps in (1e-4, 1e-8):
            g, o = _solve_both(pc, d, loss, 1.0, P, eps, max_outer=500, schedule=schedule)
            _assert_solve_parity(g, o, strict=False)
    # one sample, one feature
    d1 = synth.from_dense(np.array([[2.0]]), np.array([1], np.int8))
    g, o = _solve_both(pc, d1, loss, 1.0, 1, 1e-10, schedule=schedule)
    _assert_solve_parity(g, o, strict=False)
    # all-empty matrix: w = 0 is optimal
    d0 = synth.Data(n=3, p=4, col_ptr=np.zeros(5, np.int64), row_idx=np.zeros(0, np.int32),
                    val=np.zeros(0, np.float32), y=np.array([1, -1, 1], np.int8))
    g, o = _solve_both(pc, d0, loss, 1.0, 2, 1e-6, schedule=schedule)
    _assert_solve_parity(g, o, strict=False)
    assert g[2]["outer_iters"] == 0 and np.all(g[1] == 0)


# --------------------------------------------------------------------------
# shrinking (opt-in): the partition of each outer iteration covers only the
# features still active after the previous one
# --------------------------------------------------------------------------
@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("loss,eps", [("lr", 1e-4), ("svm", 1e-3)])
def test_shrink_parity_c1(pc, loss, eps, schedule):
    d = synth.c1()
    s = _solver(pc, d)
    g, o = _solve_both(pc, d, loss, 1.0, 32, eps, s=s, schedule=schedule, shrink=True)
    _assert_solve_parity(g, o)
    full = s.solve(1.0, 32, eps, loss, seed=1, max_outer=1000, schedule=schedule)
    s.close()
    # shrinking must have removed work, and the two runs reach the same optimum
    assert g[2]["nnz_swept"] < full[2]["nnz_swept"]
    assert g[2]["objective"] == pytest.approx(full[2]["objective"], rel=1e-3)


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("C,P,strict", [(0.5, 64, True), (4.0, 1024, True), (0.5, 1024, False)])
def test_shrink_parity_c2(pc, C, P, strict, schedule):
    """At C = 0.5, P = 1024 the ~350 active features form one bundle; its
    step leaves a coordinate geometrically approaching zero (d_j = -w_j, only
    alpha < 1 accepted), so the run ends only when a unit step passes an
    Armijo test whose two sides are at the rounding floor (the objective has
    stopped changing at 1e-14 relative well before): the outer iteration at
    which that happens is decided by rounding, on either side."""
    d = _c2_cached()
    g, o = _solve_both(pc, d, "lr", C, P, 1e-4, schedule=schedule, shrink=True)
    _assert_solve_parity(g, o, strict=strict)


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_shrink_step_by_step(pc, schedule):
    """pcdn_iterate with shrinking: after every outer iteration the GPU's
    active set equals the oracle's, so each partition is the same."""
    d = synth.c1()
    prob = oracle.Problem.from_data(d)
    C, P = 1.0, 32
    w_o, info_o, hist = oracle.solve(prob, oracle.Params(loss="lr", C=C, shrink=True), P=P,
                                     eps=1e-4, seed=1, max_outer=6)
    s = _solver(pc, d)
    rc, w_g, info_g = s.solve(C, P, 1e-4, "lr", seed=1, max_outer=6, schedule=schedule,
                              shrink=True)
    assert info_g["outer_iters"] == info_o["outer_iters"] == 6
    assert info_g["nnz_swept"] == info_o["nnz_swept"]
    assert info_g["bundles"] == info_o["bundles"]
    np.testing.assert_allclose(w_g, w_o, rtol=RTOL, atol=RTOL * np.max(np.abs(w_o)))
    s.close()


# --------------------------------------------------------------------------
# separable regularisers: elastic net and ridge in place of the l1 norm
# --------------------------------------------------------------------------
REGS = [{"penalty": "elastic", "l2": 0.5}, {"penalty": "l2", "l2": 0.7}]


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("loss", ["lr", "svm"])
@pytest.mark.parametrize("reg", REGS, ids=["elastic", "ridge"])
def test_regularised_step_parity_c1(pc, reg, loss, schedule):
    d = synth.c1()
    prob = oracle.Problem.from_data(d)
    C = 1.0
    par = oracle.Params(loss=loss, C=C, **reg)
    s = _solver(pc, d)
    rng = np.random.default_rng(6)
    for trial in range(4):
        w = _random_w(rng, d.p) if trial else np.zeros(d.p)
        s.reset(loss, C, w)
        cache = oracle.cache_from_w(prob, loss, w)
        bundle = oracle.permutation(4, trial, d.p)[:[32, 1, 500, 77][trial]]
        w_o = w.copy()
        s_orc = oracle.step(prob, par, w_o, cache, bundle)
        s_gpu = s.step(bundle, schedule=schedule, **reg)
        _compare_step(d, s_gpu, s_orc, bundle, C)
        np.testing.assert_allclose(s.w(), w_o, rtol=1e-12, atol=1e-15)
    s.close()


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("loss,eps", [("lr", 1e-4), ("svm", 1e-3)])
@pytest.mark.parametrize("reg", REGS, ids=["elastic", "ridge"])
def test_regularised_solve_parity_c1(pc, reg, loss, eps, schedule):
    d = synth.c1()
    s = _solver(pc, d)
    g, o = _solve_both(pc, d, loss, 1.0, 32, eps, s=s, schedule=schedule, **reg)
    _assert_solve_parity(g, o)
    assert g[0] == 0
    # pcdn_evaluate reports F with the regulariser the state was solved with
    F, G = s.evaluate()
    assert F == pytest.approx(o[1]["objective"], rel=RTOL)
    assert G == pytest.approx(g[2]["subgrad"], rel=1e-9)
    X, y = d.dense(), d.y.astype(float)
    a, b = oracle.Params(**reg).reg_ab()
    Fd = a * np.abs(g[1]).sum() + 0.5 * b * g[1] @ g[1] + _loss_sum(X, y, g[1], loss)
    assert g[2]["objective"] == pytest.approx(Fd, rel=1e-9)
    s.close()


def _loss_sum(X, y, w, loss):
    m = y * (X @ w)
    if loss == "lr":
        return float(np.logaddexp(0.0, -m).sum())
    return float((np.maximum(1.0 - m, 0.0) ** 2).sum())


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("reg,C,P", [({"penalty": "elastic", "l2": 2.0}, 0.5, 64),
                                     ({"penalty": "l2", "l2": 1.0}, 4.0, 1024)],
                         ids=["elastic", "ridge"])
def test_regularised_solve_parity_c2(pc, reg, C, P, schedule):
    d = _c2_cached()
    g, o = _solve_both(pc, d, "lr", C, P, 1e-4, schedule=schedule, **reg)
    _assert_solve_parity(g, o)


@pytest.mark.parametrize("schedule", SCHEDULES)
def test_elastic_net_with_shrinking_c1(pc, schedule):
    d = synth.c1()
    g, o = _solve_both(pc, d, "lr", 1.0, 32, 1e-4, schedule=schedule, shrink=True,
                       penalty="elastic", l2=0.3)
    _assert_solve_parity(g, o)


def test_regulariser_argument_errors(pc):
    from paper_1306_4080_amd import PcdnError
    d = synth.c1()
    s = _solver(pc, d)
    for bad in ({"penalty": 3, "l2": 1.0}, {"penalty": -1}, {"penalty": "l1", "l2": 0.5},
                {"penalty": "elastic", "l2": 0.0}, {"penalty": "l2", "l2": -1.0},
                {"penalty": "l2", "l2": float("inf")}):
        with pytest.raises(PcdnError, match="E_ARG"):
            s.solve(1.0, 32, 1e-4, "lr", **bad)
    s.close()


@pytest.mark.parametrize("chunk", [64, 128, 512])
def test_chunk_lengths_same_trajectory(pc, chunk):
    """The bundle sweep's range width (pcdn_opts.chunk, nonzeros per
    wavefront; 256 by default) changes only the work split and the order of
    the g_j, h_j sums: C2's long columns at P = 1,024 give the oracle's
    trajectory for every width."""
    d = _c2_cached()
    prob = oracle.Problem.from_data(d)
    w_o, io, _ = oracle.solve(prob, oracle.Params(loss="lr", C=0.5), P=1024, eps=1e-4, seed=1)
    s = _solver(pc, d)
    g = s.solve(0.5, 1024, 1e-4, "lr", seed=1, schedule="wide", chunk=chunk)
    s.close()
    _assert_solve_parity(g, (w_o, io))


def test_chunk_argument_errors(pc):
    from paper_1306_4080_amd import PcdnError
    s = _solver(pc, synth.c1())
    for bad in (1, 32, 100, 1024, -64):
        with pytest.raises(PcdnError, match="E_ARG"):
            s.solve(1.0, 32, 1e-4, "lr", chunk=bad)
    s.close()


def test_warm_start_and_max_outer(pc):
    d = synth.c1()
    prob = oracle.Problem.from_data(d)
    s = _solver(pc, d)
    # hitting max_outer returns PCDN_NOT_CONVERGED with the same state as the oracle
    g, o = _solve_both(pc, d, "lr", 1.0, 32, 1e-12, max_outer=3, s=s)
    _assert_solve_parity(g, o)
    assert g[0] == 1
    # warm start from that point
    g2, o2 = _solve_both(pc, d, "lr", 2.0, 32, 1e-4, w0=o[0], s=s)
    _assert_solve_parity(g2, o2)
    s.close()


# --------------------------------------------------------------------------
# boundary error handling
# --------------------------------------------------------------------------
def test_abi_errors(pc):
    from paper_1306_4080_amd import PcdnError
    d = synth.tiny(3, n=10, p=5, density=0.5)
    s = pc.Solver(device=0)
    with pytest.raises(PcdnError, match="E_STATE"):
        s.p = 5
        s.solve(1.0, 2, 1e-3, "lr")
    bad = d.row_idx.copy()
    j = int(np.flatnonzero(np.diff(d.col_ptr) >= 2)[0])
    lo = d.col_ptr[j]
    bad[lo], bad[lo + 1] = bad[lo + 1], bad[lo]
    with pytest.raises(PcdnError, match="E_CSC"):
        s.load(d.n, d.p, d.col_ptr, bad, d.val, d.y)
    bad = d.row_idx.copy()
    bad[0] = d.n
    with pytest.raises(PcdnError, match="E_CSC"):
        s.load(d.n, d.p, d.col_ptr, bad, d.val, d.y)
    v = d.val.copy()
    v[0] = np.nan
    with pytest.raises(PcdnError, match="E_CSC"):
        s.load(d.n, d.p, d.col_ptr, d.row_idx, v, d.y)
    y = d.y.copy()
    y[0] = 0
    with pytest.raises(PcdnError, match="E_CSC"):
        s.load(d.n, d.p, d.col_ptr, d.row_idx, d.val, y)
    s.load_data(d)
    for args in ((0.0, 2, 1e-3, "lr"), (1.0, 0, 1e-3, "lr"), (1.0, 6, 1e-3, "lr"),
                 (1.0, 2, -1.0, "lr"), (1.0, 2, 1e-3, 7)):
        with pytest.raises(PcdnError, match="E_ARG"):
            s.solve(*args)
    with pytest.raises(PcdnError, match="E_ARG"):
        s.solve(1.0, 2, 1e-3, "lr", max_ls=33)
    s.reset("lr", 1.0)
    with pytest.raises(PcdnError, match="E_ARG"):
        s.step(np.array([0, 0], np.int32))
    with pytest.raises(PcdnError, match="E_ARG"):
        s.step(np.array([5], np.int32))
    # the context stays usable after errors
    rc, w, info = s.solve(1.0, 2, 1e-3, "lr")
    assert rc == 0
    s.close()


@pytest.mark.parametrize("loss", ["lr", "svm"])
def test_bias_feature(pc, loss):
    """pcdn_load_csc_bias appends a constant feature (regularised like the
    others): the solve equals the oracle's on the matrix with that column
    written out, from host and from device arrays."""
    import torch
    from paper_1306_4080_amd import PcdnError
    d = synth.c1()
    db = synth.with_bias(d, 1.0)
    s = pc.Solver(device=0).load_data(d, bias=1.0)
    assert s.p == d.p + 1
    g = s.solve(1.0, 32, 1e-4, loss, seed=2)
    w_o, io, _ = oracle.solve(oracle.Problem.from_data(db), oracle.Params(loss=loss, C=1.0), P=32,
                              eps=1e-4, seed=2)
    _assert_solve_parity(g, (w_o, io))
    assert g[1].shape == (d.p + 1,)
    # device arrays
    dev = {k: torch.from_numpy(getattr(d, k)).cuda() for k in ("col_ptr", "row_idx", "val", "y")}
    s2 = pc.Solver(device=0)
    pc.pcdn_load_csc_bias(s2.ctx, d.n, d.p, dev["col_ptr"], dev["row_idx"], dev["val"], dev["y"], 1.0)
    s2.n, s2.p = d.n, d.p + 1
    g2 = s2.solve(1.0, 32, 1e-4, loss, seed=2)
    assert g2[2]["objective"] == pytest.approx(g[2]["objective"], rel=1e-9)
    with pytest.raises(PcdnError, match="E_ARG"):
        pc.pcdn_load_csc_bias(s2.ctx, d.n, d.p, d.col_ptr, d.row_idx, d.val, d.y, 0.0)
    bad = d.col_ptr.copy()
    bad[-1] += 1
    with pytest.raises(PcdnError, match="E_CSC"):
        pc.pcdn_load_csc_bias(s2.ctx, d.n, d.p, bad, d.row_idx, d.val, d.y, 1.0)
    s.close()
    s2.close()
