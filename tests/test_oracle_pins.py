"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test names the passage of the paper it checks.  The references in
``tests/_refs.py`` are independent computations (dense numpy, mpmath, sign
enumeration, Algorithm 1 with direct objective evaluation).
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth
from tests import _refs as R

HERE = os.path.dirname(os.path.abspath(__file__))


def _prob(d):
    return oracle.Problem.from_data(d)


# --------------------------------------------------------------------------
# random partition (eq. (8), Algorithm 3) and its generator
# --------------------------------------------------------------------------
def test_splitmix64_published_vector():
    """The counter-based generator reproduces SplitMix64's published outputs."""
    path = os.path.join(HERE, "golden", "splitmix64_seed1234567.txt")
    want = [int(l) for l in open(path) if l.strip() and not l.startswith("#")]
    got = [oracle.splitmix64(1234567, i) for i in range(len(want))]
    assert got == want


def _py_splitmix64(s, i):
    M = (1 << 64) - 1
    z = (s + (i + 1) * 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def test_permutation_matches_its_definition():
    """Outer iteration k sorts features by (upper 32 bits of output j of the
    stream seeded with output k of the stream seeded with `seed`, j); built here
    in pure Python integers from the published generator definition."""
    path = os.path.join(HERE, "golden", "splitmix64_seed1234567.txt")
    want = [int(l) for l in open(path) if l.strip() and not l.startswith("#")]
    assert [_py_splitmix64(1234567, i) for i in range(5)] == want
    for seed, k, p in ((0, 0, 17), (20130616, 3, 1000), (2**64 - 1, 7, 257)):
        stream = _py_splitmix64(seed, k)
        keys = [(_py_splitmix64(stream, j) >> 32, j) for j in range(p)]
        ref = [j for _, j in sorted(keys)]
        assert oracle.permutation(seed, k, p).tolist() == ref


def test_permutation_is_permutation_and_seeded():
    for p in (1, 2, 7, 1000):
        a = oracle.permutation(5, 0, p)
        assert sorted(a.tolist()) == list(range(p))
        assert np.array_equal(a, oracle.permutation(5, 0, p))
    assert not np.array_equal(oracle.permutation(5, 0, 1000), oracle.permutation(5, 1, 1000))
    assert not np.array_equal(oracle.permutation(5, 0, 1000), oracle.permutation(6, 0, 1000))


@pytest.mark.parametrize("P", [1, 2, 5, 13, 40])
def test_bundle_max_lambda_matches_lemma1a_closed_form(P):
    """Lemma 1(a) (appendix, closed form f(P)): the mean over partitions of
    max_{j in B} ||x^j||^2 for the first bundle equals f(P) when bundles are
    uniform random P-subsets; checked to 4 standard errors over 10^4 draws."""
    rng = np.random.default_rng(3)
    p = 40
    lams = rng.gamma(2.0, 1.0, p)
    f = R.lemma1a_expected_max(lams, P)
    N = 10000
    m = np.array([lams[oracle.permutation(11, k, p)[:P]].max() for k in range(N)])
    se = m.std(ddof=1) / math.sqrt(N) if P < p else 0.0
    assert abs(m.mean() - f) <= 4 * se + 1e-12
    if P == p:
        assert f == pytest.approx(lams.max(), rel=1e-14)


def test_lemma1a_closed_form_is_monotone():
    rng = np.random.default_rng(4)
    lams = rng.gamma(1.0, 1.0, 30)
    f = [R.lemma1a_expected_max(lams, P) for P in range(1, 31)]
    assert all(b >= a - 1e-12 for a, b in zip(f, f[1:]))
    assert all(b / (P + 2) <= a / (P + 1) + 1e-12 for P, (a, b) in enumerate(zip(f, f[1:])))
    assert R.lemma1a_expected_max([2.0] * 10, 4) == pytest.approx(2.0)


# --------------------------------------------------------------------------
# one-dimensional Newton direction (eqs. (4)-(5))
# --------------------------------------------------------------------------
def _direction_cases():
    rng = np.random.default_rng(7)
    cases = []
    for _ in range(300):
        g = rng.uniform(-5, 5)
        h = 10 ** rng.uniform(-3, 3)
        w = rng.uniform(-3, 3) * (rng.random() < 0.7)
        cases.append((g, h, w))
    # boundary cases: g + 1 = h w, g - 1 = h w, w = 0 with |g| = 1
    cases += [(1.0, 2.0, 1.0), (-3.0, 2.0, -1.0), (1.0, 1.0, 0.0), (-1.0, 1.0, 0.0),
              (0.0, 1e-12, 0.0), (0.5, 1.0, 0.0), (2.0, 1.0, 0.0), (-2.0, 0.5, 0.0)]
    return cases


def test_direction_minimises_subproblem():
    """The closed form returns the minimiser of g d + h d^2/2 + |w + d| (eq. (4)),
    checked against golden-section minimisation and the kink at d = -w."""
    for g, h, w in _direction_cases():
        d = oracle.newton_direction(g, h, w)
        f = lambda x: R.subproblem_value(g, h, w, x)
        scale = (abs(g) + 1.0) / h + abs(w) + 1.0
        bf = R.golden_section_min(f, -scale, scale)
        if f(-w) <= f(bf):
            bf = -w
        assert f(d) <= f(bf) + 1e-12 * (1.0 + abs(f(bf))), (g, h, w, d, bf)
        assert abs(d - bf) <= 1e-5 * (1.0 + abs(bf)), (g, h, w, d, bf)


def test_direction_zero_at_optimum():
    # w = 0 and |g| <= 1: zero is optimal for eq. (4)
    for g in (-1.0, -0.3, 0.0, 0.9, 1.0):
        assert oracle.newton_direction(g, 3.0, 0.0) == 0.0


# --------------------------------------------------------------------------
# gradient / Hessian diagonal from the retained quantities (eq. (11); SVM
# generalised Hessian in the proof of Lemma 1(b))
# --------------------------------------------------------------------------
@pytest.mark.parametrize("loss", ["lr", "svm"])
def test_grad_hess_match_multiprecision_finite_differences(loss):
    d = synth.tiny(21, n=25, p=5, density=0.7)
    X, y = d.dense(), d.y.astype(float)
    prob = _prob(d)
    rng = np.random.default_rng(1)
    w = rng.normal(0, 0.4, d.p)
    C = 1.7
    par = oracle.Params(loss=loss, C=C)
    cache = oracle.cache_from_w(prob, loss, w)
    g, h = oracle.grad_hess(prob, par, cache, np.arange(d.p))
    for j in range(d.p):
        gf, hf = R.grad_hess_fd(X, y, w, C, loss, j)
        assert g[j] == pytest.approx(gf, rel=1e-9, abs=1e-12)
        assert h[j] == pytest.approx(hf, rel=1e-7, abs=1e-10)


@pytest.mark.parametrize("loss,theta", [("lr", 0.25), ("svm", 2.0)])
def test_hessian_bounds_lemma1b(loss, theta):
    """Lemma 1(b): 0 < h_j <= theta C ||x^j||^2 (nu-floored for empty columns)."""
    d = synth.tiny(5, n=60, p=12, density=0.3, empty_cols=(3,))
    prob = _prob(d)
    rng = np.random.default_rng(2)
    C = 0.8
    par = oracle.Params(loss=loss, C=C)
    colsq = np.array([np.sum(d.val[d.col_ptr[j]:d.col_ptr[j + 1]].astype(float) ** 2)
                      for j in range(d.p)])
    for scale in (0.0, 0.5, 3.0):
        w = rng.normal(0, scale, d.p)
        cache = oracle.cache_from_w(prob, loss, w)
        g, h = oracle.grad_hess(prob, par, cache, np.arange(d.p))
        assert np.all(h > 0)
        assert np.all(h <= theta * C * colsq * (1 + 1e-12) + 1e-12)
        assert h[3] == 1e-12 and g[3] == 0.0


def test_grad_at_zero_closed_form():
    """At w = 0: LR g_j = -C/2 sum_i y_i x_ij, h_j = C/4 ||x^j||^2;
    SVM g_j = -2C sum_i y_i x_ij, h_j = 2C ||x^j||^2."""
    d = synth.tiny(8, n=50, p=9, density=0.5)
    X, y = d.dense(), d.y.astype(float)
    prob = _prob(d)
    for loss, gk, hk in (("lr", -0.5, 0.25), ("svm", -2.0, 2.0)):
        C = 1.3
        par = oracle.Params(loss=loss, C=C)
        g, h = oracle.grad_hess(prob, par, np.ones(d.n), np.arange(d.p))
        np.testing.assert_allclose(g, gk * C * (X.T @ y), rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(h, hk * C * (X * X).sum(0), rtol=1e-13)


# --------------------------------------------------------------------------
# descent condition from retained quantities (eq. (10))
# --------------------------------------------------------------------------
def test_loss_change_matches_multiprecision_across_ranges():
    Es = [1e-300, 1e-40, 1e-5, 0.3, 1.0, 2.5, 1e5, 1e40, 1e300]
    As = [-1000.0, -50.0, -1.0, -1e-9, 0.0, 1e-9, 1.0, 50.0, 1000.0]
    for E in Es:
        for a in As:
            for y in (1, -1):
                got = oracle.loss_change("lr", E, y, a)
                want = float(R.loss_change_mp("lr", E, y, a))
                assert abs(got - want) <= 1e-13 * abs(want) + 2e-15 * abs(a) + 1e-300, (E, a, y)
    for b in [-3.0, -1e-9, 0.0, 1e-9, 0.7, 1.0, 4.0]:
        for a in [-5.0, -0.5, 0.0, 0.3, 2.0]:
            for y in (1, -1):
                got = oracle.loss_change("svm", b, y, a)
                want = float(R.loss_change_mp("svm", b, y, a))
                assert abs(got - want) <= 1e-14 * (b * b + a * a + 1e-300), (b, a, y)


@pytest.mark.parametrize("loss", ["lr", "svm"])
def test_step_dF_equals_objective_difference(loss):
    """The accepted dF (eq. (10), retained quantities) equals F(w+alpha d) - F(w)
    recomputed from X in multiprecision, and the Armijo rule eq. (6) holds."""
    d = synth.tiny(31, n=30, p=6, density=0.6)
    X, y = d.dense(), d.y.astype(float)
    prob = _prob(d)
    par = oracle.Params(loss=loss, C=2.0)
    rng = np.random.default_rng(9)
    w = rng.normal(0, 0.3, d.p) * (rng.random(d.p) < 0.6)
    cache = oracle.cache_from_w(prob, loss, w)
    for bundle in ([0, 2, 4], [1, 3, 5], [5], list(range(6))):
        w_old = w.copy()
        s = oracle.step(prob, par, w, cache, bundle)
        assert s["q"] >= 0
        dmp = float(R.F_mp(X, y, w, 2.0, loss) - R.F_mp(X, y, w_old, 2.0, loss))
        assert s["dF"] == pytest.approx(dmp, rel=1e-9, abs=1e-12)
        assert s["dF"] <= par.sigma * s["alpha"] * s["delta"] + 1e-15
        # d^T x_i from the dense product
        dfull = np.zeros(d.p)
        dfull[bundle] = s["d"]
        np.testing.assert_allclose(s["dtx"], X @ dfull, rtol=1e-13, atol=1e-14)
        # w moved by alpha d on the bundle only
        np.testing.assert_allclose(w - w_old, s["alpha"] * dfull, rtol=0, atol=1e-15)


# --------------------------------------------------------------------------
# trajectory invariants: Lemma 1(c), Theorem 1 (safe form), cache drift
# --------------------------------------------------------------------------
def _dup_problem(seed):
    """Correlated columns (exact duplicates) so that full-bundle steps must backtrack."""
    d = synth.tiny(seed, n=40, p=4, density=0.8)
    X = d.dense()
    X = np.hstack([X, X[:, :2], 0.5 * X[:, 2:3]])
    return synth.from_dense(X, d.y)


@pytest.mark.parametrize("loss,theta", [("lr", 0.25), ("svm", 2.0)])
def test_trajectory_invariants(loss, theta):
    d = _dup_problem(12)
    X, y = d.dense(), d.y.astype(float)
    prob = _prob(d)
    C = 3.0
    par = oracle.Params(loss=loss, C=C)
    w = np.zeros(d.p)
    cache = oracle.cache_from_w(prob, loss, w)
    F_prev = R.F_dense(X, y, w, C, loss)
    backtracked = 0
    for k in range(6):
        perm = oracle.permutation(77, k, d.p)
        for P in (d.p,):
            for t in range(0, d.p, P):
                B = perm[t:t + P]
                s = oracle.step(prob, par, w, cache, B)
                H = s["h"]
                dHd = float(np.sum(H * s["d"] ** 2))
                # Lemma 1(c): Delta <= (gamma - 1) d^T H d, F non-increasing
                assert s["delta"] <= (par.gamma - 1.0) * dHd + 1e-12 * (1 + abs(dHd))
                F_now = R.F_dense(X, y, w, C, loss)
                assert F_now <= F_prev + 1e-12 * abs(F_prev)
                F_prev = F_now
                # Theorem 1, safe form: alpha >= min(1, beta * abar)
                XB = X[:, B]
                lmax = np.linalg.norm(XB, 2) ** 2
                abar = 2 * H.min() * (1 - par.sigma + par.sigma * par.gamma) / (theta * C * lmax)
                assert s["alpha"] >= min(1.0, par.beta * abar) * (1 - 1e-12)
                backtracked += s["q"] > 0
    assert backtracked > 0  # the duplicated columns force backtracking
    # retained e^{w^T x} / b stay within 1e-10 of a fresh recomputation
    fresh = oracle.cache_from_w(prob, loss, w)
    np.testing.assert_allclose(cache, fresh, rtol=1e-10, atol=1e-12)


def test_cache_objective_matches_direct_objective_on_c1():
    d = synth.c1()
    prob = _prob(d)
    par = oracle.Params(loss="lr", C=1.0)
    w, info, trace = oracle.solve(prob, par, P=32, eps=1e-4, seed=1)
    assert info["objective"] == pytest.approx(oracle.objective_direct(prob, par, w), rel=1e-12)
    assert info["objective"] == pytest.approx(R.F_dense(d.dense(), d.y.astype(float), w, 1.0, "lr"),
                                              rel=1e-12)
    fresh = oracle.cache_from_w(prob, "lr", w)
    assert np.all(np.diff(trace) <= 1e-12 * abs(trace[0]))


# --------------------------------------------------------------------------
# optimality: brute force on tiny problems, KKT, CDN as P = 1
# --------------------------------------------------------------------------
@pytest.mark.parametrize("loss", ["lr", "svm"])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_final_objective_matches_brute_force_optimum(loss, seed):
    d = synth.tiny(100 + seed, n=30, p=4, density=0.8, flip=0.15)
    X, y = d.dense(), d.y.astype(float)
    prob = _prob(d)
    C = [0.3, 1.0, 2.5][seed - 1]
    Fstar, wstar = R.brute_force_optimum(X, y, C, loss)
    for P in (1, 2, 4):
        par = oracle.Params(loss=loss, C=C)
        w, info, _ = oracle.solve(prob, par, P=P, eps=1e-12, seed=seed, max_outer=5000)
        assert info["converged"] == 1
        assert info["objective"] == pytest.approx(Fstar, rel=1e-9, abs=1e-12), (P, w, wstar)


@pytest.mark.parametrize("loss", ["lr", "svm"])
def test_kkt_at_convergence(loss):
    """At the returned w the optimality conditions of eq. (1) hold: |g_j + sign(w_j)|
    is small where w_j != 0 and |g_j| <= 1 where w_j = 0 (g from a dense formula)."""
    d = synth.c1() if loss == "lr" else synth.tiny(41, n=300, p=80, density=0.1, binary=True)
    X, y = d.dense(), d.y.astype(float)
    prob = _prob(d)
    C = 1.0
    par = oracle.Params(loss=loss, C=C)
    w, info, _ = oracle.solve(prob, par, P=16, eps=1e-8, seed=4, max_outer=3000)
    assert info["converged"] == 1
    z = X @ w
    if loss == "lr":
        err = 1.0 / (1.0 + np.exp(y * z))
        g = -C * X.T @ (y * err)
    else:
        b = 1.0 - y * z
        g = -2.0 * C * X.T @ (y * b * (b > 0))
    G0 = info["subgrad0"]
    nz = w != 0
    assert np.all(np.abs(g[nz] + np.sign(w[nz])) <= 1e-6 * G0)
    assert np.all(np.abs(g[~nz]) <= 1.0 + 1e-6 * G0)
    # reference norm at w = 0 from the dense gradient
    g0 = (-0.5 if loss == "lr" else -2.0) * C * X.T @ y
    assert G0 == pytest.approx(np.sum(np.maximum(np.abs(g0) - 1.0, 0.0)), rel=1e-12)


@pytest.mark.parametrize("loss", ["lr", "svm"])
def test_P1_equals_independent_cdn(loss):
    """With P = 1 PCDN is CDN (Algorithm 1): same coordinate order, 1-D line
    search by direct multiprecision objective evaluation, no retained quantities."""
    d = synth.tiny(55, n=40, p=6, density=0.6)
    X, y = d.dense(), d.y.astype(float)
    prob = _prob(d)
    C, K, seed = 1.5, 4, 9
    orders = [oracle.permutation(seed, k, d.p) for k in range(K)]
    w_cdn = R.cdn(X, y, C, loss, orders)
    par = oracle.Params(loss=loss, C=C)
    w, info, _ = oracle.solve(prob, par, P=1, eps=0.0, seed=seed, max_outer=K)
    assert info["outer_iters"] == K
    np.testing.assert_allclose(w, w_cdn, rtol=1e-6, atol=1e-8)


def test_single_bundle_P_equals_p_converges():
    d = synth.tiny(61, n=80, p=20, density=0.3)
    prob = _prob(d)
    for loss in ("lr", "svm"):
        par = oracle.Params(loss=loss, C=1.0)
        w, info, tr = oracle.solve(prob, par, P=d.p, eps=1e-6, seed=2, max_outer=20000)
        assert info["converged"] == 1 and info["bundles"] == info["outer_iters"]
        assert np.all(np.diff(tr) <= 1e-12 * abs(tr[0]))


def test_solve_is_deterministic_and_seed_independent_at_optimum():
    d = synth.tiny(62, n=60, p=10, density=0.4)
    prob = _prob(d)
    par = oracle.Params(loss="lr", C=1.0)
    w1, i1, _ = oracle.solve(prob, par, P=3, eps=1e-10, seed=1, max_outer=5000)
    w1b, i1b, _ = oracle.solve(prob, par, P=3, eps=1e-10, seed=1, max_outer=5000)
    w2, i2, _ = oracle.solve(prob, par, P=3, eps=1e-10, seed=2, max_outer=5000)
    assert np.array_equal(w1, w1b) and i1 == i1b
    assert i1["objective"] == pytest.approx(i2["objective"], rel=1e-10)


def test_zero_is_optimal_returns_zero_and_warm_start():
    """If ||grad^S F(0)||_1 = 0 the zero vector is returned; a warm start at the
    optimum stops before any outer iteration."""
    d = synth.tiny(63, n=30, p=5, density=0.5)
    prob = _prob(d)
    par = oracle.Params(loss="lr", C=1e-4)
    w, info, _ = oracle.solve(prob, par, P=2, eps=1e-6, seed=1, w0=np.ones(5))
    assert info["subgrad0"] == 0.0 and np.all(w == 0) and info["outer_iters"] == 0
    par = oracle.Params(loss="lr", C=1.0)
    w, info, _ = oracle.solve(prob, par, P=2, eps=1e-6, seed=1)
    w2, info2, _ = oracle.solve(prob, par, P=2, eps=1e-6, seed=1, w0=w)
    assert info2["outer_iters"] == 0 and np.array_equal(w, w2)


def test_ls_failure_leaves_state_unchanged():
    """With max_ls = 1 and duplicated columns the unit step is rejected: the
    inner iteration reports q = -1 and w, caches are untouched."""
    d = _dup_problem(12)
    prob = _prob(d)
    par = oracle.Params(loss="lr", C=3.0, max_ls=1)
    w = np.zeros(d.p)
    cache = oracle.cache_from_w(prob, "lr", w)
    found = False
    for k in range(5):
        B = oracle.permutation(77, k, d.p)
        w0, c0 = w.copy(), cache.copy()
        s = oracle.step(prob, par, w, cache, B)
        if s["q"] < 0:
            found = True
            assert np.array_equal(w, w0) and np.array_equal(cache, c0) and s["alpha"] == 0.0
            break
    assert found


# --------------------------------------------------------------------------
# shrinking (an outer-iteration active set; off by default)
# --------------------------------------------------------------------------
def test_permutation_active_matches_its_definition():
    """Active features keep their keys (capped at 2^32 - 2), inactive ones
    take 2^32 - 1; built here in pure Python integers: the active features
    lead, in the order of the full permutation."""
    rng = np.random.default_rng(3)
    for seed, k, p in ((0, 0, 17), (20130616, 3, 1000), (2**64 - 1, 7, 257)):
        active = (rng.random(p) < 0.3).astype(np.int8)
        stream = _py_splitmix64(seed, k)
        keys = []
        for j in range(p):
            key = _py_splitmix64(stream, j) >> 32
            key = min(key, 2**32 - 2) if active[j] else 2**32 - 1
            keys.append((key, j))
        ref = [j for _, j in sorted(keys)]
        perm, n_act = oracle.permutation_active(seed, k, active)
        assert perm.tolist() == ref and n_act == int(active.sum())
        full = oracle.permutation(seed, k, p).tolist()
        assert perm[:n_act].tolist() == [j for j in full if active[j]]


@pytest.mark.parametrize("loss", ["lr", "svm"])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_shrinking_reaches_brute_force_optimum(loss, seed):
    d = synth.tiny(100 + seed, n=30, p=4, density=0.8, flip=0.15)
    X, y = d.dense(), d.y.astype(float)
    C = [0.3, 1.0, 2.5][seed - 1]
    Fstar, _ = R.brute_force_optimum(X, y, C, loss)
    for P in (1, 2, 4):
        par = oracle.Params(loss=loss, C=C, shrink=True)
        w, info, _ = oracle.solve(_prob(d), par, P=P, eps=1e-12, seed=seed, max_outer=5000)
        assert info["converged"] == 1
        assert info["objective"] == pytest.approx(Fstar, rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("loss", ["lr", "svm"])
def test_shrinking_kkt_monotone_and_less_work(loss):
    """With shrinking the returned w satisfies the optimality conditions (a
    dense gradient), F never increases, the final F agrees with the solve
    without shrinking to the accuracy eps implies, and fewer nonzeros are
    swept (the solution is sparse)."""
    d = synth.c1() if loss == "lr" else synth.tiny(41, n=300, p=80, density=0.1, binary=True)
    X, y = d.dense(), d.y.astype(float)
    prob = _prob(d)
    C = 1.0
    base_w, base, _ = oracle.solve(prob, oracle.Params(loss=loss, C=C), P=16, eps=1e-8, seed=4,
                                   max_outer=3000)
    w, info, trace = oracle.solve(prob, oracle.Params(loss=loss, C=C, shrink=True), P=16, eps=1e-8,
                                  seed=4, max_outer=3000)
    assert info["converged"] == 1
    z = X @ w
    if loss == "lr":
        g = -C * X.T @ (y / (1.0 + np.exp(y * z)))
    else:
        b = 1.0 - y * z
        g = -2.0 * C * X.T @ (y * b * (b > 0))
    G0 = info["subgrad0"]
    nz = w != 0
    assert np.all(np.abs(g[nz] + np.sign(w[nz])) <= 1e-6 * G0)
    assert np.all(np.abs(g[~nz]) <= 1.0 + 1e-6 * G0)
    t = trace[:info["outer_iters"]]
    assert np.all(np.diff(t) <= 1e-12 * np.abs(t[:-1]))
    assert info["objective"] == pytest.approx(base["objective"], rel=1e-8)
    assert info["nnz_swept"] < base["nnz_swept"]


# --------------------------------------------------------------------------
# separable regularisers (the generalisation in the conclusion, Sec. 6):
# R(w) = sum_j a |w_j| + (b/2) w_j^2 in place of ||w||_1 in eqs. (1), (4),
# (6), (7); ridge a = 0, elastic net a = 1, b > 0
# --------------------------------------------------------------------------
REGS = [("elastic", 1.0, 0.5), ("elastic", 1.0, 3.0), ("l2", 0.0, 0.7)]


@pytest.mark.parametrize("a,b", [(1.0, 0.5), (1.0, 3.0), (0.0, 0.7), (0.0, 5.0), (1.0, 0.0)])
def test_regularised_direction_minimises_subproblem(a, b):
    """The closed form returns the minimiser of g d + h d^2/2 + a|w+d| +
    (b/2)(w+d)^2, against golden-section minimisation and the kink at -w."""
    cases = _direction_cases() + [(a + 0.7 * 2.0, 2.0, 0.7), (-a - 3.0, 3.0, -1.0)]
    for g, h, w in cases:
        d = oracle.newton_direction(g, h, w, a, b)
        f = lambda x: R.subproblem_value(g, h, w, x, a, b)
        scale = (abs(g) + a) / h + abs(w) + 1.0
        bf = R.golden_section_min(f, -scale, scale)
        if f(-w) <= f(bf):
            bf = -w
        assert f(d) <= f(bf) + 1e-12 * (1.0 + abs(f(bf))), (g, h, w, d, bf)
        assert abs(d - bf) <= 1e-5 * (1.0 + abs(bf)), (g, h, w, d, bf)
        if b == 0.0 and a == 1.0:
            assert d == oracle.newton_direction(g, h, w)


@pytest.mark.parametrize("loss", ["lr", "svm"])
@pytest.mark.parametrize("pen,a,b", REGS)
def test_regularised_step_dF_equals_objective_difference(loss, pen, a, b):
    """The accepted dF equals F(w + alpha d) - F(w) of the regularised
    objective recomputed from X in multiprecision; eq. (6) holds with Delta."""
    d = synth.tiny(32, n=30, p=6, density=0.6)
    X, y = d.dense(), d.y.astype(float)
    prob = _prob(d)
    par = oracle.Params(loss=loss, C=2.0, penalty=pen, l2=b)
    rng = np.random.default_rng(10)
    w = rng.normal(0, 0.3, d.p) * (rng.random(d.p) < 0.6)
    cache = oracle.cache_from_w(prob, loss, w)
    for bundle in ([0, 2, 4], [1, 3, 5], [5], list(range(6))):
        w_old = w.copy()
        s = oracle.step(prob, par, w, cache, bundle)
        assert s["q"] >= 0
        dmp = float(R.F_mp(X, y, w, 2.0, loss, a=a, b=b) - R.F_mp(X, y, w_old, 2.0, loss, a=a, b=b))
        assert s["dF"] == pytest.approx(dmp, rel=1e-9, abs=1e-12)
        assert s["dF"] <= par.sigma * s["alpha"] * s["delta"] + 1e-15
        # Delta from its definition with R in place of the l1 norm
        wb, dd, g, h = w_old[bundle], s["d"], s["g"], s["h"]
        reg = lambda u: a * np.abs(u) + 0.5 * b * u * u
        assert s["delta"] == pytest.approx(float(np.sum(g * dd + reg(wb + dd) - reg(wb))),
                                           rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("loss", ["lr", "svm"])
@pytest.mark.parametrize("seed", [1, 2])
@pytest.mark.parametrize("b", [0.5, 3.0])
def test_elastic_net_reaches_brute_force_optimum(loss, seed, b):
    d = synth.tiny(110 + seed, n=30, p=4, density=0.8, flip=0.15)
    X, y = d.dense(), d.y.astype(float)
    prob = _prob(d)
    C = [0.8, 2.5][seed - 1]
    Fstar, wstar = R.brute_force_optimum(X, y, C, loss, 1.0, b)
    for P in (1, 2, 4):
        par = oracle.Params(loss=loss, C=C, penalty="elastic", l2=b)
        w, info, _ = oracle.solve(prob, par, P=P, eps=1e-12, seed=seed, max_outer=5000)
        assert info["converged"] == 1
        assert info["objective"] == pytest.approx(Fstar, rel=1e-9, abs=1e-12), (P, w, wstar)
        assert info["objective"] == pytest.approx(R.F_dense(X, y, w, C, loss, 1.0, b), rel=1e-12)


@pytest.mark.parametrize("loss", ["lr", "svm"])
@pytest.mark.parametrize("b", [0.1, 2.0])
def test_ridge_matches_newton_optimum(loss, b):
    """Ridge (a = 0) is smooth and strongly convex: PCDN reaches the optimum
    that Newton's method finds with every feature at once."""
    d = synth.tiny(120, n=200, p=30, density=0.2)
    X, y = d.dense(), d.y.astype(float)
    prob = _prob(d)
    C = 1.0
    Fstar, wstar = R.ridge_optimum(X, y, C, loss, b)
    for P in (1, 8, 30):
        par = oracle.Params(loss=loss, C=C, penalty="l2", l2=b)
        w, info, _ = oracle.solve(prob, par, P=P, eps=1e-11, seed=3, max_outer=20000)
        assert info["converged"] == 1
        assert info["objective"] == pytest.approx(Fstar, rel=1e-10)
        np.testing.assert_allclose(w, wstar, rtol=1e-5, atol=1e-7 * np.abs(wstar).max())
        # stopping reference at w = 0 is ||grad L(0)||_1 (no soft threshold)
        g0 = (-0.5 if loss == "lr" else -2.0) * C * X.T @ y
        assert info["subgrad0"] == pytest.approx(np.abs(g0).sum(), rel=1e-12)


@pytest.mark.parametrize("loss", ["lr", "svm"])
@pytest.mark.parametrize("pen,a,b", REGS)
def test_regularised_P1_equals_independent_cdn(loss, pen, a, b):
    """P = 1 is CDN (Algorithm 1) on the regularised objective: 1-D subproblem
    minimised numerically, line search by direct multiprecision F."""
    d = synth.tiny(56, n=40, p=6, density=0.6)
    X, y = d.dense(), d.y.astype(float)
    prob = _prob(d)
    C, K, seed = 1.5, 4, 9
    orders = [oracle.permutation(seed, k, d.p) for k in range(K)]
    w_cdn = R.cdn(X, y, C, loss, orders, a=a, b=b)
    par = oracle.Params(loss=loss, C=C, penalty=pen, l2=b)
    w, info, _ = oracle.solve(prob, par, P=1, eps=0.0, seed=seed, max_outer=K)
    assert info["outer_iters"] == K
    np.testing.assert_allclose(w, w_cdn, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("loss", ["lr", "svm"])
@pytest.mark.parametrize("shrink", [False, True])
def test_elastic_net_kkt_and_monotone_on_c1(loss, shrink):
    """Elastic net on C1 (and a small SVM problem), with and without
    shrinking: F never increases and the optimality conditions hold at the
    returned w with a dense gradient: |G_j + sign(w_j)| small where w_j != 0,
    |G_j| <= 1 where w_j = 0, G = grad L + b w."""
    d = synth.c1() if loss == "lr" else synth.tiny(41, n=300, p=80, density=0.1, binary=True)
    X, y = d.dense(), d.y.astype(float)
    prob = _prob(d)
    C, b = 1.0, 0.8
    par = oracle.Params(loss=loss, C=C, penalty="elastic", l2=b, shrink=shrink)
    w, info, trace = oracle.solve(prob, par, P=16, eps=1e-8, seed=4, max_outer=3000)
    assert info["converged"] == 1
    assert np.all(np.diff(trace) <= 1e-12 * abs(trace[0]))
    z = X @ w
    if loss == "lr":
        g = -C * X.T @ (y / (1.0 + np.exp(y * z)))
    else:
        bb = 1.0 - y * z
        g = -2.0 * C * X.T @ (y * bb * (bb > 0))
    G = g + b * w
    G0 = info["subgrad0"]
    nz = w != 0
    assert np.all(np.abs(G[nz] + np.sign(w[nz])) <= 1e-6 * G0)
    assert np.all(np.abs(G[~nz]) <= 1.0 + 1e-6 * G0)
    assert info["objective"] == pytest.approx(R.F_dense(X, y, w, C, loss, 1.0, b), rel=1e-12)


@pytest.mark.parametrize("loss", ["lr", "svm"])
def test_ridge_shrinking_leaves_nothing_out(loss):
    """With a = 0 the shrinking threshold a - M/n is <= 0: every feature,
    including empty columns that keep w_j = 0, stays active, so the shrinking
    solve is the plain one step for step."""
    d = synth.tiny(121, n=120, p=23, density=0.25, empty_cols=(0, 7, 8, 15))
    prob = _prob(d)
    runs = []
    for shrink in (False, True):
        par = oracle.Params(loss=loss, C=1.0, penalty="l2", l2=0.3, shrink=shrink)
        runs.append(oracle.solve(prob, par, P=4, eps=1e-9, seed=2, max_outer=5000))
    (w0, i0, _), (w1, i1, _) = runs
    assert i0["converged"] == i1["converged"] == 1
    for k in ("outer_iters", "bundles", "ls_steps", "nnz_swept"):
        assert i0[k] == i1[k], k
    assert np.array_equal(w0, w1)
