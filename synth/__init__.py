"""Seeded synthetic inputs for PCDN, shared by the oracle tests, the GPU tests and the bench.

This module only draws data; it holds none of the method's arithmetic.  The
paper's LIBSVM benchmark sets (Sec. 5.1, Table 2) are not available, so these
generators stand in for its two regimes: text-like normalised tf-idf data
(real-sim, rcv1, news20) and huge sparse binary data (kdda, webspam).

Every generator is a pure function of its seed.  Output is CSC with sorted,
duplicate-free row indices in each column, fp32 values and int8 labels +-1.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 20130616


@dataclass
class Data:
    n: int
    p: int
    col_ptr: np.ndarray  # int64[p+1]
    row_idx: np.ndarray  # int32[nnz]
    val: np.ndarray      # float32[nnz]
    y: np.ndarray        # int8[n]
    w_star: np.ndarray = None
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col_ptr[-1])

    def col_lengths(self) -> np.ndarray:
        return np.diff(self.col_ptr)

    def dense(self) -> np.ndarray:
        """Dense float64 copy of X (small problems only)."""
        X = np.zeros((self.n, self.p))
        for j in range(self.p):
            lo, hi = self.col_ptr[j], self.col_ptr[j + 1]
            X[self.row_idx[lo:hi], j] = self.val[lo:hi]
        return X


def from_triplets(n, p, rows, cols, vals, y, w_star=None, meta=None) -> Data:
    """Assemble CSC from (row, col, value) triplets with no duplicate (row, col)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.lexsort((rows, cols))
    rows, cols = rows[order], cols[order]
    vals = np.asarray(vals, dtype=np.float32)[order]
    counts = np.bincount(cols, minlength=p)
    col_ptr = np.zeros(p + 1, dtype=np.int64)
    np.cumsum(counts, out=col_ptr[1:])
    return Data(n=n, p=p, col_ptr=col_ptr, row_idx=rows.astype(np.int32), val=vals,
                y=np.asarray(y, dtype=np.int8), w_star=w_star, meta=meta or {})


def from_dense(X: np.ndarray, y: np.ndarray) -> Data:
    n, p = X.shape
    r, c = np.nonzero(X)
    return from_triplets(n, p, r, c, X[r, c], y)


def _labels_from_scores(rng, s, flip):
    """y = sign(s), ties to a fair coin, then a fraction `flip` flipped at random."""
    y = np.where(s > 0, 1, -1).astype(np.int8)
    ties = s == 0
    y[ties] = np.where(rng.random(int(ties.sum())) < 0.5, 1, -1)
    if flip > 0:
        f = rng.random(len(y)) < flip
        y[f] = -y[f]
    return y


def _row_scores(n, rows, cols, vals, w_star):
    return np.bincount(rows, weights=vals.astype(np.float64) * w_star[cols], minlength=n)


def _zipf_cdf(p, a):
    w = np.arange(1, p + 1, dtype=np.float64) ** (-a)
    c = np.cumsum(w)
    return c / c[-1]


def _zipf_rows(rng, n, p, mean_len, a, cap=None):
    """Rows of distinct column ranks drawn from a Zipf(a) law truncated to 1..p.

    Row lengths are Poisson(mean_len) clamped to >= 1 (and <= p).  A rank drawn
    twice in one row is redrawn.  With `cap`, a column keeps only its first `cap`
    rows (in row order) and then leaves the pool; displaced entries are redrawn
    from the remaining columns.  Returns (rows, ranks) in 0-based form.
    """
    L = np.maximum(rng.poisson(mean_len, size=n), 1)
    L = np.minimum(L, p)
    rows = np.repeat(np.arange(n, dtype=np.int64), L)
    cdf = _zipf_cdf(p, a)
    alive = np.ones(p, dtype=bool)

    def draw(k):
        if alive.all():
            return np.minimum(np.searchsorted(cdf, rng.random(k), side="right"), p - 1)
        pmf = np.diff(np.concatenate(([0.0], cdf))) * alive
        c = np.cumsum(pmf)
        c /= c[-1]
        return np.minimum(np.searchsorted(c, rng.random(k), side="right"), p - 1)

    ranks = draw(len(rows))
    row_start = np.r_[0, np.cumsum(L)]
    check = np.arange(n)  # rows whose entries must be checked for duplicates
    for _ in range(500):
        # duplicates inside a row: keep the first occurrence, redraw the rest
        if len(check) == n:
            sel = np.arange(len(rows))
        else:
            lens = L[check]
            sel = np.repeat(row_start[check] - np.r_[0, np.cumsum(lens)[:-1]], lens) \
                + np.arange(int(lens.sum()))
        key = rows[sel] * p + ranks[sel]
        order = np.argsort(key, kind="stable")
        bad = np.zeros(len(rows), dtype=bool)
        bad[sel[order[1:]][key[order[1:]] == key[order[:-1]]]] = True
        if cap is not None:
            # column cap: a column keeps its first `cap` rows; later entries are displaced
            counts = np.bincount(ranks[~bad], minlength=p)
            hot = counts > cap
            if hot.any():
                idx = np.flatnonzero(hot[ranks] & ~bad)
                o2 = idx[np.lexsort((rows[idx], ranks[idx]))]
                rk = ranks[o2]
                starts = np.r_[0, np.flatnonzero(np.diff(rk)) + 1]
                pos = np.arange(len(rk)) - np.repeat(starts, np.diff(np.r_[starts, len(rk)]))
                bad[o2[pos >= cap]] = True
            alive &= counts < cap
        if not bad.any():
            break
        ranks[bad] = draw(int(bad.sum()))
        check = np.unique(rows[bad])
    else:  # pragma: no cover
        raise RuntimeError("row sampling did not settle")
    return rows, ranks


def c1(seed: int = BASE_SEED + 1) -> Data:
    """L1-LR, 1,000 x 500, 10% Bernoulli density, N(0,1) values; w* has 25
    nonzeros ~ N(0, 4); y = sign(x^T w* + logistic noise), sign(0) -> +1."""
    rng = np.random.default_rng(seed)
    n, p = 1000, 500
    mask = rng.random((n, p)) < 0.10
    r, c = np.nonzero(mask)
    v = rng.standard_normal(len(r)).astype(np.float32)
    w_star = np.zeros(p)
    sup = rng.choice(p, 25, replace=False)
    w_star[sup] = rng.normal(0.0, 2.0, 25)
    u = rng.random(n)
    noise = np.log(u / (1.0 - u))
    s = _row_scores(n, r, c, v, w_star) + noise
    y = np.where(s >= 0, 1, -1).astype(np.int8)
    return from_triplets(n, p, r, c, v, y, w_star,
                         dict(name="c1", loss="lr", C=1.0, P=32, eps=1e-4))


def c2(seed: int = BASE_SEED + 2, n: int = 20000, p: int = 50000,
       mean_len: float = 80.0) -> Data:
    """Text-like L1-LR data: Poisson(80) row lengths, Zipf(1.1) column
    frequencies, lognormal(0,1) values L2-normalised per row; w* has 500
    N(0,1) nonzeros on columns with >= 5 entries; y = sign(x^T w*) (ties to a
    coin) with 5% of labels flipped."""
    rng = np.random.default_rng(seed)
    rows, ranks = _zipf_rows(rng, n, p, mean_len, 1.1)
    colmap = rng.permutation(p)
    cols = colmap[ranks]
    v = rng.lognormal(0.0, 1.0, len(rows))
    norms = np.sqrt(np.bincount(rows, weights=v * v, minlength=n))
    v = (v / norms[rows]).astype(np.float32)
    counts = np.bincount(cols, minlength=p)
    cand = np.flatnonzero(counts >= 5)
    w_star = np.zeros(p)
    sup = rng.choice(cand, min(500, len(cand)), replace=False)
    w_star[sup] = rng.standard_normal(len(sup))
    y = _labels_from_scores(rng, _row_scores(n, rows, cols, v, w_star), 0.05)
    return from_triplets(n, p, rows, cols, v, y, w_star,
                         dict(name="c2", loss="lr", Cs=(0.5, 4.0), Ps=(64, 1024, 8192),
                              eps=1e-4))


def c3(seed: int = BASE_SEED + 3, n: int = 100000, p: int = 1000000,
       mean_len: float = 120.0, cap: int = 50000) -> Data:
    """Huge sparse binary L1-L2-SVM data: Poisson(120) row lengths, Zipf(1.05)
    column frequencies, values 1.0, at most `cap` entries per column (a capped
    column leaves the pool); w* has 2,000 N(0,1) nonzeros on columns with >= 5
    entries; y = sign(x^T w*) (ties to a coin) with 3% flipped."""
    rng = np.random.default_rng(seed)
    rows, ranks = _zipf_rows(rng, n, p, mean_len, 1.05, cap=cap)
    colmap = rng.permutation(p)
    cols = colmap[ranks]
    v = np.ones(len(rows), dtype=np.float32)
    counts = np.bincount(cols, minlength=p)
    cand = np.flatnonzero(counts >= 5)
    w_star = np.zeros(p)
    sup = rng.choice(cand, min(2000, len(cand)), replace=False)
    w_star[sup] = rng.standard_normal(len(sup))
    y = _labels_from_scores(rng, _row_scores(n, rows, cols, v, w_star), 0.03)
    return from_triplets(n, p, rows, cols, v, y, w_star,
                         dict(name="c3", loss="svm", C=1.0, P=16384, eps=1e-3))


def tiny(seed: int, n: int, p: int, density: float = 0.5, binary: bool = False,
         flip: float = 0.1, empty_cols=()) -> Data:
    """Small random problems for brute-force and invariant tests."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n, p)) < density
    for j in empty_cols:
        mask[:, j] = False
    r, c = np.nonzero(mask)
    v = np.ones(len(r)) if binary else rng.standard_normal(len(r))
    w_star = rng.standard_normal(p)
    y = _labels_from_scores(rng, _row_scores(n, r, c, v, w_star), flip)
    return from_triplets(n, p, r, c, v.astype(np.float32), y, w_star, dict(name="tiny"))


def sparse_random(seed: int, n: int, p: int, density: float, w_frac: float = 0.01,
                  binary: bool = False) -> Data:
    """Bernoulli(density) entries with N(0,1) (or binary) values and
    logistic-noise labels from a sparse w*: the mixed-problem recipe."""
    rng = np.random.default_rng(seed)
    nnz_target = int(round(n * p * density))
    # draw flat positions without replacement via sorted unique sampling
    pos = np.unique(rng.integers(0, n * p, size=int(nnz_target * 1.05) + 16))
    if len(pos) > nnz_target:
        pos = rng.choice(pos, nnz_target, replace=False)
    r, c = pos // p, pos % p
    v = np.ones(len(r)) if binary else rng.standard_normal(len(r))
    w_star = np.zeros(p)
    k = max(1, int(np.ceil(w_frac * p)))
    sup = rng.choice(p, k, replace=False)
    w_star[sup] = rng.standard_normal(k)
    u = rng.random(n)
    s = _row_scores(n, r, c, v, w_star) + np.log(u / (1.0 - u))
    y = np.where(s >= 0, 1, -1).astype(np.int8)
    return from_triplets(n, p, r, c, v.astype(np.float32), y, w_star, dict(name="sparse_random"))


def bernoulli_csc(seed: int, n: int, p: int, density: float, w_frac: float = 0.01) -> Data:
    """Bernoulli(density) entries with N(0,1) values, drawn directly in
    column-major order (no re-sort); labels y = sign(x^T w* + logistic noise)
    with ceil(w_frac p) N(0,1) nonzeros in w*.  The recipe of the batched
    independent problems."""
    rng = np.random.default_rng(seed)
    target = int(round(n * p * density))
    # distinct flat positions j * n + i, ascending = CSC order
    pos = np.unique(rng.integers(0, n * p, size=int(target * 1.02) + 16, dtype=np.int64))
    if len(pos) > target:
        keep = np.sort(rng.choice(len(pos), target, replace=False))
        pos = pos[keep]
    cols = pos // n
    rows = (pos - cols * n).astype(np.int32)
    del pos
    val = rng.standard_normal(len(rows)).astype(np.float32)
    col_ptr = np.zeros(p + 1, dtype=np.int64)
    np.cumsum(np.bincount(cols, minlength=p), out=col_ptr[1:])
    w_star = np.zeros(p)
    k = max(1, int(np.ceil(w_frac * p)))
    w_star[rng.choice(p, k, replace=False)] = rng.standard_normal(k)
    s = _row_scores(n, rows, cols, val, w_star)
    u = rng.random(n)
    s = s + np.log(u / (1.0 - u))
    y = np.where(s >= 0, 1, -1).astype(np.int8)
    return Data(n=n, p=p, col_ptr=col_ptr, row_idx=rows, val=val, y=y, w_star=w_star,
                meta=dict(name="bernoulli", density=density))


def c4_path_Cs(count: int = 32) -> np.ndarray:
    """The regularisation path's C values: log-spaced over [2^-4, 2^6], ascending."""
    return 2.0 ** (-4.0 + 10.0 * np.arange(count) / (count - 1))


def c4b_shapes(seed: int = BASE_SEED + 4, count: int = 64, scale: float = 1.0):
    """(n, p, density) of the batched independent problems: n uniform in
    [500, 20000], p uniform in [1000, 100000], density uniform in
    [0.001, 0.02]; `scale` < 1 shrinks n and p (not the density) for small
    runs."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(500, 20001))
        p = int(rng.integers(1000, 100001))
        d = float(rng.uniform(0.001, 0.02))
        out.append((max(2, int(n * scale)), max(2, int(p * scale)), d))
    return out


def c4b(seed: int = BASE_SEED + 4, count: int = 64, scale: float = 1.0) -> list:
    """The batched independent LR problems (see c4b_shapes), each drawn by
    bernoulli_csc with its own seed."""
    return [c4b_problem(i, seed, count, scale) for i in range(count)]


def c4b_problem(i: int, seed: int = BASE_SEED + 4, count: int = 64, scale: float = 1.0) -> Data:
    """Problem i of c4b alone."""
    n, p, d = c4b_shapes(seed, count, scale)[i]
    return bernoulli_csc(seed * 1000 + i, n, p, d)


def zipf_rows_csc(seed: int, n: int, p: int, row_lo: int, row_hi: int, a: float,
                  binary: bool, flip: float = 0.05, w_nnz: int = 500) -> Data:
    """Rows of U{row_lo..row_hi} entries whose columns follow a truncated
    Zipf(a) over p (column ranks mapped through a random permutation); a
    column drawn twice in one row is kept once.  Values: 1 (binary) or
    lognormal(0, 1) L2-normalised per row.  Labels y = sign(x^T w*) with
    min(w_nnz, p / 10) N(0, 1) nonzeros in w*, ties to a coin, `flip` flipped.
    Drawn in column-major order (CSC without a re-sort)."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(row_lo, row_hi + 1, size=n)
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    cdf = _zipf_cdf(p, a)
    ranks = np.minimum(np.searchsorted(cdf, rng.random(len(rows)), side="right"), p - 1)
    cols = rng.permutation(p)[ranks].astype(np.int64)
    pos = np.unique(cols * n + rows)
    cols = pos // n
    rows = (pos - cols * n).astype(np.int32)
    del pos
    if binary:
        val = np.ones(len(rows), dtype=np.float32)
    else:
        v = rng.lognormal(0.0, 1.0, len(rows))
        norm = np.sqrt(np.bincount(rows, weights=v * v, minlength=n))
        val = (v / norm[rows]).astype(np.float32)
    col_ptr = np.zeros(p + 1, dtype=np.int64)
    np.cumsum(np.bincount(cols, minlength=p), out=col_ptr[1:])
    w_star = np.zeros(p)
    k = max(1, min(w_nnz, p // 10))
    w_star[rng.choice(p, k, replace=False)] = rng.standard_normal(k)
    y = _labels_from_scores(rng, _row_scores(n, rows, cols, val, w_star), flip)
    return Data(n=n, p=p, col_ptr=col_ptr, row_idx=rows, val=val, y=y, w_star=w_star,
                meta=dict(name="zipf_rows", binary=binary))


def c5_pool(seed: int = BASE_SEED + 5, count: int = 16, scale: float = 1.0) -> list:
    """Pool of served problems: LR or SVM with probability 1/2; n log-uniform
    in [1e3, 2e5 * scale], p log-uniform in [1e3, 2e6 * scale], U{20..150}
    entries per row over Zipf(1.1) columns; LR values lognormal and
    row-normalised, SVM values binary.  Returns (data, loss) pairs."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        loss = "lr" if rng.random() < 0.5 else "svm"
        n = int(np.exp(rng.uniform(np.log(1e3), np.log(max(1e3, 2e5 * scale)))))
        p = int(np.exp(rng.uniform(np.log(1e3), np.log(max(1e3, 2e6 * scale)))))
        out.append((zipf_rows_csc(seed * 100 + i, n, p, 20, 150, 1.1, binary=(loss == "svm")),
                    loss))
    return out


def c5_stream(seed: int = BASE_SEED + 6, count: int = 500, rate: float = 50.0,
              pool: int = 16) -> list:
    """Poisson arrivals at `rate` per second: (arrival time in s, pool index,
    C log-uniform in [0.1, 10])."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    idx = rng.integers(0, pool, size=count)
    C = np.exp(rng.uniform(np.log(0.1), np.log(10.0), size=count))
    return [(float(t[k]), int(idx[k]), float(C[k])) for k in range(count)]


def with_bias(d: Data, bias: float = 1.0) -> Data:
    """The same data with a constant feature of value `bias` appended as the
    last column (every row holds it)."""
    col_ptr = np.concatenate([d.col_ptr, [d.col_ptr[-1] + d.n]]).astype(np.int64)
    row_idx = np.concatenate([d.row_idx, np.arange(d.n, dtype=np.int32)])
    val = np.concatenate([d.val, np.full(d.n, bias, dtype=np.float32)])
    w_star = None if d.w_star is None else np.concatenate([d.w_star, [0.0]])
    return Data(n=d.n, p=d.p + 1, col_ptr=col_ptr, row_idx=row_idx, val=val, y=d.y.copy(),
                w_star=w_star, meta=dict(d.meta, bias=bias))
