"""The seeded generators produce valid, reproducible CSC inputs of the stated shape."""
import numpy as np
import pytest

import synth


def _check_csc(d):
    assert d.col_ptr.dtype == np.int64 and d.row_idx.dtype == np.int32
    assert d.val.dtype == np.float32 and d.y.dtype == np.int8
    assert d.col_ptr[0] == 0 and np.all(np.diff(d.col_ptr) >= 0) and d.col_ptr[-1] == len(d.row_idx)
    assert d.row_idx.min() >= 0 and d.row_idx.max() < d.n
    for j in np.flatnonzero(np.diff(d.col_ptr) > 1)[:2000]:
        r = d.row_idx[d.col_ptr[j]:d.col_ptr[j + 1]]
        assert np.all(np.diff(r) > 0)
    assert set(np.unique(d.y).tolist()) <= {-1, 1}
    assert np.all(np.isfinite(d.val))


@pytest.mark.parametrize("make", [synth.c1, synth.c2,
                                  lambda: synth.c3(n=5000, p=40000, cap=600)])
def test_generators_valid_and_seeded(make):
    a, b = make(), make()
    _check_csc(a)
    assert np.array_equal(a.row_idx, b.row_idx) and np.array_equal(a.val, b.val)
    assert np.array_equal(a.y, b.y)


def test_c2_shape_statistics():
    d = synth.c2()
    assert (d.n, d.p) == (20000, 50000)
    assert 1.5e6 < d.nnz < 1.7e6
    cl = d.col_lengths()
    assert cl.max() == d.n  # the Zipf head saturates
    rows = np.bincount(d.row_idx, weights=d.val.astype(float) ** 2, minlength=d.n)
    np.testing.assert_allclose(rows, 1.0, rtol=1e-5)


def test_c3_cap_respected_small():
    d = synth.c3(n=5000, p=40000, cap=600)
    assert d.col_lengths().max() <= 600
    assert np.all(d.val == 1.0)


def test_bernoulli_csc_and_batched_shapes():
    d = synth.bernoulli_csc(7, 300, 500, 0.02)
    assert d.col_ptr[0] == 0 and d.col_ptr[-1] == d.nnz and np.all(np.diff(d.col_ptr) >= 0)
    assert d.nnz == round(300 * 500 * 0.02)
    for j in range(d.p):
        r = d.row_idx[d.col_ptr[j]:d.col_ptr[j + 1]]
        assert np.all(np.diff(r) > 0) and (len(r) == 0 or (r[0] >= 0 and r[-1] < d.n))
    assert set(np.unique(d.y)) <= {-1, 1}
    assert np.count_nonzero(d.w_star) == int(np.ceil(0.01 * 500))
    again = synth.bernoulli_csc(7, 300, 500, 0.02)
    assert np.array_equal(again.row_idx, d.row_idx) and np.array_equal(again.val, d.val)
    shapes = synth.c4b_shapes()
    assert len(shapes) == 64
    for n, p, dens in shapes:
        assert 500 <= n <= 20000 and 1000 <= p <= 100000 and 0.001 <= dens <= 0.02
    Cs = synth.c4_path_Cs()
    assert len(Cs) == 32 and Cs[0] == 2.0 ** -4 and abs(Cs[-1] - 2.0 ** 6) < 1e-12
    assert np.all(np.diff(np.log2(Cs)) > 0)


def test_with_bias_appends_constant_column():
    d = synth.tiny(5, n=7, p=4, density=0.5)
    b = synth.with_bias(d, 2.5)
    assert b.p == d.p + 1 and b.nnz == d.nnz + d.n
    X, Xb = d.dense(), b.dense()
    assert np.array_equal(Xb[:, :d.p], X) and np.all(Xb[:, d.p] == 2.5)
    assert np.array_equal(b.y, d.y)
