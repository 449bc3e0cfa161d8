"""Properties of the seeded input generators (structure only, no product arithmetic)."""
import math

import numpy as np
import pytest

from synth import (bfs_frontier, column_sample, erdos_renyi_fixed_degree, rmat, serving_request_operands,
                   serving_stream, shuffle_within_rows, symmetric_rmat_graph, to_dense, transpose,
                   triangle_inputs, validate)


def test_er_fixed_degree_distinct():
    a = erdos_renyi_fixed_degree(4096, 8, 1)
    validate(a)
    assert np.all(a.row_lengths() == 8)
    assert a.vals.dtype == np.float64 and a.vals.min() >= 0 and a.vals.max() < 1


def test_seeded_reproducible():
    a = rmat(10, 16, 5)
    b = rmat(10, 16, 5)
    assert np.array_equal(a.cols, b.cols) and np.array_equal(a.vals, b.vals)
    c = rmat(10, 16, 6)
    assert not (a.nnz == c.nnz and np.array_equal(a.cols, c.cols))


def test_rmat_shape_and_skew():
    a = rmat(12, 16, 2)
    validate(a)
    n = 1 << 12
    assert a.nnz <= 16 * n and a.nnz > 0.8 * 16 * n
    lens = a.row_lengths()
    assert lens[0] == lens.max()          # G500 parameters put most mass on row 0


def test_shuffle_keeps_rows():
    a = rmat(10, 16, 3)
    s = shuffle_within_rows(a, 4)
    assert np.array_equal(a.rpts, s.rpts)
    for i in range(0, a.nrows, 97):
        r0, r1 = a.rpts[i], a.rpts[i + 1]
        o = np.argsort(s.cols[r0:r1])
        assert np.array_equal(a.cols[r0:r1], s.cols[r0:r1][o])
        assert np.array_equal(a.vals[r0:r1], s.vals[r0:r1][o])


def test_triangle_inputs():
    g = symmetric_rmat_graph(9, 16, 1)
    validate(g)
    assert np.all(g.cols != g.row_ids())
    gt = transpose(g)
    assert np.array_equal(gt.cols, g.cols)          # symmetric
    for order in (False, True):
        A, L, U = triangle_inputs(g, degree_order=order)
        assert L.nnz == U.nnz == A.nnz // 2
        assert np.all(L.cols < L.row_ids()) and np.all(U.cols > U.row_ids())
    A, _, _ = triangle_inputs(g, degree_order=True)
    deg = A.row_lengths()
    assert np.all(np.diff(deg) >= 0)


def test_bfs_frontier():
    f = bfs_frontier(1000, 512, 3)
    validate(f)
    assert f.nnz == 512 and sorted(f.cols.tolist()) == list(range(512))
    assert f.vals.min() >= 1 and f.vals.max() <= 1000


def test_serving_stream():
    reqs = serving_stream(300, 1)
    t = [r.arrival_s for r in reqs]
    assert np.all(np.diff(t) > 0)
    ns = np.array([r.n for r in reqs])
    assert ns.min() >= 256 and ns.max() <= 131072
    assert 2 <= min(r.d for r in reqs) and max(r.d for r in reqs) <= 32
    ln = np.log(ns)
    assert abs(ln.mean() - (math.log(256) + math.log(131072)) / 2) < 0.5
    small = serving_stream(50, 2, max_flop=2**20)
    assert all(r.n * r.d * r.d <= 2**20 for r in small)
    for r in reqs[:6]:
        if r.n > 4000:
            continue
        a, b = serving_request_operands(r)
        validate(a, allow_duplicates=False)
        validate(b)
        assert a.shape == b.shape == (r.n, r.n)


def test_column_sample():
    # tall-skinny operand (Section 5.5): every column of B is one column of A,
    # the picked columns are distinct and kept in ascending order; A's random
    # FP64 values make its non-empty columns unique, so each is located exactly
    a = rmat(7, 8, 5)
    da = to_dense(a)
    k = 40
    b = column_sample(a, k, 11)
    assert b.shape == (a.nrows, k)
    validate(b)
    db = to_dense(b)
    src = []
    n_empty = 0
    for t in range(k):
        if not db[:, t].any():
            n_empty += 1
            continue
        hits = [j for j in range(a.ncols) if np.array_equal(db[:, t], da[:, j])]
        assert len(hits) == 1, f"column {t} of B is not exactly one column of A"
        src.append(hits[0])
    assert src == sorted(src) and len(set(src)) == len(src)
    assert n_empty <= int((~da.any(axis=0)).sum())
    b2 = column_sample(a, k, 11)
    assert np.array_equal(b.cols, b2.cols) and np.array_equal(b.rpts, b2.rpts)
    with pytest.raises(ValueError):
        column_sample(a, a.ncols + 1, 1)
