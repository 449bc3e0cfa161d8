"""Pins for the CPU oracle: checks against facts that do not come from the oracle.

Each test compares the oracle with an independent source -- dense matrix
products (numpy), closed forms, invariants, brute force on tiny inputs, or
values printed in the paper -- so that a dropped term, a wrong index or a
transposed operand in the oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
from synth import (CSR, bfs_frontier, erdos_renyi_fixed_degree, from_dense, identity,
                   permutation_matrix, random_sparse, rmat, shuffle_within_rows,
                   symmetric_rmat_graph, to_dense, transpose, triangle_inputs, with_values)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pattern_dense(a: CSR) -> np.ndarray:
    p = np.zeros(a.shape, dtype=np.int64)
    np.add.at(p, (a.row_ids(), a.cols.astype(np.int64)), 1)
    return p


def _rows_as_sets(c: CSR):
    return [set(c.cols[c.rpts[i]:c.rpts[i + 1]].tolist()) for i in range(c.nrows)]


def _assert_close_f64(got, ref, rtol=1e-12):
    got = np.asarray(got)
    ref = np.asarray(ref)
    nz = ref != 0
    assert np.all(got[~nz] == 0)
    assert np.all(np.abs(got[nz] - ref[nz]) <= rtol * np.abs(ref[nz]))


# ---------------------------------------------------------------- P1: dense products

@pytest.mark.parametrize("m,n,k,dens,seed", [
    (1, 1, 1, 1.0, 0), (7, 5, 9, 0.3, 1), (33, 17, 29, 0.2, 2), (64, 64, 64, 0.1, 3),
    (64, 40, 50, 0.5, 4), (20, 64, 3, 0.05, 5), (48, 48, 48, 0.02, 6),
])
@pytest.mark.parametrize("sorted_output", [True, False])
def test_p1_dense_matmul_f64(m, n, k, dens, seed, sorted_output):
    A = random_sparse(m, n, dens, seed, empty_rows=0.2, sorted_rows=False)
    B = random_sparse(n, k, dens, seed + 100, empty_rows=0.2, sorted_rows=False)
    C = oracle.spgemm(A, B, sorted_output=sorted_output)
    ref = to_dense(A) @ to_dense(B)
    _assert_close_f64(to_dense(C), ref)
    # structural pattern: (i,j) present iff some k has a_ik and b_kj stored
    pat = (_pattern_dense(A) @ _pattern_dense(B)) > 0
    assert np.array_equal(_pattern_dense(C) > 0, pat)
    assert np.all(_pattern_dense(C) <= 1)      # no duplicate columns in a row
    if sorted_output:
        for i in range(C.nrows):
            row = C.cols[C.rpts[i]:C.rpts[i + 1]]
            assert np.all(np.diff(row) > 0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_p1_dense_matmul_i64_exact(seed):
    A = random_sparse(40, 30, 0.2, seed, values="i64", empty_rows=0.1)
    B = random_sparse(30, 50, 0.2, seed + 7, values="i64", empty_rows=0.1)
    C = oracle.spgemm(A, B, sorted_output=True)
    assert np.array_equal(to_dense(C), to_dense(A) @ to_dense(B))


def test_p1_hand_example():
    # A = [[1,2,0],[0,0,3],[4,0,0]], B = [[0,5,0],[6,0,7],[0,8,0]]
    # row 0: 1*(0,5,0) + 2*(6,0,7) = (12,5,14); row 1: 3*(0,8,0); row 2: 4*(0,5,0)
    A = from_dense(np.array([[1, 2, 0], [0, 0, 3], [4, 0, 0]], dtype=np.float64))
    B = from_dense(np.array([[0, 5, 0], [6, 0, 7], [0, 8, 0]], dtype=np.float64))
    C = oracle.spgemm(A, B, sorted_output=True)
    assert C.rpts.tolist() == [0, 3, 4, 5]
    assert C.cols.tolist() == [0, 1, 2, 1, 1]
    assert C.vals.tolist() == [12.0, 5.0, 14.0, 24.0, 20.0]


def test_structural_zero_kept():
    # Fig. 1 inserts c_ij at its first product whatever the value: a sum that
    # cancels to zero stays in the pattern.
    A = CSR(1, 2, np.array([0, 2]), np.array([0, 1]), np.array([1.0, -1.0]))
    B = CSR(2, 1, np.array([0, 1, 2]), np.array([0, 0]), np.array([1.0, 1.0]))
    C = oracle.spgemm(A, B)
    assert C.nnz == 1 and C.cols.tolist() == [0] and C.vals.tolist() == [0.0]


def test_i64_wraps_modulo_2_64():
    A = CSR(1, 2, np.array([0, 2]), np.array([0, 1]), np.array([2**62, 2**62], dtype=np.int64))
    B = CSR(2, 1, np.array([0, 1, 2]), np.array([0, 0]), np.array([2, 2], dtype=np.int64))
    C = oracle.spgemm(A, B)
    assert C.vals.tolist() == [0]      # 2^63 + 2^63 = 2^64 = 0 mod 2^64


def test_duplicate_input_columns_add_up():
    # A repeated column is rejected by default; read as the sum of its entries
    # (a_01 = 1 + 2) when allowed, it gives row 0 of [[0, 3, 4]] @ B.
    A = CSR(1, 3, np.array([0, 3]), np.array([1, 1, 2]), np.array([1.0, 2.0, 4.0]))
    B = from_dense(np.array([[0, 0], [1, 0], [0, 1]], dtype=np.float64))
    with pytest.raises(ValueError, match="repeated"):
        oracle.spgemm(A, B)
    C = oracle.spgemm(A, B, allow_duplicates=True)
    assert sorted(zip(C.cols.tolist(), C.vals.tolist())) == [(0, 3.0), (1, 4.0)]
    ref = np.array([[0, 3.0, 4.0]]) @ to_dense(B)
    assert np.array_equal(to_dense(C), ref)


def _bad(nrows, ncols, rp, cols):
    return CSR(nrows, ncols, np.array(rp, dtype=np.int64), np.array(cols, dtype=np.int32),
               np.ones(len(cols)))


@pytest.mark.parametrize("bad,rule", [
    (_bad(2, 3, [1, 1, 2], [0, 1]), "rpts\\[0\\]"),                 # does not start at 0
    (_bad(2, 3, [0, 2, 1], [0, 1]), "decrease"),                     # row pointers decrease
    (_bad(2, 3, [0, 1, 1], [0, 1]), "nnz"),                          # end short of nnz
    (_bad(2, 3, [0, 1, 2], [0, 3]), "outside"),                      # column id == ncols
    (_bad(2, 3, [0, 1, 2], [-1, 0]), "outside"),                     # negative column id
    (_bad(1, 3, [0, 2], [2, 2]), "repeated"),                        # repeated column
])
def test_validate_rejects_malformed_csr(bad, rule):
    """Step 1 of the oracle: malformed operands are rejected before any product,
    whichever side they are on."""
    good = random_sparse(3, 2, 0.5, 1)
    with pytest.raises(ValueError, match=rule):
        oracle.validate(bad)
    with pytest.raises(ValueError, match=rule):
        oracle.spgemm(bad, random_sparse(bad.ncols, 4, 0.5, 2))
    with pytest.raises(ValueError, match=rule):
        oracle.symbolic(good, bad) if bad.nrows == 2 else oracle.symbolic(random_sparse(5, 1, 0.5, 3), bad)


def test_validate_shape_and_lengths():
    A = random_sparse(4, 5, 0.5, 1)
    with pytest.raises(ValueError, match="A.ncols"):
        oracle.spgemm(A, random_sparse(6, 3, 0.5, 2))
    short = CSR(4, 5, A.rpts[:-1], A.cols, A.vals)
    with pytest.raises(ValueError, match="nrows"):
        oracle.validate(short)
    for g in (A, rmat(8, 8, 3), erdos_renyi_fixed_degree(100, 5, 4)):
        oracle.validate(g)                                          # well formed: no error


# ---------------------------------------------------------------- P2: flop invariant

@pytest.mark.parametrize("maker", ["rmat", "er", "rect"])
def test_p2_flop_invariant(maker):
    if maker == "rmat":
        A = rmat(11, 16, 3)
        B = A
    elif maker == "er":
        A = erdos_renyi_fixed_degree(3000, 7, 4)
        B = A
    else:
        A = random_sparse(300, 200, 0.03, 5)
        B = random_sparse(200, 700, 0.02, 6)
    f = oracle.row_flop(A, B)
    # column form: sum_k nnz(A[:,k]) * nnz(B[k,:]), from a column histogram of A
    colcount = np.bincount(A.cols, minlength=A.ncols).astype(np.int64)
    assert int(f.sum()) == int(colcount @ B.row_lengths())
    # row form by brute force on a few rows
    rl = B.row_lengths()
    for i in range(0, A.nrows, max(1, A.nrows // 37)):
        assert f[i] == sum(int(rl[c]) for c in A.cols[A.rpts[i]:A.rpts[i + 1]])


def test_golden_table2_flop_counts_multiplications():
    with open(os.path.join(GOLDEN, "table2_regular_flop.txt")) as fh:
        name, n_m, nnz_m, flop_m, _ = [l for l in fh if not l.startswith("#")][0].split()
    n = int(round(float(n_m) * 1e6))
    d = int(round(float(nnz_m) / float(n_m)))
    A = erdos_renyi_fixed_degree(n, d, 11, values="")
    flop = int(oracle.row_flop(A, A).sum())
    assert round(flop / 1e6, 2) == float(flop_m)


# ---------------------------------------------------------------- P3: ER closed forms

def test_p3_er_closed_forms():
    A = erdos_renyi_fixed_degree(4096, 8, 1)
    assert int(oracle.row_flop(A, A).sum()) == 262_144
    A = erdos_renyi_fixed_degree(1 << 14, 16, 2, values="")
    f = oracle.row_flop(A, A)
    assert np.all(f == 256) and int(f.sum()) == (1 << 14) * 256


def test_p3_er_expected_collisions():
    # nnz(c_i) = flop_i minus repeated columns among 16 B rows of 16 distinct
    # uniform columns: E[repeats] ~ (C(256,2) - 16*C(16,2)) / n per row.
    n = 1 << 15
    A = erdos_renyi_fixed_degree(n, 16, 3)
    rp = oracle.symbolic(A, A)
    lost = n * 256 - int(rp[-1])
    expect = n * (math.comb(256, 2) - 16 * math.comb(16, 2)) / n
    assert abs(lost - expect) < 6 * math.sqrt(expect)


# ---------------------------------------------------------------- P4: bounds

def test_p4_bounds():
    A = rmat(12, 16, 7)
    f = oracle.row_flop(A, A)
    nz = np.diff(oracle.symbolic(A, A))
    assert np.all(nz <= np.minimum(f, A.ncols))
    assert np.all((nz == 0) == (f == 0))
    assert int(nz.sum()) <= int(f.sum())


# ---------------------------------------------------------------- P5: BFS frontier

def test_p5_bfs_identity():
    A = with_values(rmat(12, 16, 9, values=""), 0, "ones")
    F = bfs_frontier(A.ncols, 512, 10)
    C = oracle.spgemm(A, F, sorted_output=True)
    assert C.nnz == int(oracle.row_flop(A, F).sum())       # compression ratio 1
    # column j of C is v_j * column r_j of A; build from A^T without a product
    At = transpose(A)
    r_of = np.empty(F.ncols, dtype=np.int64)
    v_of = np.empty(F.ncols, dtype=np.int64)
    r_of[F.cols] = F.row_ids()
    v_of[F.cols] = F.vals
    Ct = transpose(C)
    for j in range(F.ncols):
        r = r_of[j]
        assert np.array_equal(Ct.cols[Ct.rpts[j]:Ct.rpts[j + 1]], At.cols[At.rpts[r]:At.rpts[r + 1]])
        assert np.all(Ct.vals[Ct.rpts[j]:Ct.rpts[j + 1]] == v_of[j])


# ---------------------------------------------------------------- P6: metamorphic

def test_p6_identity_and_permutation():
    A = rmat(10, 8, 12)
    I = identity(A.nrows)
    for C in (oracle.spgemm(A, I), oracle.spgemm(I, A)):
        assert np.array_equal(C.rpts, A.rpts)
        assert np.array_equal(C.cols, A.cols)
        assert np.array_equal(C.vals, A.vals)
    perm = np.random.default_rng(1).permutation(A.nrows)
    C = oracle.spgemm(permutation_matrix(perm), A)
    assert np.array_equal(to_dense(C), to_dense(A)[perm])


def test_p6_transpose_identity():
    A = random_sparse(50, 40, 0.1, 21, sorted_rows=False)
    B = random_sparse(40, 60, 0.1, 22, sorted_rows=False)
    ABt = transpose(oracle.spgemm(A, B))
    BtAt = oracle.spgemm(transpose(B), transpose(A))
    assert np.array_equal(ABt.rpts, BtAt.rpts)
    assert np.array_equal(ABt.cols, BtAt.cols)
    _assert_close_f64(BtAt.vals, ABt.vals)


# ---------------------------------------------------------------- P7: all-ones counts

def test_p7_all_ones_counts_paths():
    A = rmat(10, 8, 13)
    A1 = with_values(A, 0, "ones")
    C1 = oracle.spgemm(A1, A1)
    P = _pattern_dense(A).astype(np.float64)  # counts < 2^53: exact in binary64
    assert np.array_equal(to_dense(C1), (P @ P).astype(np.int64))
    Cf = oracle.spgemm(A, A)
    assert np.array_equal(C1.rpts, Cf.rpts) and np.array_equal(C1.cols, Cf.cols)


# ---------------------------------------------------------------- P8: triangles

def _graph(n, edges):
    d = np.zeros((n, n), dtype=np.int64)
    for u, v in edges:
        if u != v:
            d[u, v] = d[v, u] = 1
    return from_dense(d)


def _tri(a):
    A, L, U = triangle_inputs(a)
    return oracle.triangle_count(A, L, U)


@pytest.mark.parametrize("n", [3, 4, 5, 12, 100])
def test_p8_complete_graph(n):
    a = _graph(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    assert _tri(a) == math.comb(n, 3)


def test_p8_known_counts():
    assert _tri(_graph(5, [(i, 3 + j) for i in range(3) for j in range(2)])) == 0     # K_{3,2}
    assert _tri(_graph(8, [(i, (i + 1) % 8) for i in range(8)])) == 0                 # C_8
    assert _tri(_graph(3, [(0, 1), (1, 2), (2, 0)])) == 1                             # C_3
    rng = np.random.default_rng(0)
    tree = [(i, int(rng.integers(0, i))) for i in range(1, 30)]
    assert _tri(_graph(30, tree)) == 0
    for n in (4, 5, 9):                                                              # wheel W_n
        rim = [(i, (i + 1) % n) for i in range(n)]
        hub = [(n, i) for i in range(n)]
        assert _tri(_graph(n + 1, rim + hub)) == n


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_p8_trace_formula(seed):
    rng = np.random.default_rng(seed)
    n = 40
    up = np.triu(rng.random((n, n)) < 0.2, 1)
    d = (up | up.T).astype(np.int64)
    assert _tri(from_dense(d)) == int(np.trace(d @ d @ d)) // 6


def test_p8_relabel_invariance():
    a = symmetric_rmat_graph(11, 16, 4)
    A0, L0, U0 = triangle_inputs(a, degree_order=False)
    A1, L1, U1 = triangle_inputs(a, degree_order=True)
    t0 = oracle.triangle_count(A0, L0, U0)
    t1 = oracle.triangle_count(A1, L1, U1)
    assert t0 == t1 > 0
    d = to_dense(A0).astype(np.float64)      # counts < 2^53: exact in binary64
    assert t0 == int(round(np.trace(d @ d @ d))) // 6


# ---------------------------------------------------------------- P9: row independence

def test_p9_row_subset():
    A = shuffle_within_rows(rmat(11, 16, 14), 3)
    full = oracle.spgemm(A, A, sorted_output=True)
    rows = np.random.default_rng(2).choice(A.nrows, 300, replace=False)
    sub = oracle.spgemm(A, A, sorted_output=True, rows=rows)
    ref = full.take_rows(rows)
    assert np.array_equal(sub.rpts, ref.rpts)
    assert np.array_equal(sub.cols, ref.cols)
    assert np.array_equal(sub.vals, ref.vals)


def test_unsorted_output_is_permutation_of_sorted():
    A = shuffle_within_rows(rmat(10, 16, 15), 4)
    s = oracle.spgemm(A, A, sorted_output=True)
    u = oracle.spgemm(A, A, sorted_output=False)
    assert np.array_equal(s.rpts, u.rpts)
    assert _rows_as_sets(s) == _rows_as_sets(u)
    assert np.allclose(to_dense(s), to_dense(u), rtol=1e-12, atol=0)


def test_thread_count_does_not_change_result():
    A = rmat(11, 16, 16)
    c1 = oracle.spgemm(A, A, nthreads=1)
    c5 = oracle.spgemm(A, A, nthreads=5)
    assert np.array_equal(c1.cols, c5.cols) and np.array_equal(c1.vals, c5.vals)


# ---------------------------------------------------------------- Fig. 4 / Fig. 5 helpers

@pytest.mark.parametrize("tnum", [1, 2, 3, 8, 64])
def test_rows_to_threads_lower_bound(tnum):
    rng = np.random.default_rng(tnum)
    flop = rng.integers(0, 50, size=200)
    flop[rng.random(200) < 0.3] = 0
    off = oracle.rows_to_threads(flop, tnum)
    ps = np.concatenate([[0], np.cumsum(flop)])
    total = ps[-1]
    assert off[0] == 0 and off[-1] == flop.size and np.all(np.diff(off) >= 0)
    for t in range(1, tnum):
        # brute force: first id in [0, n] with ps[id] >= total * t / tnum
        ids = [i for i in range(flop.size + 1) if ps[i] * tnum >= total * t]
        assert off[t] == ids[0]


def test_lowest_p2_is_strict():
    assert [oracle.lowest_p2(x) for x in (0, 1, 2, 3, 4, 7, 8, 1023, 1024)] == \
        [1, 2, 4, 4, 8, 8, 16, 1024, 2048]
