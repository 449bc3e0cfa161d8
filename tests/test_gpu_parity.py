"""GPU parity: the HIP library through its C ABI against the CPU oracle, element by
element, on seeded inputs spanning every row bin, the column-window path of heavy
rows, both output orders, both value types and the edge cases."""
import sys

import numpy as np
import pytest

import oracle
from synth import (CSR, bfs_frontier, erdos_renyi_fixed_degree, from_dense, random_sparse, rmat,
                   shuffle_within_rows, symmetric_rmat_graph, triangle_inputs, with_values)

from _compare import assert_matches, assert_rows_match

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_01698_amd as sp
    return sp


def _dev(sp, a):
    return sp.DeviceCSR.from_host(a, device="cuda")


def _run(sp, A, B, sorted_output, validate=False):
    import torch
    dA, dB = _dev(sp, A), _dev(sp, B)
    C = sp.spgemm(dA, dB, sorted_output=sorted_output, validate=validate)
    torch.cuda.synchronize()
    return C


TINY = [
    (1, 1, 1, 1.0, 0), (7, 5, 9, 0.3, 1), (33, 17, 29, 0.2, 2), (64, 64, 64, 0.1, 3),
    (100, 80, 120, 0.3, 4), (300, 200, 500, 0.05, 5), (257, 1000, 3, 0.01, 6), (50, 50, 50, 0.9, 7),
]


@pytest.mark.parametrize("m,n,k,dens,seed", TINY)
@pytest.mark.parametrize("sorted_output", [True, False])
@pytest.mark.parametrize("vt", ["f64", "i64"])
def test_random_small(sp, m, n, k, dens, seed, sorted_output, vt):
    _note(f"case random_small m={m} n={n} k={k} dens={dens} seed={seed} sorted={sorted_output} {vt}")
    A = random_sparse(m, n, dens, seed, values=vt, empty_rows=0.2, sorted_rows=False)
    B = random_sparse(n, k, dens, seed + 50, values=vt, empty_rows=0.2, sorted_rows=False)
    C = _run(sp, A, B, sorted_output)
    assert_matches(C, oracle.spgemm(A, B, sorted_output=sorted_output), sorted_output)


def test_empty_and_degenerate(sp):
    _note("case empty_and_degenerate")
    z = CSR(5, 4, np.zeros(6, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0))
    b = random_sparse(4, 6, 0.5, 1)
    for A, B in [(z, b), (random_sparse(3, 5, 0.5, 2), CSR(5, 4, np.zeros(6, dtype=np.int64),
                                                            np.zeros(0, dtype=np.int32), np.zeros(0)))]:
        C = _run(sp, A, B, True)
        assert_matches(C, oracle.spgemm(A, B), True)
    e = CSR(0, 3, np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0))
    C = _run(sp, e, random_sparse(3, 3, 0.5, 3), True)
    assert C.nnz == 0 and C.rpts.cpu().tolist() == [0]


def test_structural_zero_and_wraparound(sp):
    _note("case structural_zero_and_wraparound")
    A = CSR(1, 2, np.array([0, 2]), np.array([0, 1]), np.array([1.0, -1.0]))
    B = CSR(2, 1, np.array([0, 1, 2]), np.array([0, 0]), np.array([1.0, 1.0]))
    C = _run(sp, A, B, True)
    rp, cols, vals = C.to_host()
    assert rp.tolist() == [0, 1] and cols.tolist() == [0] and vals.tolist() == [0.0]
    A = CSR(1, 2, np.array([0, 2]), np.array([0, 1]), np.array([2**62, 2**62], dtype=np.int64))
    B = CSR(2, 1, np.array([0, 1, 2]), np.array([0, 0]), np.array([2, 2], dtype=np.int64))
    C = _run(sp, A, B, True)
    assert C.to_host()[2].tolist() == [0]


def test_er4096_sorted(sp):
    """ER n=4096, 8 distinct uniform columns per row, A*A, sorted output."""
    _note("case er4096_sorted")
    A = erdos_renyi_fixed_degree(4096, 8, 1)
    C = _run(sp, A, A, True)
    assert_matches(C, oracle.spgemm(A, A, sorted_output=True), True)


@pytest.mark.parametrize("scale", [10, 12, 14])
@pytest.mark.parametrize("sorted_output", [True, False])
def test_rmat_mid(sp, scale, sorted_output):
    _note(f"case rmat_mid scale={scale} sorted={sorted_output}")
    A = rmat(scale, 16, scale)
    if not sorted_output:
        A = shuffle_within_rows(A, 5)
    C = _run(sp, A, A, sorted_output)
    assert_matches(C, oracle.spgemm(A, A, sorted_output=sorted_output), sorted_output)


@pytest.mark.parametrize("sorted_output", [True, False])
@pytest.mark.parametrize("low_memory", [False, True])
def test_rmat16_full(sp, sorted_output, low_memory):
    """R-MAT scale 16 ef 16 A*A: every bin, bitmap symbolic and column windows
    (with the symbolic bitmaps kept for the windows, and without)."""
    _note(f"case rmat16_full sorted={sorted_output} low_memory={low_memory}")
    A = rmat(16, 16, 1)
    if not sorted_output:
        A = shuffle_within_rows(A, 3)
    dA = _dev(sp, A)
    p = sp.Plan([dA], [dA], sorted_output=sorted_output, low_memory=low_memory)
    p.symbolic()
    C = p.numeric()[0]
    st = p.stats(0)
    assert st["status"] == 0 and st["probe_overflow"] == 0
    assert st["heavy_rows"] > 0 and st["windows"] > st["heavy_rows"]
    assert st["flop"] == int(oracle.row_flop(A, A).sum())
    assert_matches(C, oracle.spgemm(A, A, sorted_output=sorted_output), sorted_output)
    p.close()


def test_rmat_i64(sp):
    _note("case rmat_i64")
    A = with_values(rmat(13, 16, 4, values=""), 9, "i64", lo=-(2**40), hi=2**40)
    A = shuffle_within_rows(A, 2)
    for srt in (True, False):
        C = _run(sp, A, A, srt)
        assert_matches(C, oracle.spgemm(A, A, sorted_output=srt), srt)


def test_wide_columns_multipass_bitmap(sp):
    """B wider than one LDS bitmap (2,000,000 columns): the symbolic bitmap sweeps
    in passes and the heavy row still splits into column windows."""
    _note("case wide_columns_multipass_bitmap")
    k = 2_000_000
    B = erdos_renyi_fixed_degree(3000, 20, 7, ncols=k)
    rng = np.random.default_rng(8)
    rows = [np.sort(rng.choice(3000, size=s, replace=False)) for s in (1500, 30, 0, 700)]
    rp = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum([r.size for r in rows], out=rp[1:])
    A = with_values(CSR(len(rows), 3000, rp, np.concatenate(rows).astype(np.int32), None), 9, "f64")
    import torch
    dA, dB = _dev(sp, A), _dev(sp, B)
    for srt in (True, False):
        for low in (False, True):
            p = sp.Plan([dA], [dB], sorted_output=srt, low_memory=low)
            p.symbolic()
            C = p.numeric()[0]
            torch.cuda.synchronize()
            assert p.stats(0)["status"] == 0
            p.close()
            assert_matches(C, oracle.spgemm(A, B, sorted_output=srt), srt)


def test_very_wide_columns_global_window_counters(sp):
    """More than 4096 column chunks (17,000,000 columns): the window split
    counts windows per first chunk in global memory instead of LDS."""
    _note("case very_wide_columns")
    import torch
    k = 17_000_000
    B = erdos_renyi_fixed_degree(4000, 24, 11, ncols=k)
    rng = np.random.default_rng(12)
    rows = [np.sort(rng.choice(4000, size=s, replace=False)) for s in (2500, 900, 5, 0, 1200)]
    rp = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum([r.size for r in rows], out=rp[1:])
    A = with_values(CSR(len(rows), 4000, rp, np.concatenate(rows).astype(np.int32), None), 13, "f64")
    dA, dB = _dev(sp, A), _dev(sp, B)
    for srt in (True, False):
        p = sp.Plan([dA], [dB], sorted_output=srt)
        p.symbolic()
        C = p.numeric()[0]
        torch.cuda.synchronize()
        st = p.stats(0)
        assert st["status"] == 0 and st["heavy_rows"] >= 3
        p.close()
        assert_matches(C, oracle.spgemm(A, B, sorted_output=srt, nthreads=2), srt)


def test_rectangular_tall_skinny_bfs(sp):
    """Multi-source BFS step: R-MAT scale 14 (int64 ones) times a frontier stack."""
    _note("case bfs")
    A = with_values(rmat(14, 16, 9, values=""), 0, "ones")
    F = bfs_frontier(A.ncols, 512, 10)
    for srt in (True, False):
        C = _run(sp, A, F, srt)
        ref = oracle.spgemm(A, F, sorted_output=srt)
        assert_matches(C, ref, srt)
        assert C.nnz == int(oracle.row_flop(A, F).sum())


@pytest.mark.parametrize("degree_order", [False, True])
def test_triangles(sp, degree_order):
    _note(f"case triangles degree_order={degree_order}")
    g = symmetric_rmat_graph(12, 16, 4)
    A, L, U = triangle_inputs(g, degree_order=degree_order)
    t = sp.triangle_count(_dev(sp, A), _dev(sp, L), _dev(sp, U))
    assert t == oracle.triangle_count(A, L, U)
    assert sp.triangle_count(_dev(sp, A), _dev(sp, L), _dev(sp, U), fused=False) == t
    C = _run(sp, L, U, True)
    assert_matches(C, oracle.spgemm(L, U, sorted_output=True), True)


def test_triangles_closed_form(sp):
    _note("case triangles_closed_form")
    for n in (5, 100, 300):
        d = np.ones((n, n), dtype=np.int64) - np.eye(n, dtype=np.int64)
        A, L, U = triangle_inputs(from_dense(d))
        assert sp.triangle_count(_dev(sp, A), _dev(sp, L), _dev(sp, U)) == n * (n - 1) * (n - 2) // 6
    d = np.zeros((9, 9), dtype=np.int64)
    d[:4, 4:] = 1
    d[4:, :4] = 1
    A, L, U = triangle_inputs(from_dense(d))
    assert sp.triangle_count(_dev(sp, A), _dev(sp, L), _dev(sp, U)) == 0


def _mask(m, k, dens, seed):
    """A random pattern (no repeated column in a row), values irrelevant."""
    return random_sparse(m, k, dens, seed, values="ones")


@pytest.mark.parametrize("m,n,k,da,db,dm,seed", [
    (1, 1, 1, 1.0, 1.0, 1.0, 0), (40, 30, 50, 0.2, 0.2, 0.3, 1), (300, 200, 400, 0.05, 0.05, 0.1, 2),
    (120, 90, 70, 0.4, 0.3, 0.05, 3), (64, 64, 64, 0.0, 0.5, 0.5, 4), (50, 60, 70, 0.3, 0.3, 0.0, 5)])
def test_masked_product_values(sp, m, n, k, da, db, dm, seed):
    """Masked product sum with int64 values (wrap-around) against the explicit
    product summed over the mask."""
    _note(f"case masked_product m={m} n={n} k={k} seed={seed}")
    A = with_values(random_sparse(m, n, da, seed, values=""), seed + 1, "i64", lo=-(2**40), hi=2**40)
    B = with_values(random_sparse(n, k, db, seed + 2, values=""), seed + 3, "i64", lo=-(2**40), hi=2**40)
    M = _mask(m, k, dm, seed + 4)
    want = oracle.masked_sum(oracle.spgemm(A, B, sorted_output=True), M)
    got = sp.masked_product_sum_i64(_dev(sp, A), _dev(sp, B), _dev(sp, M))
    assert got == want
    ones = lambda X: with_values(X, 0, "ones")
    want1 = oracle.masked_sum(oracle.spgemm(ones(A), ones(B), sorted_output=True), M)
    assert sp.masked_product_sum_i64(_dev(sp, A), _dev(sp, B), _dev(sp, M), ones=True) == want1


def test_masked_product_wide_multipass(sp):
    """2,500,000 columns: the mask bitmap sweeps three passes."""
    _note("case masked_product wide")
    k = 2_500_000
    B = with_values(erdos_renyi_fixed_degree(2000, 16, 21, ncols=k, values=""), 22, "i64", lo=1, hi=9)
    A = with_values(random_sparse(300, 2000, 0.01, 23, values=""), 24, "i64", lo=1, hi=9)
    # the mask holds half of each row's product columns plus unrelated columns
    C = oracle.spgemm(A, B, sorted_output=True)
    rng = np.random.default_rng(25)
    rows = []
    for i in range(C.nrows):
        cols = C.cols[C.rpts[i]:C.rpts[i + 1]]
        keep = cols[rng.random(cols.size) < 0.5]
        extra = rng.choice(k, 5, replace=False)
        rows.append(np.unique(np.concatenate([keep, extra])).astype(np.int32))
    rp = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum([r.size for r in rows], out=rp[1:])
    M = CSR(len(rows), k, rp, np.concatenate(rows), np.ones(int(rp[-1]), dtype=np.int64))
    assert sp.masked_product_sum_i64(_dev(sp, A), _dev(sp, B), _dev(sp, M)) == oracle.masked_sum(C, M)


def test_repeat_runs_identical_pattern(sp):
    _note("case determinism")
    A = shuffle_within_rows(rmat(14, 16, 21), 1)
    C1 = _run(sp, A, A, False)
    C2 = _run(sp, A, A, False)
    r1, c1, v1 = C1.to_host()
    r2, c2, v2 = C2.to_host()
    assert np.array_equal(r1, r2)
    rows = np.repeat(np.arange(A.nrows), np.diff(r1))
    o1, o2 = np.lexsort((c1, rows)), np.lexsort((c2, rows))
    assert np.array_equal(c1[o1], c2[o2])
    assert np.allclose(v1[o1], v2[o2], rtol=1e-12, atol=0)


def test_numeric_reuse_with_new_values(sp):
    """Plan and symbolic once, numeric twice with different values (same pattern)."""
    _note("case numeric_reuse")
    import torch
    A1 = rmat(13, 16, 3)
    A2 = with_values(A1, 77, "f64")
    d1, d2 = _dev(sp, A1), _dev(sp, A2)
    d2.rpts, d2.cols = d1.rpts, d1.cols
    p = sp.Plan([d1], [d1], sorted_output=True)
    p.symbolic()
    C = p.numeric()[0]
    torch.cuda.synchronize()
    assert_matches(C, oracle.spgemm(A1, A1), True)
    C = p.numeric([d2], [d2])[0]
    torch.cuda.synchronize()
    assert_matches(C, oracle.spgemm(A2, A2), True)
    assert p.stats(0)["status"] == 0
    p.close()


def test_validate_rejects_bad_column(sp):
    _note("case validate")
    A = random_sparse(20, 10, 0.3, 1)
    A.cols[3] = 10            # == ncols: out of range
    B = random_sparse(10, 10, 0.3, 2)
    with pytest.raises(sp.SpgemmError) as ei:
        _run(sp, A, B, True, validate=True)
    assert ei.value.status == -3


def test_sampled_rows_api(sp):
    """Row independence (P9) used for large products: rows of the full device
    product equal the oracle computed on those rows alone."""
    _note("case sampled_rows")
    A = shuffle_within_rows(rmat(15, 16, 6), 4)
    C = _run(sp, A, A, False)
    f = oracle.row_flop(A, A)
    rows = np.unique(np.concatenate([np.argsort(f)[-50:], np.random.default_rng(0).choice(A.nrows, 200)]))
    ref = oracle.spgemm(A, A, sorted_output=False, rows=rows)
    assert_rows_match(C, ref, rows, False)


@pytest.mark.parametrize("ncols", [300000, 2000000])
def test_sorted_wide_bins_rank_passes(sp, ncols):
    # rows of the 512- and 1024-thread bins with their columns spread over
    # 300,000 columns (sorted output ranks them in several column passes) or
    # over 2,000,000 (more passes than allowed: bitonic sorting)
    _note(f"case sorted_wide_bins_rank_passes ncols={ncols}")
    rng = np.random.default_rng(21)
    n = 4000
    degs = np.repeat([300, 800, 1500, 2000], 8)
    rows = [np.sort(rng.choice(n, size=d, replace=False)) for d in degs]
    rp = np.zeros(len(degs) + 1, dtype=np.int64)
    rp[1:] = np.cumsum(degs)
    A = with_values(CSR(len(degs), n, rp, np.concatenate(rows).astype(np.int32), None), 3, "f64")
    bcols = np.concatenate([np.sort(rng.choice(ncols, size=3, replace=False)) for _ in range(n)])
    B = with_values(CSR(n, ncols, np.arange(0, 3 * n + 1, 3, dtype=np.int64), bcols.astype(np.int32), None),
                    4, "f64")
    for srt in (True, False):
        C = _run(sp, shuffle_within_rows(A, 5), B, srt)
        assert_matches(C, oracle.spgemm(A, B, sorted_output=srt), srt)


def test_masked_sums_on_a_side_stream(sp):
    """Masked sums launched on a non-default stream: the binding allocates on
    that stream and reads the result only after it is done."""
    import torch
    _note("case masked sums on a side stream")
    g = symmetric_rmat_graph(12, 16, 5)
    A, L, U = triangle_inputs(g, degree_order=False)
    ref = oracle.triangle_count(A, L, U)
    dA, dL, dU = _dev(sp, A), _dev(sp, L), _dev(sp, U)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):
        # keep the current stream busy so that a read on it would run early
        busy = torch.randn(1 << 22, device="cuda")
        for _ in range(8):
            busy = busy * 1.0001
        assert sp.triangle_count(dA, dL, dU, stream=side) == ref
        assert sp.triangle_count(dA, dL, dU, stream=side, fused=False) == ref
    torch.cuda.synchronize()


def test_numeric_before_symbolic_is_a_state_error(sp):
    """spgemm_numeric on a plan whose symbolic phase has not run, or with
    operands other than the planned ones, returns SPGEMM_ERR_STATE (-6)."""
    import ctypes
    import torch
    from paper_1804_01698_amd import binding as b
    _note("case state errors")
    A = random_sparse(50, 40, 0.2, 1)
    B = random_sparse(40, 30, 0.2, 2)
    dA, dB = _dev(sp, A), _dev(sp, B)
    p = sp.Plan([dA], [dB])
    out_c = torch.empty(1, dtype=torch.int32, device="cuda")
    out_v = torch.empty(1, dtype=torch.float64, device="cuda")
    cc = (ctypes.c_void_p * 1)(out_c.data_ptr())
    cv = (ctypes.c_void_p * 1)(out_v.data_ptr())
    assert b._lib.spgemm_numeric(p._h, p._ca, p._cb, cc, cv) == -6
    p.symbolic()
    other = _dev(sp, random_sparse(50, 40, 0.2, 3))
    ca = (b._Csr * 1)(other._c())
    C = p.allocate_output()[0]
    cc = (ctypes.c_void_p * 1)(C.cols.data_ptr())
    cv = (ctypes.c_void_p * 1)(C.vals.data_ptr())
    assert b._lib.spgemm_numeric(p._h, ca, p._cb, cc, cv) == -6      # not the planned A
    assert b._lib.spgemm_numeric(p._h, p._ca, p._cb, cc, cv) == 0
    torch.cuda.synchronize()
    assert_matches(C, oracle.spgemm(A, B), True)
    p.close()


def test_repeated_input_columns_add_up(sp):
    """A row of A or B may repeat a column (the library's documented reading):
    its products add up, as the oracle computes when repeats are allowed."""
    _note("case repeated input columns")
    rng = np.random.default_rng(8)
    for seed in range(3):
        A = random_sparse(200, 150, 0.05, 30 + seed)
        B = random_sparse(150, 300, 0.05, 40 + seed)
        # repeat about a tenth of the entries of each operand inside their rows
        def dup(X, s):
            r = np.random.default_rng(s)
            rows, cols, vals = [], [], []
            for i in range(X.nrows):
                c = X.cols[X.rpts[i]:X.rpts[i + 1]]
                v = X.vals[X.rpts[i]:X.rpts[i + 1]]
                pick = r.random(c.size) < 0.1
                cc = np.concatenate([c, c[pick]])
                vv = np.concatenate([v, r.random(int(pick.sum()))])
                o = r.permutation(cc.size)
                rows.append(cc[o]); vals.append(vv[o])
            rp = np.zeros(X.nrows + 1, dtype=np.int64)
            np.cumsum([x.size for x in rows], out=rp[1:])
            return CSR(X.nrows, X.ncols, rp, np.concatenate(rows).astype(np.int32), np.concatenate(vals))
        Ad, Bd = dup(A, seed), dup(B, seed + 10)
        for srt in (True, False):
            C = _run(sp, Ad, Bd, srt)
            assert_matches(C, oracle.spgemm(Ad, Bd, sorted_output=srt, allow_duplicates=True), srt)
