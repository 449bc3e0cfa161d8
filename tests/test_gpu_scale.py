"""GPU parity at the full sizes of the measured workloads, in the launch
configuration bench.py times.

Products too large for a full host-side comparison are checked row by row:
every row count (hence all int64 row pointers) against the oracle's symbolic
phase, and a sample of rows -- random ones plus the heaviest -- entry by entry
against the oracle on those rows (rows of C are independent)."""
import sys

import numpy as np
import pytest

import oracle
from synth import (bfs_frontier, erdos_renyi_fixed_degree, rmat, symmetric_rmat_graph,
                   triangle_inputs, with_values)

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


def _product(sp, A, B, sorted_output):
    import torch
    dA = sp.DeviceCSR.from_host(A, device="cuda")
    dB = dA if B is A else sp.DeviceCSR.from_host(B, device="cuda")
    p = sp.Plan([dA], [dB], sorted_output=sorted_output)
    p.symbolic()
    C = p.numeric()[0]
    torch.cuda.synchronize()
    st = p.stats(0)
    p.close()
    assert st["status"] == 0 and st["probe_overflow"] == 0
    return C, st


def _sample_rows(f, n_random, n_heavy, seed):
    rng = np.random.default_rng(seed)
    heavy = np.argsort(f)[-n_heavy:]
    rand = rng.choice(f.size, n_random, replace=False)
    return np.unique(np.concatenate([heavy, rand, [0, f.size - 1]]))


def _check_large(sp, A, sorted_output, n_random, n_heavy):
    C, st = _product(sp, A, A, sorted_output)
    ref_rp = oracle.symbolic(A, A)
    rp = C.rpts.cpu().numpy()
    assert np.array_equal(rp, ref_rp), "row pointers differ from the oracle's symbolic phase"
    f = oracle.row_flop(A, A)
    assert st["flop"] == int(f.sum()) and st["nnz_C"] == int(ref_rp[-1])
    rows = _sample_rows(f, n_random, n_heavy, 7)
    ref = oracle.spgemm(A, A, sorted_output=sorted_output, rows=rows)
    assert_rows_match(C, ref, rows, sorted_output)
    return C, st


def test_er_2p20_unsorted(sp):
    """ER n=2^20, 16 distinct uniform columns per row, A*A, unsorted output."""
    _note("case er20 full size")
    A = erdos_renyi_fixed_degree(1 << 20, 16, 1, sorted_rows=False)
    C, st = _check_large(sp, A, False, 20000, 100)
    assert st["flop"] == (1 << 20) * 256


def test_rmat_scale20_unsorted(sp):
    """R-MAT scale 20 ef 16 A*A (9.7e9 entries: int64 row pointers), unsorted."""
    _note("case rmat20 full size")
    A = rmat(20, 16, 1, sorted_rows=False)
    C, st = _check_large(sp, A, False, 300, 60)
    assert st["nnz_C"] > 2**31
    assert st["heavy_rows"] > 100000 and st["windows"] > st["heavy_rows"]


def test_rmat_scale18_sorted(sp):
    _note("case rmat18 sorted")
    A = rmat(18, 16, 2)
    _check_large(sp, A, True, 2000, 100)


def test_triangles_scale18(sp):
    """Triangle count on symmetric R-MAT scale 18 ef 16: the fused masked count
    in natural order (L*U would hold 2.4e9 entries) and degree order, and the
    formed product in degree order, against the oracle on the degree-ordered
    graph (the count does not depend on the vertex order)."""
    _note("case triangles scale 18")
    g = symmetric_rmat_graph(18, 16, 1)
    A0, L0, U0 = triangle_inputs(g, degree_order=False)
    A1, L1, U1 = triangle_inputs(g, degree_order=True)
    ref = oracle.triangle_count(A1, L1, U1)
    dev = lambda a: sp.DeviceCSR.from_host(a, device="cuda")
    t1 = sp.triangle_count(dev(A1), dev(L1), dev(U1))
    assert t1 == ref
    t0 = sp.triangle_count(dev(A0), dev(L0), dev(U0))
    assert t0 == ref
    assert sp.triangle_count(dev(A1), dev(L1), dev(U1), fused=False) == ref
    _note(f"triangles: {ref}")


def test_bfs_scale18(sp):
    """Multi-source BFS step: A (R-MAT scale 18, int64 ones) times F (n x 512)."""
    _note("case bfs scale 18")
    A = with_values(rmat(18, 16, 3, values=""), 0, "ones")
    F = bfs_frontier(A.ncols, 512, 4)
    for srt in (True, False):
        C, st = _product(sp, A, F, srt)
        assert_matches(C, oracle.spgemm(A, F, sorted_output=srt), srt)
