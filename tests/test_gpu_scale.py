"""GPU parity at the full sizes of the measured workloads, in the launch
configuration bench.py times.

Products too large for one host-side comparison are checked in row blocks:
the oracle computes a block of rows on its own (rows of C are independent),
the block goes to the device, and row pointers, column sets (or sorted
columns) and values are compared entry by entry, over every row."""
import sys

import numpy as np
import pytest

import oracle
from synth import (bfs_frontier, erdos_renyi_fixed_degree, rmat, symmetric_rmat_graph,
                   triangle_inputs, with_values)

from _compare import assert_blocks_match, assert_matches, assert_rows_match

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


def _check_large(sp, A, sorted_output):
    """The whole product on the device, every row against the oracle."""
    oracle.validate(A)
    C, st = _product(sp, A, A, sorted_output)
    f = oracle.row_flop(A, A, validate_inputs=False)
    assert st["flop"] == int(f.sum())
    n = assert_blocks_match(C, A, A, sorted_output, max_entries=4e8, note=_note)
    assert st["nnz_C"] == int(C.rpts.cpu()[-1].item())
    return C, st, n


def test_er_2p20_unsorted(sp):
    """ER n=2^20, 16 distinct uniform columns per row, A*A, unsorted output."""
    _note("case er20 full size")
    A = erdos_renyi_fixed_degree(1 << 20, 16, 1, sorted_rows=False)
    C, st, _ = _check_large(sp, A, False)
    assert st["flop"] == (1 << 20) * 256


def test_rmat_scale20_unsorted(sp):
    """R-MAT scale 20 ef 16 A*A (9.7e9 entries: int64 row pointers), unsorted:
    the whole product, every row, against the oracle in row blocks."""
    _note("case rmat20 full size, every row")
    A = rmat(20, 16, 1, sorted_rows=False)
    oracle.validate(A)
    C, st = _product(sp, A, A, False)
    assert st["nnz_C"] > 2**31
    assert st["heavy_rows"] > 100000 and st["windows"] > st["heavy_rows"]
    assert st["flop"] == int(oracle.row_flop(A, A, validate_inputs=False).sum())
    n = assert_blocks_match(C, A, A, False, max_entries=4e8, note=_note)
    assert C.rpts.cpu()[-1].item() == st["nnz_C"]
    _note(f"rmat20: {n} row blocks, {st['nnz_C']} entries compared")


def test_rmat_scale18_sorted(sp):
    _note("case rmat18 sorted")
    A = rmat(18, 16, 2)
    _check_large(sp, A, True)


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


def test_triangles_natural_order_formed_scale18(sp):
    """Triangle count on symmetric R-MAT scale 18 ef 16 in natural vertex order
    with C = L*U formed (Section 5.6): 2.45e9 entries (int64 row pointers past
    2^31), every row against the oracle (sorted mode, int64 values exact), and
    the masked sum of C over A equal to the oracle's count."""
    _note("case triangles scale 18 natural order, C formed")
    import torch
    g = symmetric_rmat_graph(18, 16, 1)
    A0, L0, U0 = triangle_inputs(g, degree_order=False)
    A1, L1, U1 = triangle_inputs(g, degree_order=True)
    ref = oracle.triangle_count(A1, L1, U1)            # the count does not depend on the order
    dev = lambda a: sp.DeviceCSR.from_host(a, device="cuda")
    dL, dU, dA = dev(L0), dev(U0), dev(A0)
    p = sp.Plan([dL], [dU], sorted_output=True)
    p.symbolic()
    C = p.numeric()[0]
    torch.cuda.synchronize()
    st = p.stats(0)
    p.close()
    assert st["status"] == 0 and st["probe_overflow"] == 0
    assert st["nnz_C"] > 2**31
    s = sp.masked_sum_i64(C, dA)
    assert s == 2 * ref, (s, ref)
    oracle.validate(L0)
    oracle.validate(U0)
    n = assert_blocks_match(C, L0, U0, True, max_entries=4e8, note=_note)
    _note(f"natural-order L*U: {st['nnz_C']} entries in {n} blocks, {ref} triangles")


def test_bfs_scale18(sp):
    """Multi-source BFS step: A (R-MAT scale 18, int64 ones) times F (n x 512)."""
    _note("case bfs scale 18")
    A = with_values(rmat(18, 16, 3, values=""), 0, "ones")
    F = bfs_frontier(A.ncols, 512, 4)
    for srt in (True, False):
        C, st = _product(sp, A, F, srt)
        assert_matches(C, oracle.spgemm(A, F, sorted_output=srt), srt)
