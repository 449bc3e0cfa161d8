"""The Heap accumulator (Section 4.2.3) as a plan option, the collision-factor
counters of Eq. 2, and the plan's device row flop, against the oracle."""
import sys

import numpy as np
import pytest

import oracle
from synth import (CSR, erdos_renyi_fixed_degree, random_sparse, rmat, sort_within_rows,
                   symmetric_rmat_graph, triangle_inputs, with_values)

from _compare import assert_matches

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


def _heap_product(sp, A, B, heap=1, **kw):
    import torch
    dA = sp.DeviceCSR.from_host(A, device="cuda")
    dB = dA if B is A else sp.DeviceCSR.from_host(B, device="cuda")
    cfg = dict(sp.default_config(), heap=heap)
    p = sp.Plan([dA], [dB], sorted_output=True, config=cfg, **kw)
    p.symbolic()
    C = p.numeric()[0]
    torch.cuda.synchronize()
    st = p.stats(0)
    p.close()
    assert st["status"] == 0, st
    return C, st


def test_heap_degree_ordered_lu(sp):
    """L*U of a symmetric R-MAT graph in degree order (the low-compression
    product of Section 5.6), int64 ones: exact against the oracle."""
    _note("case heap L*U degree order scale 14")
    g = symmetric_rmat_graph(14, 16, 2)
    A, L, U = triangle_inputs(g, degree_order=True)
    C, st = _heap_product(sp, L, U)
    assert st["heap_rows"] > 0
    assert_matches(C, oracle.spgemm(L, U, sorted_output=True), True)


def test_heap_uniform_square(sp):
    """A*A of a fixed-degree ER matrix (sorted rows): every row lies in the heap
    envelope (16 entries of A, 256 products)."""
    _note("case heap ER n=2^13 d=16")
    A = erdos_renyi_fixed_degree(1 << 13, 16, 3, sorted_rows=True)
    C, st = _heap_product(sp, A, A)
    assert st["heap_rows"] == A.nrows
    assert_matches(C, oracle.spgemm(A, A, sorted_output=True), True)


def test_heap_matches_hash_path_rmat(sp):
    """R-MAT A*A with the heap option: rows inside the envelope merge, the rest
    (wide rows, heavy rows) keep the hash tables and windows; the product is
    the oracle's either way (f64 to 1e-12)."""
    _note("case heap R-MAT scale 14")
    A = rmat(14, 16, 4)
    C, st = _heap_product(sp, A, A)
    assert 0 < st["heap_rows"] < A.nrows and st["heavy_rows"] > 0
    assert_matches(C, oracle.spgemm(A, A, sorted_output=True), True)


def test_heap_repeated_columns(sp):
    """Repeated columns inside sorted rows of B and repeated k inside rows of A
    (they add up, as in the oracle): int64 exact."""
    _note("case heap repeated columns")
    rng = np.random.default_rng(7)
    def dup(m, n, per):
        rp = np.arange(0, m * per + 1, per, dtype=np.int64)
        cols = rng.integers(0, n, m * per).astype(np.int32)
        vals = rng.integers(1, 50, m * per).astype(np.int64)
        return sort_within_rows(CSR(m, n, rp, cols, vals))
    A = dup(300, 200, 9)
    B = dup(200, 500, 12)
    C, st = _heap_product(sp, A, B)
    assert st["heap_rows"] > 0
    ref = oracle.spgemm(A, B, sorted_output=True, allow_duplicates=True)
    assert_matches(C, ref, True)


def test_heap_rejects_unsorted_b(sp):
    _note("case heap unsorted B")
    A = rmat(10, 8, 5, sorted_rows=False)
    with pytest.raises(sp.SpgemmError) as ei:
        _heap_product(sp, A, A)
    assert ei.value.status == -8


def test_plan_row_flop_is_fig4(sp):
    _note("case plan row flop")
    A = random_sparse(3000, 2000, 0.003, 11)
    B = random_sparse(2000, 2500, 0.004, 12)
    dA, dB = sp.DeviceCSR.from_host(A, device="cuda"), sp.DeviceCSR.from_host(B, device="cuda")
    p = sp.Plan([dA], [dB], sorted_output=False)
    assert np.array_equal(p.row_flop(0).astype(np.int64), oracle.row_flop(A, B).astype(np.int64))
    p.close()


def test_plan_row_flop_every_row_class(sp):
    """Per-row flop on the device against the oracle for rows summed by a
    thread (at most 32 entries), by a wave from the list of longer rows (up to
    4096) and by a block from the list of the longest, several hundred of the
    middle class so that the list spans many waves."""
    _note("case plan row flop, every row class")
    rng = np.random.default_rng(5)
    nb = 50000
    rows_b = [np.unique(rng.integers(0, 1 << 20, size=int(L))) for L in rng.integers(0, 41, size=nb)]
    B = CSR(nb, 1 << 20, np.concatenate([[0], np.cumsum([len(r) for r in rows_b])]),
            np.concatenate(rows_b).astype(np.int32), None)        # 0 to 40 entries per row
    lens = np.concatenate([rng.integers(0, 33, size=3000), rng.integers(33, 4097, size=600),
                           [0, 1, 32, 33, 4096, 4097, 10000, 40000]])
    rng.shuffle(lens)
    cols = np.concatenate([np.sort(rng.choice(nb, size=int(L), replace=False)) for L in lens])
    A = CSR(len(lens), nb, np.concatenate([[0], np.cumsum(lens)]), cols.astype(np.int32), None)
    A, B = with_values(A, 1, "f64"), with_values(B, 2, "f64")
    dA, dB = sp.DeviceCSR.from_host(A, device="cuda"), sp.DeviceCSR.from_host(B, device="cuda")
    p = sp.Plan([dA], [dB], sorted_output=False)
    ref = oracle.row_flop(A, B).astype(np.int64)
    assert np.array_equal(p.row_flop(0).astype(np.int64), ref)
    assert p.stats(0)["flop"] == int(ref.sum())
    p.close()


@pytest.mark.parametrize("degenerate", [False, True])
def test_collision_factor_counters(sp, degenerate):
    """Probe counters (SPGEMM_PROBE_COUNT): every insertion makes at least one
    LDS probe, so probes >= flop per bin; under the hash that sends every key
    to bucket 0, probes grow like the square of the keys per row."""
    import torch
    _note(f"case probe counters degenerate={degenerate}")
    A = rmat(12, 8, 6)
    dA = sp.DeviceCSR.from_host(A, device="cuda")
    cfg = dict(sp.default_config(), hash_mul=0) if degenerate else None
    p = sp.Plan([dA], [dA], sorted_output=False, config=cfg, probe_count=True)
    p.symbolic()
    C = p.numeric()[0]
    torch.cuda.synchronize()
    st = p.stats(0)
    p.close()
    assert st["status"] == 0
    ref = oracle.spgemm(A, A, sorted_output=False)
    assert_matches(C, ref, False)
    flop = oracle.row_flop(A, A).astype(np.int64)
    assert sum(st["sym_flop"]) + sum(st["num_flop"]) > 0
    for f, pr in zip(st["sym_flop"] + st["num_flop"], st["sym_probes"] + st["num_probes"]):
        assert pr >= f
        assert pr <= f * (16384 // 4 + 1)
    c_sym = sum(st["sym_probes"]) / max(sum(st["sym_flop"]), 1)
    _note(f"collision factor c (symbolic, all bins) = {c_sym:.3f}")
    if degenerate:
        assert c_sym > 4.0
    else:
        assert c_sym < 2.0
    # the same plan without counting reports no probes
    p = sp.Plan([dA], [dA], sorted_output=False)
    p.symbolic()
    st2 = p.stats(0)
    p.close()
    assert sum(st2["sym_probes"]) == 0 and st2["sym_flop"] == st["sym_flop"]
    assert int(flop.sum()) == st["flop"]
