"""GPU parity where the persistent kernels claim rows from counters: bins with
more rows than twice their grid (so that claims, not the fixed first rows,
hand out most of them), the bitmap bin and the column windows, with the
numeric phase run twice on one symbolic result (the claim counters of the
numeric phase must start again from zero)."""
import sys

import numpy as np
import pytest

import oracle
from synth import CSR, erdos_renyi_fixed_degree, with_values

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


def _stack(parts, ncols):
    rp = [np.zeros(1, np.int64)]
    cols, vals, base = [], [], 0
    for p in parts:
        rp.append(p.rpts[1:] + base)
        base += p.nnz
        cols.append(p.cols)
        vals.append(p.vals)
    return CSR(sum(p.nrows for p in parts), ncols, np.concatenate(rp), np.concatenate(cols),
               np.concatenate(vals))


def _operands():
    """B: 4096 rows of 100 distinct columns out of 2^20 (products of one row of
    A rarely share a column).  A: 2500 rows each of 15, 30 and 60 entries
    (nnz(c_i) about 1500, 3000 and 6000: numeric bins of 2048, 4096 and 8448
    entries, symbolic bins of 2048, 4096 and 8448 keys) and 200 rows of 100
    entries (about 10^4 entries each: heavy rows, column windows)."""
    nb = 4096
    B = erdos_renyi_fixed_degree(nb, 100, 11, ncols=1 << 20)
    parts = [erdos_renyi_fixed_degree(n, d, 20 + d, ncols=nb) for n, d in ((2500, 15), (2500, 30), (2500, 60), (200, 100))]
    return _stack(parts, nb), B


def test_claimed_rows_and_numeric_rerun(sp):
    import torch
    _note("case claims: bins above twice their grid, heavy rows, numeric twice")
    A1, B1 = _operands()
    A2, B2 = with_values(A1, 5, "f64"), with_values(B1, 6, "f64")
    d1a, d1b = sp.DeviceCSR.from_host(A1, device="cuda"), sp.DeviceCSR.from_host(B1, device="cuda")
    d2a, d2b = sp.DeviceCSR.from_host(A2, device="cuda"), sp.DeviceCSR.from_host(B2, device="cuda")
    d2a.rpts, d2a.cols, d2b.rpts, d2b.cols = d1a.rpts, d1a.cols, d1b.rpts, d1b.cols
    p = sp.Plan([d1a], [d1b], sorted_output=False)
    p.symbolic()
    st = p.stats(0)
    # numeric bins 7, 8 and 9 (list index b - 1) and the windows all hold rows
    assert all(st["num_flop"][b - 1] > 0 for b in (7, 8, 9)), st["num_flop"]
    assert all(st["sym_flop"][b - 1] > 0 for b in (8, 9)), st["sym_flop"]
    assert st["heavy_rows"] == 200 and st["windows"] > 200, st
    C = p.numeric()[0]
    torch.cuda.synchronize()
    assert_matches(C, oracle.spgemm(A1, B1, sorted_output=False), False)
    del C
    C = p.numeric([d2a], [d2b])[0]
    torch.cuda.synchronize()
    assert_matches(C, oracle.spgemm(A2, B2, sorted_output=False), False)
    assert p.stats(0)["status"] == 0
    p.close()
