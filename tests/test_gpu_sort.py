"""Sorted output against the oracle on rows built to stress the in-LDS sorts:
keys crowded into a few buckets of the row's [min, max] range (a cluster
plus a far outlier), keys spanning fewer columns than there are buckets, and
rows of every bin width, through the single-product path and a batch."""
import sys

import numpy as np
import pytest

import oracle
from synth.csr import CSR

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


def _csr(nrows, ncols, rows, seed):
    """CSR with the given column lists per row and seeded FP64 values."""
    rng = np.random.default_rng(seed)
    rp = np.zeros(nrows + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    cols = np.concatenate([np.asarray(r, dtype=np.int32) for r in rows]) if rp[-1] else np.zeros(0, np.int32)
    return CSR(nrows, ncols, rp, cols, rng.random(int(rp[-1])))


def _clustered(n_b, ncols, band, spread, seed):
    """B whose row k holds a band of `band` consecutive columns starting below
    `spread`, plus the last column: the products' rows crowd a few low
    buckets and stretch [min, max] to the whole width."""
    rng = np.random.default_rng(seed)
    rows = []
    for k in range(n_b):
        s = int(rng.integers(0, spread))
        rows.append(list(range(s, s + band)) + [ncols - 1])
    return _csr(n_b, ncols, rows, seed + 1)


@pytest.mark.parametrize("deg,band,spread", [(2, 20, 80), (8, 30, 120), (32, 40, 2000), (64, 64, 8000),
                                             (128, 64, 16000)])
def test_sorted_clustered_rows(sp, deg, band, spread):
    """Row sizes from the 64-slot bin to the 8192- and 11264-slot bins (2^20
    columns: too wide for the rank passes), every row's keys in a cluster at
    the low end plus one key at the last column."""
    _note(f"case sorted clustered deg={deg} band={band} spread={spread}")
    ncols = 1 << 20
    B = _clustered(4096, ncols, band, spread, 11 + deg)
    rng = np.random.default_rng(5 + deg)
    A = _csr(512, 4096, [sorted(rng.choice(4096, size=deg, replace=False).tolist()) for _ in range(512)], 7)
    dA, dB = sp.DeviceCSR.from_host(A), sp.DeviceCSR.from_host(B)
    C = sp.spgemm(dA, dB, sorted_output=True)
    assert_matches(C, oracle.spgemm(A, B, sorted_output=True), True)


def test_sorted_dense_span(sp):
    """Rows whose keys span fewer columns than there are buckets (one bucket
    per column value) and rows whose keys are every column of a range."""
    _note("case sorted dense span")
    rng = np.random.default_rng(3)
    B = _csr(256, 300, [sorted(rng.choice(300, size=int(rng.integers(1, 40)), replace=False).tolist())
                        for _ in range(256)], 4)
    A = _csr(300, 256, [sorted(rng.choice(256, size=int(rng.integers(0, 24)), replace=False).tolist())
                        for _ in range(300)], 5)
    dA, dB = sp.DeviceCSR.from_host(A), sp.DeviceCSR.from_host(B)
    C = sp.spgemm(dA, dB, sorted_output=True)
    assert_matches(C, oracle.spgemm(A, B, sorted_output=True), True)


def test_batch_sorted_clustered(sp):
    """The same stress through the batched path (sorted per product flag)."""
    import torch
    _note("case batch sorted clustered")
    pairs = []
    for deg, band, spread in ((4, 16, 64), (16, 30, 600), (40, 50, 4000)):
        B = _clustered(2048, 1 << 18, band, spread, 21 + deg)
        rng = np.random.default_rng(9 + deg)
        A = _csr(128, 2048, [sorted(rng.choice(2048, size=deg, replace=False).tolist()) for _ in range(128)], 8)
        pairs.append((A, B))
    dev = [(sp.DeviceCSR.from_host(a), sp.DeviceCSR.from_host(b)) for a, b in pairs]
    bt = sp.Batch([x for x, _ in dev], [y for _, y in dev], True)
    bt.run()
    torch.cuda.synchronize()
    for (a, b), C in zip(pairs, bt.outputs()):
        assert_matches(C, oracle.spgemm(a, b, sorted_output=True), True)
