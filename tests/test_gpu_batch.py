"""Batched products (one launch sequence for many small products) against the
oracle, product by product; graph capture and replay of a batch."""
import sys

import numpy as np
import pytest

import oracle
from synth import (erdos_renyi_fixed_degree, random_sparse, rmat, serving_request_operands,
                   serving_stream, shuffle_within_rows, with_values)

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


def _mixed_products(n, seed, small=True):
    reqs = serving_stream(n, seed, max_flop=2**18 if small else None, n_hi=8192)
    pairs, flags = [], []
    for r in reqs:
        a, b = serving_request_operands(r)
        pairs.append((a, b))
        flags.append(r.sorted_out)
    return pairs, flags


def test_batch_matches_oracle(sp):
    import torch
    _note("case batch mixed f64")
    pairs, flags = _mixed_products(40, 3)
    pairs.append((random_sparse(0, 5, 0.5, 1), random_sparse(5, 7, 0.5, 2)))      # empty product
    flags.append(True)
    pairs.append((random_sparse(30, 20, 0.0, 1), random_sparse(20, 9, 0.3, 2)))   # all rows empty
    flags.append(False)
    # fixed-degree products whose rows fall in the 4096-, 8192- and 16384-slot
    # tables (key bounds 1600, 2500 and 4900 with 20,000 columns)
    for d, seed in ((40, 61), (50, 62), (70, 63)):
        a = erdos_renyi_fixed_degree(600, d, seed, ncols=20000)
        b = erdos_renyi_fixed_degree(20000, d, seed + 10)
        pairs.append((a, b))
        flags.append(seed % 2 == 0)
    dev = [(sp.DeviceCSR.from_host(a), sp.DeviceCSR.from_host(b)) for a, b in pairs]
    bt = sp.Batch([x for x, _ in dev], [y for _, y in dev], flags)
    bins = bt.bin_rows()
    assert all(bins[b] > 0 for b in range(1, 10)), bins    # every LDS table size is used
    assert bins[10] == 0 and sum(bins) == sum(a.nrows for a, _ in pairs)
    bt.run()
    torch.cuda.synchronize()
    outs = bt.outputs()
    for (a, b), f, C in zip(pairs, flags, outs):
        assert C is not None
        assert_matches(C, oracle.spgemm(a, b, sorted_output=f), f)
    assert sum(bt.flop) == sum(int(oracle.row_flop(a, b).sum()) for a, b in pairs)


def test_batch_i64_and_unsupported_row(sp):
    import torch
    _note("case batch i64 + out-of-range row")
    a1 = random_sparse(50, 40, 0.2, 4, values="i64")
    b1 = random_sparse(40, 60, 0.2, 5, values="i64")
    big = with_values(rmat(14, 16, 2, values=""), 3, "i64")          # hub rows above the batched range
    a3 = random_sparse(64, 64, 0.1, 6, values="i64")
    pairs = [(a1, b1), (big, big), (a3, a3)]
    dev = [(sp.DeviceCSR.from_host(a), sp.DeviceCSR.from_host(b)) for a, b in pairs]
    bt = sp.Batch([x for x, _ in dev], [y for _, y in dev], [True, True, False])
    assert bt.max_key[1] > sp.BATCH_XMAX
    bt.run()
    torch.cuda.synchronize()
    outs = bt.outputs()
    assert bt.status == [0, -8, 0]
    assert outs[1] is None
    assert_matches(outs[0], oracle.spgemm(a1, b1, sorted_output=True), True)
    assert_matches(outs[2], oracle.spgemm(a3, a3, sorted_output=False), False)


def test_batch_graph_replay(sp):
    """A captured batch replayed several times, with eager work in between,
    gives the eager result every time."""
    import torch
    _note("case batch graph replay")
    pairs, flags = _mixed_products(24, 5)
    dev = [(sp.DeviceCSR.from_host(a), sp.DeviceCSR.from_host(b)) for a, b in pairs]
    bt = sp.Batch([x for x, _ in dev], [y for _, y in dev], flags)
    bt.run()
    torch.cuda.synchronize()
    eager = [(c.rpts.clone(), c.cols.clone(), c.vals.clone()) for c in bt.outputs()]
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bt.run(stream=torch.cuda.current_stream())
    for rep in range(3):
        bt.arena.zero_()
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()       # unrelated eager work
        g.replay()
        torch.cuda.synchronize()
        for (rp, cl, vl), c, srt in zip(eager, bt.outputs(), flags):
            assert torch.equal(rp, c.rpts)
            a, b = _row_major(rp, cl, vl, srt), _row_major(c.rpts, c.cols, c.vals, srt)
            assert np.array_equal(a[0], b[0])
            assert np.allclose(a[1], b[1], rtol=1e-12, atol=0)
        del junk


def test_batch_replay_api(sp):
    """Batch.replay(): the captured launch sequence replayed after the operand
    values change (structure fixed) gives the product of the new values."""
    import torch
    _note("case batch replay api")
    pairs, flags = _mixed_products(16, 7)
    dev = [(sp.DeviceCSR.from_host(a), sp.DeviceCSR.from_host(b)) for a, b in pairs]
    bt = sp.Batch([x for x, _ in dev], [y for _, y in dev], flags)
    for rep in range(3):
        scale = float(rep + 1)
        for (a, b), (_, db) in zip(pairs, dev):
            db.vals.copy_(torch.from_numpy(b.vals * scale).to(db.vals.device))
        bt.replay()
        torch.cuda.synchronize()
        for (a, b), f, C in zip(pairs, flags, bt.outputs()):
            b2 = type(b)(b.nrows, b.ncols, b.rpts, b.cols, b.vals * scale)
            assert_matches(C, oracle.spgemm(a, b2, sorted_output=f), f)


def _row_major(rp, cl, vl, srt):
    """Columns and values of a product; unsorted rows (whose order depends on
    which thread claimed each table slot) are put in column order first."""
    rp, cl, vl = rp.cpu().numpy(), cl.cpu().numpy(), vl.cpu().numpy()
    if srt:
        return cl, vl
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    o = np.lexsort((cl, rows))
    return cl[o], vl[o]
