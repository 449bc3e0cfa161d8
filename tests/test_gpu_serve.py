"""Serving loop on the GPU: every result against the oracle, alone versus in
the mix, and admission under a small memory budget."""
import sys

import numpy as np
import pytest

import oracle
from synth import ServingRequest, serving_request_operands, serving_stream

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


def _stream_with_large(n, seed):
    """Small requests plus two R-MAT products whose hub rows exceed the batched range."""
    reqs = serving_stream(n, seed, n_hi=8192, rate_per_s=20000.0)
    t = reqs[-1].arrival_s
    reqs.append(ServingRequest(len(reqs), t * 0.3, 16384, 12, "rmat", True, 77))
    reqs.append(ServingRequest(len(reqs), t * 0.6, 16384, 8, "rmat", False, 78))
    return reqs


def _build(sp, reqs):
    from paper_1804_01698_amd.serve import Request
    host, dev = {}, []
    for r in reqs:
        a, b = serving_request_operands(r)
        host[r.rid] = (a, b, r.sorted_out)
        dev.append(Request(r.rid, r.arrival_s, sp.DeviceCSR.from_host(a), sp.DeviceCSR.from_host(b), r.sorted_out))
    return host, dev


class _Collect:
    def __init__(self):
        self.out = {}

    def __call__(self, req, C):
        rp, cl, vl = C.to_host()
        self.out[req.rid] = (rp, cl, vl)


class _HostC:
    def __init__(self, t):
        self.t = t

    def to_host(self):
        return self.t


def _check_all(host, got):
    for rid, (a, b, srt) in host.items():
        assert rid in got, f"request {rid} has no result"
        assert_matches(_HostC(got[rid]), oracle.spgemm(a, b, sorted_output=srt), srt)


def test_serve_matches_oracle_realtime(sp):
    from paper_1804_01698_amd.serve import Server
    _note("case serve realtime mix")
    reqs = _stream_with_large(40, 21)
    host, dev = _build(sp, reqs)
    col = _Collect()
    rep = Server(8 << 30, on_result=col).run(dev, realtime=True)
    s = rep.summary()
    _note(f"serve summary {s}")
    assert s["ok"] == len(reqs)
    assert s["planned"] >= 2 and s["batched"] >= len(reqs) - 2
    _check_all(host, col.out)
    for c in rep.completions:
        assert c.done_s >= c.arrival_s


def test_serve_budget_and_alone_vs_mix(sp):
    """A budget far below the mix's needs forces split batches and waiting; the
    results equal those of each request served alone (patterns exactly, values
    within the FP64 bound)."""
    from paper_1804_01698_amd.serve import Server
    _note("case serve small budget")
    reqs = _stream_with_large(30, 22)
    host, dev = _build(sp, reqs)
    col = _Collect()
    budget = 400 << 20           # every request fits alone, the whole mix does not
    rep = Server(budget, on_result=col, max_batch=8).run(dev, realtime=False)
    s = rep.summary()
    _note(f"budget summary {s}; batch sizes {rep.batch_sizes}")
    assert rep.peak_reserved_bytes <= budget
    assert s["ok"] == len(reqs), [(c.rid, c.path, c.status) for c in rep.completions if c.status]
    assert rep.batches >= 3 and max(rep.batch_sizes) <= 8
    _check_all(host, col.out)
    _note("case serve alone")
    for r in dev:
        one = _Collect()
        Server(8 << 30, on_result=one).run([r], realtime=False)
        rp0, cl0, vl0 = one.out[r.rid]
        rp1, cl1, vl1 = col.out[r.rid]
        assert np.array_equal(rp0, rp1)
        rows = np.repeat(np.arange(rp0.size - 1), np.diff(rp0))
        o0, o1 = np.lexsort((cl0, rows)), np.lexsort((cl1, rows))
        assert np.array_equal(cl0[o0], cl1[o1])
        nz = vl0[o0] != 0
        assert np.all(vl1[o1][~nz] == 0)
        assert np.all(np.abs(vl1[o1][nz] - vl0[o0][nz]) <= 1e-12 * np.abs(vl0[o0][nz]))


def test_serve_rejects_request_over_budget(sp):
    from paper_1804_01698_amd.serve import Server
    _note("case serve over budget")
    reqs = [ServingRequest(0, 0.0, 32768, 32, "rmat", True, 77), ServingRequest(1, 0.0, 512, 4, "er", True, 5)]
    host, dev = _build(sp, reqs)
    col = _Collect()
    rep = Server(4 << 20, on_result=col).run(dev, realtime=False)
    st = {c.rid: c.status for c in rep.completions}
    assert st[0] == -9 and st[1] == 0
    assert_matches(_HostC(col.out[1]), oracle.spgemm(*host[1][:2], sorted_output=True), True)
