"""GPU parity on the paper's other synthetic workloads (Section 5.4 density and
size sweeps, Section 5.5 square x tall-skinny) at sizes the oracle finishes in
seconds, and the stanza read probe against a host sum of the same words."""
import sys

import numpy as np
import pytest

import oracle
from synth import column_sample, erdos_renyi_fixed_degree, rmat

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


def _product(sp, A, B, sorted_output):
    import torch
    dA = sp.DeviceCSR.from_host(A, device="cuda")
    dB = dA if B is A else sp.DeviceCSR.from_host(B, device="cuda")
    C = sp.spgemm(dA, dB, sorted_output=sorted_output)
    torch.cuda.synchronize()
    return C


@pytest.mark.parametrize("family", ["er", "g500"])
@pytest.mark.parametrize("ef", [2, 64])
@pytest.mark.parametrize("sorted_output", [True, False])
def test_density_extremes(sp, family, ef, sorted_output):
    _note(f"case density family={family} ef={ef} sorted={sorted_output}")
    if family == "er":
        A = erdos_renyi_fixed_degree(1 << 11, ef, 3, sorted_rows=sorted_output)
    else:
        A = rmat(11, ef, 3, sorted_rows=sorted_output)
    C = _product(sp, A, A, sorted_output)
    assert_matches(C, oracle.spgemm(A, A, sorted_output=sorted_output), sorted_output)


@pytest.mark.parametrize("family", ["er", "g500"])
@pytest.mark.parametrize("scale", [7, 9])
def test_size_small(sp, family, scale):
    _note(f"case size family={family} scale={scale}")
    A = (erdos_renyi_fixed_degree(1 << scale, 16, 4, sorted_rows=False) if family == "er"
         else rmat(scale, 16, 4, sorted_rows=False))
    C = _product(sp, A, A, False)
    assert_matches(C, oracle.spgemm(A, A, sorted_output=False), False)


@pytest.mark.parametrize("logk", [8, 11])
@pytest.mark.parametrize("sorted_output", [True, False])
def test_tall_skinny(sp, logk, sorted_output):
    _note(f"case tall_skinny scale=13 k=2^{logk} sorted={sorted_output}")
    A = rmat(13, 16, 5, sorted_rows=sorted_output)
    B = column_sample(A, 1 << logk, 9)
    C = _product(sp, A, B, sorted_output)
    assert_matches(C, oracle.spgemm(A, B, sorted_output=sorted_output), sorted_output)


@pytest.mark.parametrize("lw", [0, 3, 7, 12])
def test_stanza_read_sum(sp, lw):
    import torch
    _note(f"case stanza lw={lw}")
    rng = np.random.default_rng(lw + 1)
    nwords = 1 << 22
    host = rng.integers(0, 1 << 62, size=nwords, dtype=np.int64).view(np.uint64)
    L = 1 << lw
    nst = max(8, (1 << 20) >> lw)
    starts = rng.integers(0, nwords - L + 1, size=nst, dtype=np.int64)
    starts[:3] = [-1, nwords - L + 1, nwords]        # do not fit: skipped, not read
    ok = (starts >= 0) & (starts <= nwords - L)
    idx = (starts[ok][:, None] + np.arange(L, dtype=np.int64)[None, :]).ravel()
    want = int(host[idx].sum(dtype=np.uint64))
    base = torch.from_numpy(host.view(np.int64)).to("cuda")
    st = torch.from_numpy(starts).to("cuda")
    out = sp.stanza_read(base, st, lw)
    torch.cuda.synchronize()
    got_sum, got_skipped = [int(x) for x in out.cpu().numpy().view(np.uint64)]
    assert got_skipped == int((~ok).sum())
    assert got_sum == want


def test_stanza_read_rejects_bad_arguments(sp):
    import torch
    base = torch.zeros(16, dtype=torch.int64, device="cuda")
    st = torch.zeros(4, dtype=torch.int64, device="cuda")
    with pytest.raises(sp.SpgemmError):
        sp.stanza_read(base, st, 25)
    with pytest.raises(sp.SpgemmError):
        sp.stanza_read(base, st.to(torch.int32), 0)


@pytest.mark.parametrize("nbytes", [16, 16 * 1023, 16 * (4096 * 4 + 7), 16 * ((1 << 22) + 5)])
def test_stream_copy_is_exact(sp, nbytes):
    """The copy-rate probe copies every byte (ragged tails of its 4-deep
    per-lane steps included) and nothing past the count."""
    import torch
    _note(f"case stream copy {nbytes} bytes")
    g = torch.Generator(device="cpu").manual_seed(nbytes)
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, generator=g).to("cuda")
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    sp.stream_copy(dst[:nbytes], src)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src)
    assert int(dst[nbytes:].sum()) == 0
