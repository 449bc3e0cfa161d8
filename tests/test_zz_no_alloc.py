"""spgemm_symbolic_static (symbolic phase in the library's static per-GPU
workspace) against spgemm_symbolic with a caller workspace, through the C ABI:
two products in a row on the same GPU, the second smaller, each compared
entry by entry with the caller-workspace result and with the oracle; a plan
whose workspace exceeds the static scratch is rejected before any work."""
import sys

import numpy as np
import pytest

import oracle
from synth import erdos_renyi_fixed_degree, rmat, shuffle_within_rows

from _compare import assert_matches

pytestmark = pytest.mark.gpu

STATIC_WS_BYTES = 64 << 20
ERR_STATIC_LIMIT = -11


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


def _run(sp, A, sorted_output, static):
    import torch
    dA = sp.DeviceCSR.from_host(A, device="cuda")
    p = sp.Plan([dA], [dA], sorted_output=sorted_output, defer_workspace=static)
    assert p.workspace_bytes <= STATIC_WS_BYTES
    nnz = p.symbolic_static() if static else p.symbolic()
    C = p.numeric()[0]
    torch.cuda.synchronize()
    st = p.stats(0)
    p.close()
    assert st["status"] == 0 and st["probe_overflow"] == 0
    assert p.workspace is None or not static
    return nnz[0], C, st


def _same(C1, C0, sorted_output):
    """C1 (static workspace) equals C0 (caller workspace): row pointers and
    columns bit-exact (as sets per row when unsorted), values to 1e-12."""
    r1, c1, v1 = C1.to_host()
    r0, c0, v0 = C0.to_host()
    assert np.array_equal(r1, r0)
    rows = np.repeat(np.arange(C0.nrows, dtype=np.int64), np.diff(r0))
    o1 = np.lexsort((c1, rows)) if not sorted_output else np.arange(c1.size)
    o0 = np.lexsort((c0, rows)) if not sorted_output else np.arange(c0.size)
    assert np.array_equal(c1[o1], c0[o0])
    a, b = v1[o1], v0[o0]
    nz = b != 0
    assert np.all(a[~nz] == 0)
    if nz.any():
        assert float(np.max(np.abs(a[nz] - b[nz]) / np.abs(b[nz]))) <= 1e-12


@pytest.mark.parametrize("sorted_output", [False, True])
def test_static_workspace_matches_caller_workspace(sp, sorted_output):
    # the first product has rows above the LDS tables (bitmap symbolic, column
    # windows, bucketed B: the workspace's largest parts); the second is smaller
    cases = [("rmat scale 14", shuffle_within_rows(rmat(14, 16, 5), 6)),
             ("er n=3000 d=7", erdos_renyi_fixed_degree(3000, 7, 8, sorted_rows=False))]
    for name, A in cases:
        _note(f"case static workspace {name} sorted={sorted_output}")
        n1, C1, st1 = _run(sp, A, sorted_output, static=True)
        n0, C0, st0 = _run(sp, A, sorted_output, static=False)
        assert n1 == n0 == st0["nnz_C"]
        assert st1["heavy_rows"] == st0["heavy_rows"] and st1["windows"] == st0["windows"]
        _same(C1, C0, sorted_output)
        assert_matches(C1, oracle.spgemm(A, A, sorted_output=sorted_output), sorted_output)
        if name.startswith("rmat"):
            assert st1["heavy_rows"] > 0 and st1["windows"] >= st1["heavy_rows"]
    assert st0["heavy_rows"] == 0


def test_static_workspace_rejects_large_plans(sp):
    import torch
    _note("case static workspace over the limit")
    A = rmat(18, 16, 9)
    dA = sp.DeviceCSR.from_host(A, device="cuda")
    p = sp.Plan([dA], [dA], sorted_output=False, defer_workspace=True)
    assert p.workspace_bytes > STATIC_WS_BYTES
    with pytest.raises(sp.SpgemmError) as ei:
        p.symbolic_static()
    assert ei.value.status == ERR_STATIC_LIMIT
    assert "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    # the plan is untouched: the caller-workspace path still runs it
    p.symbolic()
    p.numeric()
    torch.cuda.synchronize()
    assert p.stats(0)["status"] == 0
    p.close()
