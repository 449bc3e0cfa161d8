"""Comparison of a device product with the oracle (test infrastructure)."""
import numpy as np

FP64_RTOL = 1e-12   # per-entry relative bound: only the summation order differs


def host(C):
    """(rpts, cols, vals) numpy triple of a DeviceCSR."""
    return C.to_host()


def assert_matches(C, ref, sorted_output: bool, rtol: float = FP64_RTOL):
    rp, cols, vals = host(C)
    assert rp.shape == ref.rpts.shape, "row pointer length"
    assert np.array_equal(rp, ref.rpts), "row pointers differ"
    assert cols.shape == ref.cols.shape
    if sorted_output:
        assert np.array_equal(cols, ref.cols), "columns differ (sorted mode)"
        gv, rv = vals, ref.vals
    else:
        rows = np.repeat(np.arange(ref.nrows, dtype=np.int64), np.diff(ref.rpts))
        og = np.lexsort((cols, rows))
        orf = np.lexsort((ref.cols, rows))
        assert np.array_equal(cols[og], ref.cols[orf]), "column sets differ (unsorted mode)"
        gv, rv = vals[og], ref.vals[orf]
    if rv.dtype == np.int64:
        assert np.array_equal(gv, rv), "int64 values differ"
    else:
        nz = rv != 0
        assert np.all(gv[~nz] == 0), "zero entries differ"
        if nz.any():
            rel = np.abs(gv[nz] - rv[nz]) / np.abs(rv[nz])
            assert rel.max() <= rtol, f"max relative error {rel.max():.3e} > {rtol}"


def fetch_rows(C, rows):
    """Row pointers of C and the entries of the selected rows, copied from the
    device without copying the whole product."""
    import torch
    rp = C.rpts.cpu().numpy()
    rows = np.asarray(rows, dtype=np.int64)
    lens = rp[rows + 1] - rp[rows]
    sel = np.concatenate([np.arange(rp[i], rp[i + 1], dtype=np.int64) for i in rows]) if lens.sum() else \
        np.zeros(0, dtype=np.int64)
    idx = torch.from_numpy(sel).to(C.cols.device)
    cols = C.cols.index_select(0, idx).cpu().numpy()
    vals = C.vals.index_select(0, idx).cpu().numpy()
    sub_rp = np.zeros(rows.size + 1, dtype=np.int64)
    np.cumsum(lens, out=sub_rp[1:])
    return rp, sub_rp, cols, vals


def assert_rows_match(C, ref_rows, rows, sorted_output: bool, rtol: float = FP64_RTOL):
    """Selected rows of a device product against the oracle on those rows."""
    rp, sub_rp, cols, vals = fetch_rows(C, rows)
    assert np.array_equal(sub_rp, ref_rows.rpts), "row lengths differ"
    row_of = np.repeat(np.arange(len(rows), dtype=np.int64), np.diff(sub_rp))
    if sorted_output:
        assert np.array_equal(cols, ref_rows.cols), "columns differ (sorted mode)"
        gv, rv = vals, ref_rows.vals
    else:
        og = np.lexsort((cols, row_of))
        orf = np.lexsort((ref_rows.cols, row_of))
        assert np.array_equal(cols[og], ref_rows.cols[orf]), "column sets differ"
        gv, rv = vals[og], ref_rows.vals[orf]
    if rv.dtype == np.int64:
        assert np.array_equal(gv, rv)
    else:
        nz = rv != 0
        assert np.all(gv[~nz] == 0)
        if nz.any():
            rel = np.abs(gv[nz] - rv[nz]) / np.abs(rv[nz])
            assert rel.max() <= rtol, f"max relative error {rel.max():.3e}"
    return rp
