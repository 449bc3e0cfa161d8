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


def assert_blocks_match(C, A, B, sorted_output: bool, max_entries: float = 4e8, rtol: float = FP64_RTOL,
                        note=None):
    """Every row of the device product C = A*B against the oracle, in
    contiguous row blocks of at most ``max_entries`` entries (rows of C are
    independent, so a block of the oracle equals the same rows of the whole
    product).  The oracle's block is copied to the device and, for unsorted
    output, both sides are put in (row, column) order there before the entries
    are compared; row pointers are compared on the host.  Returns the number of
    blocks."""
    import oracle
    import torch
    dev = C.cols.device
    rp = C.rpts.cpu().numpy()
    m = C.nrows
    nblocks = 0
    r0 = 0
    while r0 < m:
        r1 = int(np.searchsorted(rp, rp[r0] + max_entries, side="right")) - 1
        r1 = min(max(r1, r0 + 1), m)
        ref = oracle.spgemm(A, B, sorted_output=sorted_output, rows=np.arange(r0, r1, dtype=np.int64),
                            validate_inputs=False)
        assert np.array_equal(rp[r0:r1 + 1] - rp[r0], ref.rpts), f"row pointers differ in rows [{r0}, {r1})"
        p0, p1 = int(rp[r0]), int(rp[r1])
        if p1 > p0:
            gc, gv = C.cols[p0:p1], C.vals[p0:p1]
            oc = torch.from_numpy(ref.cols).to(dev)
            ov = torch.from_numpy(ref.vals).to(dev)
            if not sorted_output:
                lens = torch.from_numpy(np.diff(ref.rpts)).to(dev)
                rowid = torch.repeat_interleave(torch.arange(r1 - r0, device=dev, dtype=torch.int64), lens)
                kg, og = torch.sort(rowid * C.ncols + gc.to(torch.int64))
                ko, oo = torch.sort(rowid * C.ncols + oc.to(torch.int64))
                del rowid, lens
                assert torch.equal(kg, ko), f"column sets differ in rows [{r0}, {r1})"
                del kg, ko
                gv, ov = gv[og], ov[oo]
                del og, oo
            else:
                assert torch.equal(gc, oc), f"columns differ in rows [{r0}, {r1}) (sorted mode)"
            if ov.dtype == torch.int64:
                assert torch.equal(gv, ov), f"int64 values differ in rows [{r0}, {r1})"
            else:
                nz = ov != 0
                assert bool((gv[~nz] == 0).all()), f"zero entries differ in rows [{r0}, {r1})"
                if bool(nz.any()):
                    rel = float(((gv[nz] - ov[nz]).abs() / ov[nz].abs()).max())
                    assert rel <= rtol, f"max relative error {rel:.3e} in rows [{r0}, {r1})"
            del gc, gv, oc, ov
        nblocks += 1
        if note is not None:
            note(f"  rows [{r0}, {r1}) match ({p1 - p0} entries)")
        r0 = r1
    return nblocks
