"""Host-side CSR container and layout helpers (no product arithmetic here).

CSR as the paper defines it (Section 2, the CSR paragraph): ``rpts`` of length
``nrows + 1``, ``cols`` and ``vals`` of length ``nnz``; the columns of row ``i``
are ``cols[rpts[i]:rpts[i+1]]``, in any order unless a function says otherwise.
Row pointers are held as int64 on the host; column ids as int32.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np


@dataclass
class CSR:
    nrows: int
    ncols: int
    rpts: np.ndarray            # int64[nrows + 1]
    cols: np.ndarray            # int32[nnz]
    vals: Optional[np.ndarray]  # float64[nnz] or int64[nnz] (None = pattern only)

    def __post_init__(self):
        self.rpts = np.ascontiguousarray(self.rpts, dtype=np.int64)
        self.cols = np.ascontiguousarray(self.cols, dtype=np.int32)
        if self.vals is not None:
            self.vals = np.ascontiguousarray(self.vals)

    @property
    def nnz(self) -> int:
        return int(self.rpts[-1]) if self.rpts.size else 0

    @property
    def shape(self):
        return (self.nrows, self.ncols)

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rpts)

    def row_ids(self) -> np.ndarray:
        """Row id of every stored entry (int64[nnz])."""
        return np.repeat(np.arange(self.nrows, dtype=np.int64), self.row_lengths())

    def copy(self) -> "CSR":
        return CSR(self.nrows, self.ncols, self.rpts.copy(), self.cols.copy(),
                   None if self.vals is None else self.vals.copy())

    def rows(self, r0: int, r1: int) -> "CSR":
        """Rows [r0, r1) as a CSR of their own (row pointers rebased to 0)."""
        a, b = int(self.rpts[r0]), int(self.rpts[r1])
        return CSR(r1 - r0, self.ncols, self.rpts[r0:r1 + 1] - a, self.cols[a:b],
                   None if self.vals is None else self.vals[a:b])

    def take_rows(self, ids) -> "CSR":
        """The listed rows, in the listed order, as a CSR of their own."""
        ids = np.asarray(ids, dtype=np.int64)
        lens = self.row_lengths()[ids]
        rp = np.zeros(ids.size + 1, dtype=np.int64)
        np.cumsum(lens, out=rp[1:])
        src = np.repeat(self.rpts[ids] - rp[:-1], lens) + np.arange(rp[-1], dtype=np.int64)
        return CSR(ids.size, self.ncols, rp, self.cols[src],
                   None if self.vals is None else self.vals[src])


def validate(a: CSR, allow_duplicates: bool = False) -> None:
    """Raise ValueError unless ``a`` is well-formed CSR."""
    rp = a.rpts
    if rp.shape != (a.nrows + 1,):
        raise ValueError("rpts has wrong length")
    if rp[0] != 0 or np.any(np.diff(rp) < 0):
        raise ValueError("rpts must start at 0 and be non-decreasing")
    if rp[-1] != a.cols.size:
        raise ValueError("rpts[-1] != len(cols)")
    if a.vals is not None and a.vals.size != a.cols.size:
        raise ValueError("len(vals) != len(cols)")
    if a.cols.size and (a.cols.min() < 0 or a.cols.max() >= a.ncols):
        raise ValueError("column index out of range")
    if not allow_duplicates and a.cols.size:
        key = a.row_ids() * max(a.ncols, 1) + a.cols.astype(np.int64)
        if np.unique(key).size != key.size:
            raise ValueError("duplicate column in a row")


def to_dense(a: CSR, dtype=None) -> np.ndarray:
    """Dense copy; duplicates (if any) are summed. Pattern-only CSR gives ones."""
    vals = a.vals if a.vals is not None else np.ones(a.nnz, dtype=np.int64)
    d = np.zeros((a.nrows, a.ncols), dtype=dtype or vals.dtype)
    np.add.at(d, (a.row_ids(), a.cols.astype(np.int64)), vals)
    return d


def from_dense(d: np.ndarray, pattern: Optional[np.ndarray] = None) -> CSR:
    """CSR of the entries where ``pattern`` (default ``d != 0``) holds, sorted rows."""
    mask = (d != 0) if pattern is None else pattern.astype(bool)
    r, c = np.nonzero(mask)
    rp = np.zeros(d.shape[0] + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=d.shape[0]), out=rp[1:])
    return CSR(d.shape[0], d.shape[1], rp, c.astype(np.int32), d[r, c].copy())


def _group_by_row(nrows: int, r: np.ndarray, c: np.ndarray, v, ncols: int) -> CSR:
    order = np.lexsort((c, r))
    r, c = r[order], c[order]
    rp = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=nrows), out=rp[1:])
    return CSR(nrows, ncols, rp, c.astype(np.int32), None if v is None else v[order])


def transpose(a: CSR) -> CSR:
    """Transpose with sorted rows."""
    return _group_by_row(a.ncols, a.cols.astype(np.int64), a.row_ids(), a.vals, a.nrows)


def sort_within_rows(a: CSR) -> CSR:
    order = np.lexsort((a.cols, a.row_ids()))
    return CSR(a.nrows, a.ncols, a.rpts.copy(), a.cols[order],
               None if a.vals is None else a.vals[order])


def shuffle_within_rows(a: CSR, seed: int) -> CSR:
    """Randomly permute the entries inside each row (row contents unchanged).

    This is the reading taken for the unsorted-output runs of the paper
    (Section 5.1, input types): entries of each input row are put in random
    order, which leaves the matrix itself, and hence A*A, unchanged.
    """
    rng = np.random.default_rng(seed)
    key = rng.random(a.nnz)
    order = np.lexsort((key, a.row_ids()))
    return CSR(a.nrows, a.ncols, a.rpts.copy(), a.cols[order],
               None if a.vals is None else a.vals[order])
