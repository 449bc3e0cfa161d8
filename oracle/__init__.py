"""CPU oracle for row-wise SpGEMM (Gustavson with a sparse accumulator).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_1804_01698_amd``) never imports it, and it never imports the product
path; they share no code.  The arithmetic lives in ``spgemm_oracle.c`` (plain C,
OpenMP over flop-balanced row blocks); this module is ctypes marshalling plus a
few plain-numpy helpers.

Every function cites the passage of the paper it restates.  Pins (checks of this
oracle against things other than itself) live in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from synth.csr import CSR

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names another build of spgemm_oracle.c (the sanitized one of the
# sanitizer test); default: the in-tree liboracle.so
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

F64, I64 = 0, 1


def build(force: bool = False) -> str:
    """Compile the oracle (gcc -O2 -fopenmp).  Returns the library path."""
    from .build import build_oracle
    return build_oracle(force=force)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        if "ORACLE_LIB" in os.environ:
            raise FileNotFoundError(_LIB_PATH)
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    p = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.oracle_row_flop.restype = i64
    lib.oracle_row_flop.argtypes = [i64, p, p, p, p, p, ctypes.c_int]
    lib.oracle_rows_to_threads.restype = None
    lib.oracle_rows_to_threads.argtypes = [i64, p, ctypes.c_int, p]
    lib.oracle_symbolic.restype = i64
    lib.oracle_symbolic.argtypes = [i64, p, i64, p, p, p, p, p, ctypes.c_int]
    lib.oracle_numeric.restype = ctypes.c_int
    lib.oracle_numeric.argtypes = [ctypes.c_int, ctypes.c_int, i64, p, i64,
                                   p, p, p, p, p, p, p, p, p, ctypes.c_int]
    lib.oracle_masked_sum_i64.restype = i64
    lib.oracle_masked_sum_i64.argtypes = [i64, i64, p, p, p, p, p, ctypes.c_int]
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_validate_csr.restype = ctypes.c_int
    lib.oracle_validate_csr.argtypes = [i64, i64, i64, p, p, ctypes.c_int]
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _prep(a: CSR):
    rp = np.ascontiguousarray(a.rpts, dtype=np.int64)
    cols = np.ascontiguousarray(a.cols, dtype=np.int32)
    return rp, cols


def _rows_arg(rows, nrows):
    if rows is None:
        return None, nrows
    r = np.ascontiguousarray(rows, dtype=np.int64)
    return r, r.size


_CSR_RULES = {
    1: "rpts[0] != 0",
    2: "row pointers decrease",
    3: "rpts[nrows] != nnz",
    4: "column id outside [0, ncols)",
    5: "column repeated within a row",
    6: "scratch memory unavailable",
}


def validate(a: CSR, allow_duplicates: bool = False) -> None:
    """Structure check of a CSR operand (CSR as defined in Section 2): row
    pointers start at 0, never decrease and end at nnz, column ids lie in
    [0, ncols) and, unless ``allow_duplicates``, no row repeats a column.
    Raises ValueError naming the first rule that fails."""
    lib = _load()
    rp, cols = _prep(a)
    if rp.size != a.nrows + 1:
        raise ValueError("malformed CSR: rpts must have nrows + 1 entries")
    if a.vals is not None and np.asarray(a.vals).size != cols.size:
        raise ValueError("malformed CSR: vals and cols differ in length")
    # nnz is the length of the column array; rule 3 checks that rpts ends there
    st = lib.oracle_validate_csr(a.nrows, a.ncols, cols.size, _ptr(rp), _ptr(cols), 0 if allow_duplicates else 1)
    if st:
        raise ValueError(f"malformed CSR: {_CSR_RULES.get(st, st)}")


def _check_operands(A: CSR, B: CSR, validate_inputs: bool, allow_duplicates: bool) -> None:
    if A.ncols != B.nrows:
        raise ValueError("A.ncols != B.nrows")
    if validate_inputs:
        validate(A, allow_duplicates)
        if B is not A:
            validate(B, allow_duplicates)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def row_flop(A: CSR, B: CSR, rows=None, nthreads: int = 0, validate_inputs: bool = True,
             allow_duplicates: bool = True) -> np.ndarray:
    """flop of each (selected) row of C = A*B: the sum over stored a_ik of nnz(b_k*)
    (Fig. 4, part 1).  Counts multiplications (Section 2, flop definition); a
    repeated column counts once per occurrence."""
    _check_operands(A, B, validate_inputs, allow_duplicates)
    lib = _load()
    rpa, ca = _prep(A)
    rpb, _ = _prep(B)
    r, n = _rows_arg(rows, A.nrows)
    out = np.empty(n, dtype=np.int64)
    lib.oracle_row_flop(n, _ptr(r), _ptr(rpa), _ptr(ca), _ptr(rpb), _ptr(out), nthreads)
    return out


def rows_to_threads(flop: np.ndarray, tnum: int) -> np.ndarray:
    """Fig. 4, part 2: thread t gets rows [offset[t], offset[t+1]); offset[t] is the
    first row whose exclusive flop prefix reaches t*total/tnum (lower bound)."""
    lib = _load()
    f = np.ascontiguousarray(flop, dtype=np.int64)
    off = np.empty(tnum + 1, dtype=np.int64)
    lib.oracle_rows_to_threads(f.size, _ptr(f), tnum, _ptr(off))
    return off


def symbolic(A: CSR, B: CSR, rows=None, nthreads: int = 0, validate_inputs: bool = True,
             allow_duplicates: bool = False) -> np.ndarray:
    """Symbolic phase (Section 2 two-phase method; Fig. 5): int64 row pointers of
    C (or of the selected rows of C) from the number of distinct columns per row.
    Operands are validated first (``validate``) unless ``validate_inputs`` is
    False (for callers that validated them once already)."""
    _check_operands(A, B, validate_inputs, allow_duplicates)
    lib = _load()
    rpa, ca = _prep(A)
    rpb, cb = _prep(B)
    r, n = _rows_arg(rows, A.nrows)
    rp = np.empty(n + 1, dtype=np.int64)
    tot = lib.oracle_symbolic(n, _ptr(r), B.ncols, _ptr(rpa), _ptr(ca), _ptr(rpb), _ptr(cb),
                              _ptr(rp), nthreads)
    if tot < 0:
        raise MemoryError("oracle symbolic: scratch allocation failed")
    return rp


def _dtype_code(A: CSR, B: CSR):
    if A.vals is None or B.vals is None:
        raise ValueError("numeric phase needs values")
    if A.vals.dtype == np.float64 and B.vals.dtype == np.float64:
        return F64, np.float64
    if A.vals.dtype == np.int64 and B.vals.dtype == np.int64:
        return I64, np.int64
    raise TypeError("values must both be float64 or both int64")


def spgemm(A: CSR, B: CSR, sorted_output: bool = True, rows=None, nthreads: int = 0,
           validate_inputs: bool = True, allow_duplicates: bool = False) -> CSR:
    """C = A*B by Gustavson's row-wise algorithm (Fig. 1) with a sparse accumulator
    (Section 2), two-phase (symbolic then numeric, Fig. 5).  ``rows`` selects a
    subset of rows of C (returned in the given order); rows of C are independent
    (Section 2), so this equals the same rows of the full product.  Operands are
    validated first (see ``validate``; a repeated column in a row is rejected
    unless ``allow_duplicates``, and then its products simply add up)."""
    code, dt = _dtype_code(A, B)
    rp = symbolic(A, B, rows, nthreads, validate_inputs, allow_duplicates)
    lib = _load()
    rpa, ca = _prep(A)
    rpb, cb = _prep(B)
    va = np.ascontiguousarray(A.vals, dtype=dt)
    vb = np.ascontiguousarray(B.vals, dtype=dt)
    r, n = _rows_arg(rows, A.nrows)
    nnz = int(rp[-1])
    cols = np.empty(nnz, dtype=np.int32)
    vals = np.empty(nnz, dtype=dt)
    st = lib.oracle_numeric(code, 1 if sorted_output else 0, n, _ptr(r), B.ncols,
                            _ptr(rpa), _ptr(ca), _ptr(va), _ptr(rpb), _ptr(cb), _ptr(vb),
                            _ptr(rp), _ptr(cols), _ptr(vals), nthreads)
    if st != 0:
        raise RuntimeError(f"oracle numeric failed ({st})")
    return CSR(n, B.ncols, rp, cols, vals)


def masked_sum(C: CSR, M: CSR, nthreads: int = 0) -> int:
    """Sum of C_ij over the positions stored in M (int64, wrap-around).  With
    C = L*U and M = A this is twice the triangle count (Section 5.6)."""
    if C.vals is None or C.vals.dtype != np.int64:
        raise TypeError("masked_sum needs int64 values")
    if C.nrows != M.nrows or C.ncols != M.ncols:
        raise ValueError("C and M differ in shape")
    validate(C, allow_duplicates=True)     # a product of this oracle: no repeats by construction
    validate(M)
    lib = _load()
    rpc, cc = _prep(C)
    rpm, cm = _prep(M)
    vc = np.ascontiguousarray(C.vals)
    return int(lib.oracle_masked_sum_i64(C.nrows, C.ncols, _ptr(rpc), _ptr(cc), _ptr(vc),
                                         _ptr(rpm), _ptr(cm), nthreads))


def triangle_count(A: CSR, L: CSR, U: CSR, nthreads: int = 0) -> int:
    """Triangles of the undirected graph A (Section 5.6): C = L*U counts, for each
    pair (i,j), the wedges i-k-j whose middle vertex k is below both; every
    triangle is closed by the edge (i,j) in both directions, hence /2."""
    C = spgemm(L, U, sorted_output=True, nthreads=nthreads)
    s = masked_sum(C, A, nthreads)
    if s % 2:
        raise AssertionError("masked sum of L*U over a symmetric A must be even")
    return s // 2


def lowest_p2(x: int) -> int:
    """Smallest power of two strictly greater than x (Fig. 5, table sizing)."""
    p = 1
    while p <= x:
        p <<= 1
    return p
