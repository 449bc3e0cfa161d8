"""Seeded generators for the workloads the paper measures on (Section 5).

Seeds: structure is drawn from ``seed``, values from ``seed + 1`` (after duplicate
merging, in CSR order), row shuffles from ``seed + 2``.  All arrays are numpy.

Readings of the paper taken here (the paper leaves them open):
  * Erdos-Renyi (ER): every row holds exactly ``d`` distinct columns drawn
    uniformly without replacement (the paper draws ER with R-MAT at
    a=b=c=d=0.25, Section 5.1; the fixed-degree form is the one measured here).
  * R-MAT (Section 5.1): ``edge_factor * 2**scale`` edges are drawn, each by
    ``scale`` independent quadrant choices with probabilities (a, b, c, d);
    no noise, no vertex permutation; duplicate edges are merged; self loops
    are kept for A*A.
  * Triangle inputs (Section 5.6): the R-MAT graph is symmetrised, self loops
    dropped, optionally relabelled by ascending degree (ties by vertex id), and
    split into strict lower L and strict upper U.
  * Multi-source BFS frontier (Section 5.5 use case): F is n x s with one
    nonzero per column, at a uniformly drawn row, value uniform in {1..1000}.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from .csr import CSR, shuffle_within_rows

G500 = (0.57, 0.19, 0.19, 0.05)
ER_RMAT = (0.25, 0.25, 0.25, 0.25)


def _rpts_from_rows(nrows: int, rows: np.ndarray) -> np.ndarray:
    rp = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=nrows), out=rp[1:])
    return rp


def with_values(a: CSR, seed: int, kind: str = "f64", lo: int = 1, hi: int = 1000) -> CSR:
    """Attach values drawn in CSR order: 'f64' U[0,1), 'i64' uniform {lo..hi}, 'ones' int64 1."""
    rng = np.random.default_rng(seed)
    if kind == "f64":
        v = rng.random(a.nnz)
    elif kind == "i64":
        v = rng.integers(lo, hi + 1, size=a.nnz, dtype=np.int64)
    elif kind == "ones":
        v = np.ones(a.nnz, dtype=np.int64)
    else:
        raise ValueError(kind)
    return CSR(a.nrows, a.ncols, a.rpts, a.cols, v)


def erdos_renyi_fixed_degree(n: int, d: int, seed: int, ncols: Optional[int] = None,
                             values: str = "f64", sorted_rows: bool = True) -> CSR:
    """n x ncols matrix, each row exactly ``d`` distinct uniform columns."""
    ncols = n if ncols is None else ncols
    if d > ncols:
        raise ValueError("d > ncols")
    rng = np.random.default_rng(seed)
    cols = np.empty((n, d), dtype=np.int64)
    todo = np.arange(n)
    while todo.size:
        draw = np.sort(rng.integers(0, ncols, size=(todo.size, d), dtype=np.int64), axis=1)
        ok = np.all(np.diff(draw, axis=1) != 0, axis=1) if d > 1 else np.ones(todo.size, bool)
        cols[todo[ok]] = draw[ok]
        todo = todo[~ok]
    rp = np.arange(0, n * d + 1, d, dtype=np.int64)
    a = CSR(n, ncols, rp, cols.reshape(-1).astype(np.int32), None)
    if values:
        a = with_values(a, seed + 1, values)
    if not sorted_rows:
        a = shuffle_within_rows(a, seed + 2)
    return a


def rmat_edges(scale: int, edge_factor: int, seed: int, abcd=G500):
    """Raw R-MAT edge list (row, col) as int64 arrays, duplicates included."""
    a, b, c, _ = abcd
    n_edges = edge_factor * (1 << scale)
    rng = np.random.default_rng(seed)
    rows = np.zeros(n_edges, dtype=np.int64)
    cols = np.zeros(n_edges, dtype=np.int64)
    t_ab, t_abc = np.float32(a + b), np.float32(a + b + c)
    t_a = np.float32(a)
    for level in range(scale):
        u = rng.random(n_edges, dtype=np.float32)
        bit = np.int64(1 << (scale - 1 - level))
        rbit = u >= t_ab
        cbit = ((u >= t_a) & (u < t_ab)) | (u >= t_abc)
        rows += rbit.astype(np.int64) * bit
        cols += cbit.astype(np.int64) * bit
        del u, rbit, cbit
    return rows, cols


def _csr_from_edges(n: int, rows: np.ndarray, cols: np.ndarray) -> CSR:
    key = np.unique(rows * n + cols)          # merges duplicates, sorts by (row, col)
    r = key // n
    c = (key - r * n).astype(np.int32)
    return CSR(n, n, _rpts_from_rows(n, r), c, None)


def rmat(scale: int, edge_factor: int, seed: int, abcd=G500, values: str = "f64",
         sorted_rows: bool = True) -> CSR:
    """2**scale square R-MAT matrix, duplicates merged, self loops kept."""
    n = 1 << scale
    r, c = rmat_edges(scale, edge_factor, seed, abcd)
    a = _csr_from_edges(n, r, c)
    del r, c
    if values:
        a = with_values(a, seed + 1, values)
    if not sorted_rows:
        a = shuffle_within_rows(a, seed + 2)
    return a


def symmetric_rmat_graph(scale: int, edge_factor: int, seed: int, abcd=G500) -> CSR:
    """Undirected simple graph (symmetric pattern, no self loops), int64 values 1."""
    n = 1 << scale
    r, c = rmat_edges(scale, edge_factor, seed, abcd)
    keep = r != c
    r, c = r[keep], c[keep]
    a = _csr_from_edges(n, np.concatenate([r, c]), np.concatenate([c, r]))
    return with_values(a, 0, "ones")


def relabel_by_degree(a: CSR) -> CSR:
    """Symmetric relabel P A P^T, vertices ordered by ascending degree, ties by id."""
    deg = a.row_lengths()
    order = np.lexsort((np.arange(a.nrows), deg))   # new id -> old id
    new_id = np.empty(a.nrows, dtype=np.int64)
    new_id[order] = np.arange(a.nrows)
    r = new_id[a.row_ids()]
    c = new_id[a.cols.astype(np.int64)]
    out = _csr_from_edges(a.nrows, r, c)
    return with_values(out, 0, "ones")


def triangle_inputs(a: CSR, degree_order: bool = False):
    """(A', L, U) with A' = A or its degree relabel, L/U its strict triangles (int64 ones)."""
    if degree_order:
        a = relabel_by_degree(a)
    rows = a.row_ids()
    cols = a.cols.astype(np.int64)
    lo = cols < rows
    up = cols > rows

    def part(mask):
        return with_values(CSR(a.nrows, a.ncols, _rpts_from_rows(a.nrows, rows[mask]),
                               cols[mask].astype(np.int32), None), 0, "ones")
    return a, part(lo), part(up)


def column_sample(a: CSR, k: int, seed: int) -> CSR:
    """Tall-skinny operand of Section 5.5: k distinct columns of ``a`` drawn
    uniformly (seeded), kept in ascending order and renumbered 0..k-1, with
    their entries and values; the row order of ``a`` is kept."""
    if not 0 < k <= a.ncols:
        raise ValueError("0 < k <= ncols required")
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(a.ncols, size=k, replace=False))
    new_id = np.full(a.ncols, -1, dtype=np.int64)
    new_id[pick] = np.arange(k)
    nc = new_id[a.cols.astype(np.int64)]
    keep = nc >= 0
    rows = a.row_ids()[keep]
    vals = None if a.vals is None else a.vals[keep]
    return CSR(a.nrows, k, _rpts_from_rows(a.nrows, rows), nc[keep].astype(np.int32), vals)


def bfs_frontier(n: int, nsources: int, seed: int) -> CSR:
    """n x nsources frontier stack: one nonzero per column, uniform row, value in {1..1000}."""
    rng = np.random.default_rng(seed)
    r = rng.integers(0, n, size=nsources, dtype=np.int64)
    v = rng.integers(1, 1001, size=nsources, dtype=np.int64)
    c = np.arange(nsources, dtype=np.int64)
    order = np.lexsort((c, r))
    return CSR(n, nsources, _rpts_from_rows(n, r[order]), c[order].astype(np.int32), v[order])


def identity(n: int, kind: str = "f64") -> CSR:
    v = np.ones(n, dtype=np.float64 if kind == "f64" else np.int64)
    return CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), v)


def permutation_matrix(perm: np.ndarray, kind: str = "f64") -> CSR:
    """P with P[i, perm[i]] = 1, so (P B) row i = B row perm[i]."""
    n = perm.size
    v = np.ones(n, dtype=np.float64 if kind == "f64" else np.int64)
    return CSR(n, n, np.arange(n + 1, dtype=np.int64), perm.astype(np.int32), v)


def random_sparse(m: int, n: int, density: float, seed: int, values: str = "f64",
                  empty_rows: float = 0.0, sorted_rows: bool = True) -> CSR:
    """Small random matrix: each entry present with probability ``density``;
    a fraction ``empty_rows`` of rows is forced empty."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    if empty_rows > 0 and m:
        mask[rng.random(m) < empty_rows] = False
    r, c = np.nonzero(mask)
    a = CSR(m, n, _rpts_from_rows(m, r), c.astype(np.int32), None)
    if values:
        a = with_values(a, seed + 1, values)
    if not sorted_rows:
        a = shuffle_within_rows(a, seed + 2)
    return a


# --------------------------------------------------------------------------- serving

@dataclass
class ServingRequest:
    rid: int
    arrival_s: float
    n: int
    d: int
    family: str          # "er" or "rmat"
    sorted_out: bool
    seed: int


def serving_stream(nreq: int, seed: int, rate_per_s: float = 1000.0,
                   n_lo: int = 256, n_hi: int = 131072, d_lo: int = 2, d_hi: int = 32,
                   max_flop: Optional[float] = None) -> List[ServingRequest]:
    """Poisson arrivals of independent C = A*B requests.

    n is log-uniform in [n_lo, n_hi] (rounded), nnz/row uniform in {d_lo..d_hi},
    ER / R-MAT 50/50, sorted / unsorted output 50/50.  ``max_flop`` (if given)
    keeps only requests whose expected flop n*d*d stays at or below it, which
    draws the small stratum of the same distribution.
    """
    rng = np.random.default_rng(seed)
    out: List[ServingRequest] = []
    t = 0.0
    rid = 0
    while len(out) < nreq:
        t += rng.exponential(1.0 / rate_per_s)
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        d = int(rng.integers(d_lo, d_hi + 1))
        fam = "er" if rng.random() < 0.5 else "rmat"
        srt = bool(rng.random() < 0.5)
        s = int(rng.integers(0, 2**31 - 8))
        if max_flop is not None and n * d * d > max_flop:
            continue
        out.append(ServingRequest(rid, t, n, min(d, n), fam, srt, s))
        rid += 1
    return out


def _rmat_n(n: int, d: int, seed: int) -> CSR:
    """R-MAT structure on n vertices (n need not be a power of two): drawn at
    scale ceil(log2 n), edges falling outside n x n are rejected, n*d edges kept."""
    scale = max(1, int(math.ceil(math.log2(n))))
    want = n * d
    rs, cs = [], []
    got = 0
    sub = seed
    while got < want:
        ef = max(1, int(math.ceil((want - got) / (1 << scale) * 1.3)) + 1)
        r, c = rmat_edges(scale, ef, sub)
        keep = (r < n) & (c < n)
        r, c = r[keep], c[keep]
        rs.append(r)
        cs.append(c)
        got += r.size
        sub += 7919
    r = np.concatenate(rs)[:want]
    c = np.concatenate(cs)[:want]
    return _csr_from_edges(n, r, c)


def serving_request_operands(req: ServingRequest):
    """(A, B) for one request: independent n x n operands of the request's family."""
    if req.family == "er":
        a = erdos_renyi_fixed_degree(req.n, req.d, req.seed, values="f64")
        b = erdos_renyi_fixed_degree(req.n, req.d, req.seed + 3, values="f64")
    else:
        a = with_values(_rmat_n(req.n, req.d, req.seed), req.seed + 1, "f64")
        b = with_values(_rmat_n(req.n, req.d, req.seed + 3), req.seed + 4, "f64")
    if not req.sorted_out:
        a = shuffle_within_rows(a, req.seed + 2)
        b = shuffle_within_rows(b, req.seed + 5)
    return a, b


# --------------------------------------------------------------------------- named workloads

WORKLOADS = {
    # name: (description, builder)
    "er4096": "C=A*A, ER n=4096, 8 distinct uniform cols/row, f64, sorted output",
    "rmat16": "C=A*A, R-MAT scale 16 ef 16 G500, f64 (sorted and unsorted runs)",
    "er20": "C=A*A, ER n=2^20, 16 distinct uniform cols/row, f64, unsorted",
    "rmat20": "C=A*A, R-MAT scale 20 ef 16 G500, f64, unsorted (rows shuffled)",
    "tri18": "triangles: symmetric R-MAT scale 18 ef 16, L*U int64, count = sum(C o A)/2",
    "bfs18": "C=A*F, A R-MAT scale 18 ef 16 int64 ones, F n x 512 one nonzero per column",
}


def workload(name: str, seed: int = 1, scale: Optional[int] = None, sorted_rows: Optional[bool] = None):
    """Build a named workload; ``scale`` shrinks it for quick runs (same recipe)."""
    if name == "er4096":
        n = 4096 if scale is None else (1 << scale)
        return erdos_renyi_fixed_degree(n, 8, seed, sorted_rows=True if sorted_rows is None else sorted_rows)
    if name == "rmat16":
        return rmat(16 if scale is None else scale, 16, seed,
                    sorted_rows=True if sorted_rows is None else sorted_rows)
    if name == "er20":
        n = (1 << 20) if scale is None else (1 << scale)
        return erdos_renyi_fixed_degree(n, 16, seed, sorted_rows=False if sorted_rows is None else sorted_rows)
    if name == "rmat20":
        return rmat(20 if scale is None else scale, 16, seed,
                    sorted_rows=False if sorted_rows is None else sorted_rows)
    raise KeyError(name)
