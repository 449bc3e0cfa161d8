"""Seeded synthetic CSR inputs shared by the tests, the benchmark and the smoke check.

This package only *draws* inputs (matrix structure, values, request streams) and
converts between layouts.  It holds none of the sparse-product arithmetic: the CPU
reference (``oracle/``) and the HIP library (``paper_1804_01698_amd``) each compute
the product on their own from what these functions return.
"""
from .csr import CSR, to_dense, from_dense, transpose, shuffle_within_rows, sort_within_rows, validate
from .generators import (
    erdos_renyi_fixed_degree,
    rmat,
    rmat_edges,
    symmetric_rmat_graph,
    triangle_inputs,
    bfs_frontier,
    column_sample,
    identity,
    permutation_matrix,
    random_sparse,
    with_values,
    ServingRequest,
    serving_stream,
    serving_request_operands,
    WORKLOADS,
    workload,
)

__all__ = [
    "CSR", "to_dense", "from_dense", "transpose", "shuffle_within_rows", "sort_within_rows", "validate",
    "erdos_renyi_fixed_degree", "rmat", "rmat_edges", "symmetric_rmat_graph", "triangle_inputs",
    "bfs_frontier", "column_sample", "identity", "permutation_matrix", "random_sparse", "with_values",
    "ServingRequest", "serving_stream", "serving_request_operands", "WORKLOADS", "workload",
]
