"""MI355X (gfx950) hash-table SpGEMM: Python binding of ``libspgemm.so``.

Only argument marshalling lives here: every step of the product runs in the HIP
kernels of the library (``csrc/``).  PyTorch supplies device memory and the
stream.  The binding raises ``ImportError`` when the library has not been built:
there is no CPU fallback.
"""
from .binding import (
    Batch,
    BATCH_XMAX,
    batch_arena_bytes,
    batch_scratch_bytes,
    config_ok,
    default_config,
    plan_scratch_bytes,
    DeviceCSR,
    Plan,
    SpgemmError,
    F64,
    I64,
    SORTED,
    VALIDATE,
    lib_path,
    masked_product_sum_i64,
    masked_sum_i64,
    spgemm,
    stanza_read,
    stream_copy,
    triangle_count,
)

__all__ = [
    "Batch", "BATCH_XMAX", "batch_arena_bytes", "batch_scratch_bytes", "plan_scratch_bytes", "config_ok", "default_config", "DeviceCSR", "Plan", "SpgemmError", "F64", "I64", "SORTED", "VALIDATE", "lib_path",
    "masked_product_sum_i64", "masked_sum_i64", "spgemm", "stanza_read", "stream_copy", "triangle_count",
]
