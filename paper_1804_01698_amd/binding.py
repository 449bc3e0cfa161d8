"""ctypes marshalling for the C ABI declared in include/spgemm.h."""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libspgemm.so")

F64, I64 = 0, 1
SORTED, VALIDATE, TIMING, LOW_MEMORY, PROBE_COUNT = 1, 2, 4, 8, 16
STATIC_WS_BYTES = 64 << 20          # SPGEMM_STATIC_WS_BYTES
PLAN_HDR_BYTES = 512                # plan scratch: header, then uint32 row flop per row
ERR_STATIC_LIMIT = -11


def lib_path() -> str:
    return _LIB


class SpgemmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {_lib.spgemm_strerror(status).decode()} (status {status})")


class _Csr(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rpts", ctypes.c_void_p), ("cols", ctypes.c_void_p), ("vals", ctypes.c_void_p)]


class _Stats(ctypes.Structure):
    _fields_ = [("flop", ctypes.c_int64), ("max_row_flop", ctypes.c_int64), ("nnz_C", ctypes.c_int64),
                ("heavy_rows", ctypes.c_int64), ("windows", ctypes.c_int64),
                ("probe_overflow", ctypes.c_int64), ("heap_rows", ctypes.c_int64),
                ("sym_flop", ctypes.c_int64 * 9), ("sym_probes", ctypes.c_int64 * 9),
                ("num_flop", ctypes.c_int64 * 9), ("num_probes", ctypes.c_int64 * 9)]


class _Config(ctypes.Structure):
    _fields_ = [("hash_mul", ctypes.c_uint32), ("sym_max", ctypes.c_int32 * 9), ("num_max", ctypes.c_int32 * 9),
                ("bucket_slots", ctypes.c_uint32), ("heap", ctypes.c_uint32)]


class _KTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("ms", ctypes.c_double), ("launches", ctypes.c_int64),
                ("alg_bytes", ctypes.c_double)]


def _load():
    if not os.path.exists(_LIB):
        raise ImportError(f"libspgemm.so is not built ({_LIB}); run __graft_entry__.build() "
                          "or python paper_1804_01698_amd/build.py")
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    pp = ctypes.POINTER(P)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.spgemm_plan_scratch_bytes.restype = ctypes.c_size_t
    lib.spgemm_plan_scratch_bytes.argtypes = [ctypes.c_int, ctypes.POINTER(_Csr)]
    lib.spgemm_plan.restype = ctypes.c_int
    lib.spgemm_plan.argtypes = [pp, ctypes.c_int, ctypes.POINTER(_Csr), ctypes.POINTER(_Csr), ctypes.c_int,
                                ctypes.c_uint, P, P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_Config)]
    lib.spgemm_config_default.restype = None
    lib.spgemm_config_default.argtypes = [ctypes.POINTER(_Config)]
    lib.spgemm_config_check.restype = ctypes.c_int
    lib.spgemm_config_check.argtypes = [ctypes.POINTER(_Config)]
    lib.spgemm_symbolic.restype = ctypes.c_int
    lib.spgemm_symbolic.argtypes = [P, P, pp, i64p]
    lib.spgemm_symbolic_static.restype = ctypes.c_int
    lib.spgemm_symbolic_static.argtypes = [P, pp, i64p]
    lib.spgemm_numeric.restype = ctypes.c_int
    lib.spgemm_numeric.argtypes = [P, ctypes.POINTER(_Csr), ctypes.POINTER(_Csr), pp, pp]
    lib.spgemm_free.restype = ctypes.c_int
    lib.spgemm_free.argtypes = [P]
    lib.spgemm_strerror.restype = ctypes.c_char_p
    lib.spgemm_strerror.argtypes = [ctypes.c_int]
    lib.spgemm_plan_stats.restype = ctypes.c_int
    lib.spgemm_plan_stats.argtypes = [P, ctypes.c_int, ctypes.POINTER(_Stats)]
    lib.spgemm_plan_set_timing.restype = ctypes.c_int
    lib.spgemm_plan_set_timing.argtypes = [P, ctypes.c_int]
    lib.spgemm_plan_kernel_times.restype = ctypes.c_int
    lib.spgemm_plan_kernel_times.argtypes = [P, ctypes.POINTER(_KTime), ctypes.c_int]
    lib.spgemm_masked_sum_i64.restype = ctypes.c_int
    lib.spgemm_masked_sum_i64.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P, ctypes.POINTER(_Csr), P, P]
    lib.spgemm_masked_product_sum_i64.restype = ctypes.c_int
    lib.spgemm_masked_product_sum_i64.argtypes = [ctypes.POINTER(_Csr), ctypes.POINTER(_Csr), ctypes.POINTER(_Csr),
                                                  P, P, P]
    lib.spgemm_stream_copy.restype = ctypes.c_int
    lib.spgemm_stream_copy.argtypes = [P, P, ctypes.c_size_t, P]
    lib.spgemm_stanza_read.restype = ctypes.c_int
    lib.spgemm_stanza_read.argtypes = [P, ctypes.c_size_t, P, ctypes.c_int64, ctypes.c_int, P, P, P]
    lib.spgemm_batch_scratch_bytes.restype = ctypes.c_size_t
    lib.spgemm_batch_scratch_bytes.argtypes = [ctypes.c_int, ctypes.POINTER(_Csr)]
    lib.spgemm_batch_prepare.restype = ctypes.c_int
    lib.spgemm_batch_prepare.argtypes = [ctypes.c_int, ctypes.POINTER(_Csr), ctypes.POINTER(_Csr),
                                         ctypes.POINTER(ctypes.c_uint), P, P]
    lib.spgemm_batch_analyse.restype = ctypes.c_int
    lib.spgemm_batch_analyse.argtypes = [ctypes.c_int, ctypes.POINTER(_Csr), P, i64p, i64p, i64p, P]
    lib.spgemm_batch_bin_rows.restype = ctypes.c_int
    lib.spgemm_batch_bin_rows.argtypes = [ctypes.c_int, ctypes.POINTER(_Csr), P, i64p, P]
    lib.spgemm_batch_arena_bytes.restype = ctypes.c_size_t
    lib.spgemm_batch_arena_bytes.argtypes = [ctypes.c_int, ctypes.POINTER(_Csr), i64p]
    lib.spgemm_batch_run.restype = ctypes.c_int
    lib.spgemm_batch_run.argtypes = [ctypes.c_int, ctypes.POINTER(_Csr), ctypes.c_int, i64p, P, P,
                                     ctypes.c_size_t, P, P]
    return lib


_lib = _load()


def _check(st: int, where: str):
    if st != 0:
        raise SpgemmError(st, where)


def _stream_handle(stream) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _on_stream(stream):
    """The torch stream the library's work goes to (``stream`` or the current
    one).  Buffers the library uses are allocated on it, so that torch's
    caching allocator never hands them to other work while the library's
    kernels still run."""
    return stream if stream is not None else torch.cuda.current_stream()


@dataclass
class DeviceCSR:
    """CSR operand resident in device memory (int32 rpts/cols; f64 or i64 vals).
    Row pointers of products are int64 (``rpts64``) since nnz(C) may exceed 2^31."""
    nrows: int
    ncols: int
    rpts: torch.Tensor                    # int32 [nrows+1] (operands) or int64 (products)
    cols: torch.Tensor                    # int32 [nnz]
    vals: Optional[torch.Tensor]          # float64 / int64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.cols.numel())

    @staticmethod
    def from_host(a, device="cuda", vals=True) -> "DeviceCSR":
        """From any object with nrows/ncols/rpts/cols/vals numpy fields."""
        if a.nnz >= 2**31 - 1:
            raise ValueError("operand nnz must be < 2^31 - 1")
        rp = torch.from_numpy(np.ascontiguousarray(a.rpts, dtype=np.int32)).to(device)
        cl = torch.from_numpy(np.ascontiguousarray(a.cols, dtype=np.int32)).to(device)
        vv = None
        if vals and a.vals is not None:
            vv = torch.from_numpy(np.ascontiguousarray(a.vals)).to(device)
        return DeviceCSR(int(a.nrows), int(a.ncols), rp, cl, vv)

    def to_host(self):
        """(rpts int64, cols int32, vals) as numpy arrays."""
        return (self.rpts.cpu().numpy().astype(np.int64), self.cols.cpu().numpy(),
                None if self.vals is None else self.vals.cpu().numpy())

    def _c(self) -> _Csr:
        if self.rpts.dtype != torch.int32:
            raise TypeError("operand row pointers must be int32")
        return _Csr(self.nrows, self.ncols, self.nnz, self.rpts.data_ptr(),
                    self.cols.data_ptr() if self.nnz else None,
                    self.vals.data_ptr() if (self.vals is not None and self.nnz) else None)


def _dtype_code(A: DeviceCSR, B: DeviceCSR) -> int:
    kinds = {t.vals.dtype for t in (A, B) if t.vals is not None}
    if kinds <= {torch.float64}:
        return F64
    if kinds == {torch.int64}:
        return I64
    raise TypeError("values must both be float64 or both be int64")


def default_config() -> dict:
    """The library's default plan configuration as a dict
    {hash_mul, sym_max[9], num_max[9], bucket_slots} (see spgemm_config)."""
    c = _Config()
    _lib.spgemm_config_default(ctypes.byref(c))
    return {"hash_mul": int(c.hash_mul), "sym_max": list(c.sym_max), "num_max": list(c.num_max),
            "bucket_slots": int(c.bucket_slots), "heap": int(c.heap)}


def _config_struct(cfg: Optional[dict]) -> Optional[_Config]:
    if cfg is None:
        return None
    c = _Config()
    c.hash_mul = int(cfg["hash_mul"]) & 0xFFFFFFFF
    for i in range(9):
        c.sym_max[i] = int(cfg["sym_max"][i])
        c.num_max[i] = int(cfg["num_max"][i])
    c.bucket_slots = int(cfg.get("bucket_slots", 4))
    c.heap = int(cfg.get("heap", 0))
    return c


def config_ok(cfg: dict) -> bool:
    """Whether the library accepts this configuration."""
    return _lib.spgemm_config_check(ctypes.byref(_config_struct(cfg))) == 0


class Plan:
    """One planned batch of products C[p] = A[p] @ B[p] (plan -> symbolic -> numeric).

    Device buffers (plan scratch, workspace, C) are torch tensors owned here;
    the library itself allocates no device memory."""

    def __init__(self, As: Sequence[DeviceCSR], Bs: Sequence[DeviceCSR], sorted_output: bool = True,
                 dtype: Optional[int] = None, validate: bool = False, stream=None, timing: bool = False,
                 defer_workspace: bool = False, config: Optional[dict] = None, low_memory: bool = False,
                 probe_count: bool = False):
        if len(As) != len(Bs) or not As:
            raise ValueError("need equal, non-empty lists of operands")
        self.As, self.Bs = list(As), list(Bs)
        self.n = len(As)
        self.dtype = _dtype_code(As[0], Bs[0]) if dtype is None else dtype
        self.sorted = bool(sorted_output)
        self.stream = stream
        self.device = As[0].rpts.device
        self._h = ctypes.c_void_p()
        self._ca = (_Csr * self.n)(*[a._c() for a in self.As])
        self._cb = (_Csr * self.n)(*[b._c() for b in self.Bs])
        nbytes = _lib.spgemm_plan_scratch_bytes(self.n, self._ca)
        with torch.cuda.stream(_on_stream(stream)):
            self.plan_scratch = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)
        ws = ctypes.c_size_t(0)
        flags = ((SORTED if self.sorted else 0) | (VALIDATE if validate else 0) | (TIMING if timing else 0)
                 | (LOW_MEMORY if low_memory else 0) | (PROBE_COUNT if probe_count else 0))
        cs = _config_struct(config)
        st = _lib.spgemm_plan(ctypes.byref(self._h), self.n, self._ca, self._cb, self.dtype, flags,
                              ctypes.c_void_p(self.plan_scratch.data_ptr()), _stream_handle(stream),
                              ctypes.byref(ws), None if cs is None else ctypes.byref(cs))
        _check(st, "spgemm_plan")
        self.workspace_bytes = int(ws.value)
        self.workspace = None
        if not defer_workspace:
            self.allocate_workspace()
        self.rpts_C: List[torch.Tensor] = []
        self.nnz_C: List[int] = []
        self.C: List[DeviceCSR] = []

    def allocate_workspace(self):
        if self.workspace is None:
            with torch.cuda.stream(_on_stream(self.stream)):
                self.workspace = torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=self.device)

    def output_bytes(self) -> int:
        """Device bytes of C (after symbolic): int32 columns and 8-byte values."""
        return 12 * sum(self.nnz_C)

    def symbolic(self) -> List[int]:
        self.allocate_workspace()
        with torch.cuda.stream(_on_stream(self.stream)):
            self.rpts_C = [torch.empty(a.nrows + 1, dtype=torch.int64, device=self.device) for a in self.As]
        arr = (ctypes.c_void_p * self.n)(*[t.data_ptr() for t in self.rpts_C])
        nnz = (ctypes.c_int64 * self.n)()
        st = _lib.spgemm_symbolic(self._h, ctypes.c_void_p(self.workspace.data_ptr()), arr, nnz)
        _check(st, "spgemm_symbolic")
        self.nnz_C = [int(x) for x in nnz]
        return self.nnz_C

    def symbolic_static(self) -> List[int]:
        """spgemm_symbolic_static: the symbolic phase in the library's static
        per-GPU workspace (no workspace tensor; rpts_C is still the caller's)."""
        with torch.cuda.stream(_on_stream(self.stream)):
            self.rpts_C = [torch.empty(a.nrows + 1, dtype=torch.int64, device=self.device) for a in self.As]
        arr = (ctypes.c_void_p * self.n)(*[t.data_ptr() for t in self.rpts_C])
        nnz = (ctypes.c_int64 * self.n)()
        st = _lib.spgemm_symbolic_static(self._h, arr, nnz)
        _check(st, "spgemm_symbolic_static")
        self.nnz_C = [int(x) for x in nnz]
        return self.nnz_C

    def allocate_output(self):
        vt = torch.float64 if self.dtype == F64 else torch.int64
        with torch.cuda.stream(_on_stream(self.stream)):
            self.C = [DeviceCSR(a.nrows, b.ncols, rp, torch.empty(nz, dtype=torch.int32, device=self.device),
                                torch.empty(nz, dtype=vt, device=self.device))
                      for a, b, rp, nz in zip(self.As, self.Bs, self.rpts_C, self.nnz_C)]
        return self.C

    def numeric(self, As: Optional[Sequence[DeviceCSR]] = None, Bs: Optional[Sequence[DeviceCSR]] = None):
        if As is not None:
            self.As = list(As)
            self._ca = (_Csr * self.n)(*[a._c() for a in self.As])
        if Bs is not None:
            self.Bs = list(Bs)
            self._cb = (_Csr * self.n)(*[b._c() for b in self.Bs])
        if not self.C:
            self.allocate_output()
        cc = (ctypes.c_void_p * self.n)(*[c.cols.data_ptr() for c in self.C])
        cv = (ctypes.c_void_p * self.n)(*[c.vals.data_ptr() for c in self.C])
        st = _lib.spgemm_numeric(self._h, self._ca, self._cb, cc, cv)
        _check(st, "spgemm_numeric")
        return self.C

    def stats(self, i: int = 0) -> dict:
        s = _Stats()
        st = _lib.spgemm_plan_stats(self._h, i, ctypes.byref(s))
        d = {}
        for f, _ in _Stats._fields_:
            v = getattr(s, f)
            d[f] = [int(x) for x in v] if isinstance(v, ctypes.Array) else int(v)
        d["status"] = st
        return d

    def row_flop(self, i: int = 0) -> np.ndarray:
        """Row flop of product i as the plan computed it on the device (Fig. 4
        part 1; uint32 per row, saturated at 2^32 - 1), copied to the host."""
        off = sum(_lib.spgemm_plan_scratch_bytes(1, ctypes.byref(self._ca[j])) for j in range(i))
        m = self.As[i].nrows
        t = self.plan_scratch[off + PLAN_HDR_BYTES: off + PLAN_HDR_BYTES + 4 * m]
        return t.view(torch.int32).cpu().numpy().view(np.uint32).copy()

    def kernel_times(self) -> List[dict]:
        buf = (_KTime * 64)()
        n = _lib.spgemm_plan_kernel_times(self._h, buf, 64)
        if n < 0:
            _check(n, "spgemm_plan_kernel_times")
        return [{"name": buf[i].name.decode(), "ms": buf[i].ms, "launches": int(buf[i].launches),
                 "alg_bytes": buf[i].alg_bytes} for i in range(n)]

    def close(self):
        if self._h:
            _lib.spgemm_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_scratch_bytes(As: Sequence[DeviceCSR]) -> int:
    """Device bytes Plan allocates before spgemm_plan (host-side query)."""
    ca = (_Csr * len(As))(*[a._c() for a in As])
    return int(_lib.spgemm_plan_scratch_bytes(len(As), ca))


def batch_scratch_bytes(As: Sequence[DeviceCSR]) -> int:
    """Device scratch bytes of a batch with these left operands."""
    ca = (_Csr * len(As))(*[a._c() for a in As])
    return int(_lib.spgemm_batch_scratch_bytes(len(As), ca))


def batch_arena_bytes(As: Sequence[DeviceCSR], bounds: Sequence[int]) -> int:
    """Arena bytes of a batch with these left operands and per-product bounds."""
    ca = (_Csr * len(As))(*[a._c() for a in As])
    b = (ctypes.c_int64 * len(As))(*bounds)
    return int(_lib.spgemm_batch_arena_bytes(len(As), ca, b))


BATCH_RESULT_BYTES = 48   # spgemm_batch_result: 5 x int64 + 2 x int32
BATCH_XMAX = 8448          # rows above this key bound are outside the batched range


class Batch:
    """Many small products C[p] = A[p] @ B[p] through one fixed sequence of
    launches (spgemm_batch_*).  Construction uploads the batch and analyses it
    (row flop and bins; synchronises the stream) and, unless
    ``allocate=False``, allocates the arena (``arena_bytes``).  ``run()``
    enqueues kernels only (capturable in a HIP graph); ``outputs()`` reads the
    per-product results back and returns views into the arena."""

    def __init__(self, As: Sequence[DeviceCSR], Bs: Sequence[DeviceCSR], sorted_flags=True,
                 dtype: Optional[int] = None, stream=None, allocate: bool = True):
        if len(As) != len(Bs) or not As:
            raise ValueError("need equal, non-empty lists of operands")
        self.As, self.Bs = list(As), list(Bs)
        self.n = len(As)
        self.dtype = _dtype_code(As[0], Bs[0]) if dtype is None else dtype
        self.device = As[0].rpts.device
        self.stream = stream
        if isinstance(sorted_flags, bool):
            sorted_flags = [sorted_flags] * self.n
        self.sorted = [bool(x) for x in sorted_flags]
        self._ca = (_Csr * self.n)(*[a._c() for a in self.As])
        self._cb = (_Csr * self.n)(*[b._c() for b in self.Bs])
        nb = _lib.spgemm_batch_scratch_bytes(self.n, self._ca)
        if nb == 0:
            raise SpgemmError(-1, "spgemm_batch_scratch_bytes: invalid batch")
        with torch.cuda.stream(_on_stream(stream)):
            self.scratch = torch.empty(nb, dtype=torch.uint8, device=self.device)
        flags = (ctypes.c_uint * self.n)(*[SORTED if x else 0 for x in self.sorted])
        _check(_lib.spgemm_batch_prepare(self.n, self._ca, self._cb, flags,
                                         ctypes.c_void_p(self.scratch.data_ptr()), _stream_handle(stream)),
               "spgemm_batch_prepare")
        self._flop = (ctypes.c_int64 * self.n)()
        self._bound = (ctypes.c_int64 * self.n)()
        self._maxk = (ctypes.c_int64 * self.n)()
        _check(_lib.spgemm_batch_analyse(self.n, self._ca, ctypes.c_void_p(self.scratch.data_ptr()), self._flop,
                                         self._bound, self._maxk, _stream_handle(stream)), "spgemm_batch_analyse")
        self.flop = [int(x) for x in self._flop]
        self.bound = [int(x) for x in self._bound]
        self.max_key = [int(x) for x in self._maxk]
        self.arena_bytes = int(_lib.spgemm_batch_arena_bytes(self.n, self._ca, self._bound))
        self.arena = None
        self.results = None
        self.status: List[int] = []
        self._graph = None
        if allocate:
            self.allocate()

    def bin_rows(self) -> List[int]:
        """Rows of the batch per bin: [empty, bins 1..9 (the LDS table sizes),
        outside the batched range] (spgemm_batch_bin_rows)."""
        out = (ctypes.c_int64 * 11)()
        _check(_lib.spgemm_batch_bin_rows(self.n, self._ca, ctypes.c_void_p(self.scratch.data_ptr()), out,
                                          _stream_handle(self.stream)), "spgemm_batch_bin_rows")
        return [int(x) for x in out]

    @property
    def supported(self) -> List[bool]:
        """Products whose every row lies inside the batched range."""
        return [k <= BATCH_XMAX for k in self.max_key]

    def allocate(self):
        if self.arena is None:
            with torch.cuda.stream(_on_stream(self.stream)):
                self.arena = torch.empty(max(self.arena_bytes, 1), dtype=torch.uint8, device=self.device)
                self.results = torch.zeros(self.n * BATCH_RESULT_BYTES, dtype=torch.uint8, device=self.device)

    def run(self, stream=None):
        if self.arena is None:
            raise SpgemmError(-6, "Batch.run: arena not allocated")
        st = _lib.spgemm_batch_run(self.n, self._ca, self.dtype, self._bound,
                                   ctypes.c_void_p(self.scratch.data_ptr()), ctypes.c_void_p(self.arena.data_ptr()),
                                   self.arena_bytes, ctypes.c_void_p(self.results.data_ptr()),
                                   _stream_handle(stream if stream is not None else self.stream))
        _check(st, "spgemm_batch_run")

    def replay(self, stream=None):
        """Run the batch by replaying a HIP graph of its launch sequence,
        captured on the first call: the sequence is fixed while the batch's
        structure is (operand values may change between replays), so a batch
        of the same shapes run again costs one graph launch instead of some
        thirty kernel launches.  The arena, results and scratch stay put."""
        if self.arena is None:
            raise SpgemmError(-6, "Batch.replay: arena not allocated")
        s = _on_stream(stream if stream is not None else self.stream)
        if self._graph is None:
            cap = torch.cuda.Stream(device=self.device)
            cap.wait_stream(s)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=cap):
                self.run(stream=cap)
            s.wait_stream(cap)
            self._graph = g
        with torch.cuda.stream(s):
            self._graph.replay()

    def outputs(self) -> List[Optional[DeviceCSR]]:
        """Per-product results as DeviceCSR views into the arena (None where the
        product is outside the batched range or failed; see ``status``)."""
        raw = self.results.cpu().numpy()
        ints = raw.view(np.int64).reshape(self.n, BATCH_RESULT_BYTES // 8)
        status = raw.view(np.int32).reshape(self.n, BATCH_RESULT_BYTES // 4)[:, 10]
        vt = torch.float64 if self.dtype == F64 else torch.int64
        out: List[Optional[DeviceCSR]] = []
        self.status = [int(x) for x in status]
        for p in range(self.n):
            if status[p] != 0:
                out.append(None)
                continue
            nnz, ro, co, vo = (int(ints[p, 1]), int(ints[p, 2]), int(ints[p, 3]), int(ints[p, 4]))
            m = self.As[p].nrows
            rp = self.arena[ro:ro + 8 * (m + 1)].view(torch.int64)
            cl = self.arena[co:co + 4 * nnz].view(torch.int32)
            vl = self.arena[vo:vo + 8 * nnz].view(vt)
            out.append(DeviceCSR(m, self.Bs[p].ncols, rp, cl, vl))
        return out


def spgemm(A: DeviceCSR, B: DeviceCSR, sorted_output: bool = True, validate: bool = False,
           stream=None) -> DeviceCSR:
    """C = A @ B on the GPU (two-phase hash SpGEMM).  C has int64 row pointers."""
    p = Plan([A], [B], sorted_output=sorted_output, validate=validate, stream=stream)
    p.symbolic()
    C = p.numeric()[0]
    st = p.stats(0)
    p.close()
    if st["status"] != 0:
        raise SpgemmError(st["status"], "spgemm (device check)")
    return C


def masked_sum_i64(C: DeviceCSR, M: DeviceCSR, stream=None) -> int:
    """Sum of C_ij over the positions stored in M (int64, wrap-around), on the device.
    The output is allocated on ``stream`` and read back after that stream is done."""
    s = _on_stream(stream)
    with torch.cuda.stream(s):
        out = torch.empty(1, dtype=torch.int64, device=C.cols.device)
    m = _Csr(M.nrows, M.ncols, M.nnz, M.rpts.data_ptr(), M.cols.data_ptr() if M.nnz else None, None)
    st = _lib.spgemm_masked_sum_i64(C.nrows, C.ncols, ctypes.c_void_p(C.rpts.data_ptr()),
                                    ctypes.c_void_p(C.cols.data_ptr() if C.nnz else None),
                                    ctypes.c_void_p(C.vals.data_ptr() if C.nnz else None),
                                    ctypes.byref(m), ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    _check(st, "spgemm_masked_sum_i64")
    s.synchronize()
    return int(out.item())


MASKED_WS_BYTES = 256


def masked_product_sum_i64(A: DeviceCSR, B: DeviceCSR, M: DeviceCSR, ones: bool = False, stream=None) -> int:
    """Sum of (A*B)_ij over the positions stored in M, without forming A*B
    (int64, wrap-around).  ones=True counts products (every value 1).  The
    workspace and output are allocated on ``stream`` and read back after that
    stream is done."""
    dev = A.rpts.device
    s = _on_stream(stream)
    with torch.cuda.stream(s):
        ws = torch.empty(MASKED_WS_BYTES, dtype=torch.uint8, device=dev)
        out = torch.empty(1, dtype=torch.int64, device=dev)
    ca, cb = A._c(), B._c()
    if ones:
        ca.vals = None
        cb.vals = None
    m = _Csr(M.nrows, M.ncols, M.nnz, M.rpts.data_ptr(), M.cols.data_ptr() if M.nnz else None, None)
    st = _lib.spgemm_masked_product_sum_i64(ctypes.byref(ca), ctypes.byref(cb), ctypes.byref(m),
                                            ctypes.c_void_p(ws.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(s.cuda_stream))
    _check(st, "spgemm_masked_product_sum_i64")
    s.synchronize()
    return int(out.item())


def triangle_count(A: DeviceCSR, L: DeviceCSR, U: DeviceCSR, stream=None, fused: bool = True) -> int:
    """Triangles of the undirected graph A: sum(C o A) / 2 with C = L*U.  fused
    (default): the masked product counts L*U's products that land on A's pattern
    without forming C; otherwise C is formed (int64, sorted rows) and summed
    over A's pattern."""
    if fused:
        s = masked_product_sum_i64(L, U, A, ones=True, stream=stream)
        if s % 2:
            raise SpgemmError(-10, "masked count of L*U over symmetric A is odd")
        return s // 2
    C = spgemm(L, U, sorted_output=True, stream=stream)
    s = masked_sum_i64(C, A, stream)
    if s % 2:
        raise SpgemmError(-10, "masked sum of L*U over symmetric A is odd")
    return s // 2


def stream_copy(dst: torch.Tensor, src: torch.Tensor, stream=None):
    n = min(dst.numel() * dst.element_size(), src.numel() * src.element_size()) // 16 * 16
    _check(_lib.spgemm_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), n,
                                   _stream_handle(stream)), "spgemm_stream_copy")


def stanza_read(base: torch.Tensor, start: torch.Tensor, log2_words: int, out: Optional[torch.Tensor] = None,
                stream=None) -> torch.Tensor:
    """Stanza probe: read the stanzas of 2**log2_words 8-byte words of the
    device tensor ``base`` that start at the word offsets ``start`` (int64,
    on the device).  Returns a 2-element int64 device tensor (``out`` if
    given): the wrap-around sum of the words read and the number of stanzas
    skipped because they did not fit.  Asynchronous on ``stream``."""
    if not base.is_contiguous() or not start.is_contiguous() or start.dtype != torch.int64:
        raise SpgemmError(-1, "stanza_read: contiguous base and int64 starts expected")
    if out is None:
        out = torch.empty(2, dtype=torch.int64, device=base.device)
    nbytes = base.numel() * base.element_size() // 8 * 8
    _check(_lib.spgemm_stanza_read(ctypes.c_void_p(base.data_ptr()), nbytes, ctypes.c_void_p(start.data_ptr()),
                                   start.numel(), int(log2_words), ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr() + 8), _stream_handle(stream)),
           "spgemm_stanza_read")
    return out
