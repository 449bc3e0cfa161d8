"""Continuous-batching server for independent products C = A*B on one GPU.

Requests (operands already in device memory) arrive over time.  Two workers
share the GPU, each on a stream of its own:

* the batch worker takes every request queued when it becomes free and
  analyses them together (row flop and key bounds of every row, Fig. 4).
  Products whose rows all fit the batched LDS tables and whose arena
  (sized from the rows' upper bounds) is small run as one batch; products with a row outside
  that range, more than ``batch_flop_max`` multiplications or an upper-bound
  arena above an eighth of the budget go to the plan worker;
* the plan worker runs those products one at a time through the two-phase
  path (Fig. 5).  Its symbolic phase gives the exact output size, and the
  output is admitted on that exact size (the two-phase scheme of Section 2
  allocates exactly what the product needs).

Admission: every device buffer a worker allocates for a request (scratch,
arena, workspace, row pointers, output) is first reserved against one byte
budget; a reservation that does not fit waits until others are released.
The batch worker never waits while holding a reservation (its arena is only
tried; on failure the batch is re-formed in groups reserved in one step);
plan workers reserve workspace, then the exact output, under a stage lock, so
at most one worker ever waits while holding memory.  A batch larger than the
budget is split into consecutive groups in arrival order.  A request that
cannot fit the budget even alone fails with a status instead of waiting
forever.

The GPU work itself is done by the library's kernels; this module only
schedules calls to it.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np
import torch

from .binding import (BATCH_XMAX, Batch, DeviceCSR, Plan, batch_arena_bytes, batch_scratch_bytes,
                      plan_scratch_bytes)


@dataclass
class Request:
    rid: int
    arrival_s: float          # offset from the start of the run
    A: DeviceCSR
    B: DeviceCSR
    sorted_out: bool


@dataclass
class Completion:
    rid: int
    arrival_s: float
    done_s: float
    path: str                 # "batch" or "plan"
    flop: int
    nnz: int
    status: int               # 0 ok, else a library status or -9 (does not fit the budget)

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


@dataclass
class ServeReport:
    completions: List[Completion]
    wall_s: float
    peak_reserved_bytes: int          # the admission gate's high-water mark
    peak_allocated_bytes: int         # torch's, over the run (operands included)
    batches: int
    batch_sizes: List[int] = field(default_factory=list)
    gate_waits: int = 0

    def summary(self) -> Dict[str, float]:
        lat = np.array([c.latency_s for c in self.completions])
        ok = [c for c in self.completions if c.status == 0]
        t0 = min(c.arrival_s for c in self.completions)
        t1 = max(c.done_s for c in self.completions)
        return {
            "requests": len(self.completions),
            "ok": len(ok),
            "products_per_s": len(self.completions) / max(t1 - t0, 1e-9),
            "gflops": 2.0 * sum(c.flop for c in ok) / max(t1 - t0, 1e-9) / 1e9,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "batched": sum(1 for c in self.completions if c.path == "batch"),
            "planned": sum(1 for c in self.completions if c.path == "plan"),
            "batches": self.batches,
            "gate_waits": self.gate_waits,
            "peak_reserved_gb": self.peak_reserved_bytes / 1e9,
            "peak_allocated_gb": self.peak_allocated_bytes / 1e9,
        }


class MemoryGate:
    """Byte budget shared by the workers (admission control)."""

    def __init__(self, budget: int):
        self.budget = int(budget)
        self.used = 0
        self.peak = 0
        self.waits = 0                     # acquisitions that had to wait
        self._cv = threading.Condition()

    def fits(self, n: int) -> bool:
        return n <= self.budget

    def acquire(self, n: int):
        if n > self.budget:
            raise MemoryError(f"request needs {n} bytes, budget is {self.budget}")
        with self._cv:
            if self.used + n > self.budget:
                self.waits += 1
            while self.used + n > self.budget:
                self._cv.wait(0.05)
            self.used += n
            self.peak = max(self.peak, self.used)

    def try_acquire(self, n: int) -> bool:
        with self._cv:
            if self.used + n > self.budget:
                return False
            self.used += n
            self.peak = max(self.peak, self.used)
            return True

    def release(self, n: int):
        with self._cv:
            self.used -= n
            self._cv.notify_all()


def split_to_budget(sizes: Sequence[int], budget: int, fixed: int = 0) -> List[List[int]]:
    """Consecutive groups of item indices whose sizes plus ``fixed`` fit the
    budget; an item that does not fit even alone forms a group of its own."""
    groups: List[List[int]] = []
    cur: List[int] = []
    tot = fixed
    for i, s in enumerate(sizes):
        if cur and tot + s > budget:
            groups.append(cur)
            cur, tot = [], fixed
        cur.append(i)
        tot += s
    if cur:
        groups.append(cur)
    return groups


class Server:
    """Serve a list of requests; ``run`` replays their arrival times (or takes
    them all at once with ``realtime=False``) and returns a ServeReport."""

    def __init__(self, mem_budget_bytes: int, on_result: Optional[Callable[[Request, DeviceCSR], None]] = None,
                 max_batch: int = 4096, batch_flop_max: int = 1 << 26, plan_workers: int = 2):
        self.gate = MemoryGate(mem_budget_bytes)
        self.plan_workers = max(1, plan_workers)
        self.on_result = on_result
        self.max_batch = max_batch
        self.batch_flop_max = batch_flop_max

    def _batchable(self, an: Batch, i: int, req: Request) -> bool:
        """Batch a product only if its rows fit the batched tables, it is not
        large and its upper-bound arena is small next to the budget (the plan
        path allocates exactly nnz(C) instead)."""
        return (an.supported[i] and an.flop[i] <= self.batch_flop_max
                and 24 * an.bound[i] + 8 * (req.A.nrows + 1) <= self.gate.budget // 8)

    # ------------------------------------------------------------------ workers
    def _done(self, req: Request, path: str, flop: int, nnz: int, status: int, C: Optional[DeviceCSR]):
        t = time.perf_counter() - self._t0
        if C is not None and self.on_result is not None:
            self.on_result(req, C)
        with self._lock:
            self._completions.append(Completion(req.rid, req.arrival_s, t, path, flop, nnz, status))

    def _batch_worker(self):
        stream = self._sb
        with torch.cuda.stream(stream):
            while True:
                with self._cv:
                    while not self._incoming and not self._closed:
                        self._cv.wait(0.05)
                    if not self._incoming and self._closed:
                        break
                    reqs = self._drain()
                try:
                    self._serve_batch(reqs, stream)
                except Exception as e:          # report, never hang the other worker
                    for r in reqs:
                        self._done(r, "batch", 0, 0, -10, None)
                    self._errors.append(repr(e))
        for _ in range(self.plan_workers):
            self._plan_q_put(None)

    def _drain(self) -> List[Request]:
        """Queued requests for one batch: at most max_batch, and as many as keep
        the batch's analysis scratch (about 64 bytes per row) within a quarter
        of the budget (at least one)."""
        reqs: List[Request] = []
        est = 0
        while self._incoming and len(reqs) < self.max_batch:
            e = 64 * (self._incoming[0].A.nrows + 1) + 512
            if reqs and est + e > self.gate.budget // 4:
                break
            reqs.append(self._incoming.popleft())
            est += e
        return reqs

    def _serve_batch(self, reqs: List[Request], stream):
        # The batch worker never waits while it holds a reservation: scratch is
        # reserved on its own, the arena only tried; if it does not fit, the
        # analysis is dropped and the batch goes in groups reserved whole.
        As = [r.A for r in reqs]
        Bs = [r.B for r in reqs]
        flags = [r.sorted_out for r in reqs]
        sb = batch_scratch_bytes(As)
        self.gate.acquire(sb)
        try:
            an = Batch(As, Bs, flags, stream=stream, allocate=False)
        except BaseException:
            self.gate.release(sb)
            raise
        ok = [self._batchable(an, i, reqs[i]) for i in range(len(reqs))]
        small = [i for i in range(len(reqs)) if ok[i]]
        big = [i for i in range(len(reqs)) if not ok[i]]
        for i in big:
            self._plan_q_put((reqs[i], an.flop[i]))
        if small and not big and self.gate.try_acquire(an.arena_bytes):
            try:
                self._run_group(an, reqs, stream)
            finally:
                self.gate.release(an.arena_bytes)
                self.gate.release(sb)
            return
        bounds = an.bound
        del an
        self.gate.release(sb)
        if not small:
            return
        est = [12 * bounds[i] + 8 * (reqs[i].A.nrows + 1) + 768 for i in small]
        fixed = batch_scratch_bytes([As[i] for i in small])
        for g in split_to_budget(est, self.gate.budget, fixed):
            sub = [reqs[small[j]] for j in g]
            gb = [bounds[small[j]] for j in g]
            gs = batch_scratch_bytes([r.A for r in sub])
            ga = batch_arena_bytes([r.A for r in sub], gb)
            if not self.gate.fits(gs + ga):
                for r in sub:
                    self._done(r, "batch", 0, 0, -9, None)
                continue
            self.gate.acquire(gs + ga)                 # one step: nothing held while waiting
            try:
                bt = Batch([r.A for r in sub], [r.B for r in sub], [r.sorted_out for r in sub], stream=stream,
                           allocate=False)
                self._run_group(bt, sub, stream)
                del bt
            finally:
                self.gate.release(gs + ga)

    def _run_group(self, bt: Batch, reqs: List[Request], stream):
        """Run an analysed batch whose arena is already admitted; complete its requests."""
        bt.allocate()
        bt.run(stream=stream)
        stream.synchronize()
        outs = bt.outputs()
        self._batches += 1
        self._batch_sizes.append(len(reqs))
        for j, r in enumerate(reqs):
            C = outs[j]
            self._done(r, "batch", bt.flop[j], 0 if C is None else C.nnz, bt.status[j], C)
        del outs
        bt.arena = None
        bt.results = None

    def _plan_q_put(self, item):
        with self._pcv:
            self._plan_q.append(item)
            self._pcv.notify_all()

    def _plan_worker(self, stream):
        with torch.cuda.stream(stream):
            while True:
                with self._pcv:
                    while not self._plan_q:
                        self._pcv.wait(0.05)
                    item = self._plan_q.popleft()
                if item is None:
                    break
                req, flop = item
                try:
                    self._serve_plan(req, flop, stream)
                except MemoryError:
                    self._done(req, "plan", flop, 0, -9, None)
                except Exception as e:
                    self._done(req, "plan", flop, 0, -10, None)
                    self._errors.append(repr(e))

    def _serve_plan(self, req: Request, flop: int, stream):
        ps = plan_scratch_bytes([req.A])
        held = 0
        try:
            # Plan workers take the stage lock from their first reservation to
            # their last, so at most one worker waits while holding a partial
            # reservation; the memory it waits for is held by fully admitted
            # work (the batch worker never waits while holding any), which
            # finishes without the lock.
            with self._stage:
                self.gate.acquire(ps)
                held = ps
                p = Plan([req.A], [req.B], sorted_output=req.sorted_out, stream=stream, defer_workspace=True)
                ws = p.workspace_bytes + 8 * (req.A.nrows + 1)
                if not self.gate.fits(held + ws):
                    raise MemoryError("product workspace does not fit the budget")
                self.gate.acquire(ws)
                held += ws
                nnz = p.symbolic()[0]            # the exact output size (synchronises the stream)
                ob = p.output_bytes()
                if not self.gate.fits(held + ob):
                    raise MemoryError("product output does not fit the budget")
                self.gate.acquire(ob)
                held += ob
            C = p.numeric()[0]
            stream.synchronize()
            st = p.stats(0)["status"]
            self._done(req, "plan", flop, nnz, st, C)
            p.close()
            del p, C
        finally:
            if held:
                self.gate.release(held)

    # ------------------------------------------------------------------ driver
    def run(self, requests: Sequence[Request], realtime: bool = True) -> ServeReport:
        self._incoming: deque = deque()
        self._plan_q: deque = deque()
        self._cv = threading.Condition()
        self._pcv = threading.Condition()
        self._lock = threading.Lock()
        self._stage = threading.Lock()     # a plan worker's reservation sequence
        self._closed = False
        self._completions: List[Completion] = []
        self._errors: List[str] = []
        self._batches = 0
        self._batch_sizes: List[int] = []
        self._sb = torch.cuda.Stream()
        plan_streams = [torch.cuda.Stream() for _ in range(self.plan_workers)]
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        order = sorted(requests, key=lambda r: r.arrival_s)
        tb = threading.Thread(target=self._batch_worker, name="spgemm-batch", daemon=True)
        tps = [threading.Thread(target=self._plan_worker, args=(st,), name=f"spgemm-plan{i}", daemon=True)
               for i, st in enumerate(plan_streams)]
        self._t0 = time.perf_counter()
        tb.start()
        for t in tps:
            t.start()
        for r in order:
            if realtime:
                wait = r.arrival_s - (time.perf_counter() - self._t0)
                if wait > 0:
                    time.sleep(wait)
            else:
                r = Request(r.rid, 0.0, r.A, r.B, r.sorted_out)
            with self._cv:
                self._incoming.append(r)
                self._cv.notify_all()
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        tb.join()
        for t in tps:
            t.join()
        wall = time.perf_counter() - self._t0
        torch.cuda.synchronize()
        if self._errors:
            raise RuntimeError("serving worker failed: " + "; ".join(self._errors[:3]))
        return ServeReport(sorted(self._completions, key=lambda c: c.rid), wall, self.gate.peak,
                           torch.cuda.max_memory_allocated(), self._batches, self._batch_sizes, self.gate.waits)


def serial_products(requests: Sequence[Request], stream=None) -> float:
    """One launch sequence per product, one product at a time (plan, symbolic,
    allocate, numeric, synchronise, free): the per-call baseline.  Returns the
    wall time in seconds."""
    torch.cuda.synchronize()
    t = time.perf_counter()
    for r in requests:
        p = Plan([r.A], [r.B], sorted_output=r.sorted_out, stream=stream)
        p.symbolic()
        p.numeric()
        torch.cuda.synchronize()
        p.close()
        del p
    return time.perf_counter() - t
