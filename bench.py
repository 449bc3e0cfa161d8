#!/usr/bin/env python3
"""Benchmark of the gfx950 hash SpGEMM on one MI355X.

A step is one whole product C = A*B through the library's C ABI: plan (row
flop + bins), symbolic (row counts, int64 row pointers, nnz(C) read back),
allocation of C, numeric (accumulate, compact, sort if asked).  Inputs are
resident in HBM before the timed region.  Prints ONE JSON line.

Default workload: A*A for R-MAT scale 20, edge factor 16, (a,b,c,d) =
(0.57,0.19,0.19,0.05), FP64 U[0,1) values, rows shuffled, unsorted output.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SpGEMM GFLOP/s (2×mults) and HBM-roofline fraction; served products/s + p99"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "rmat20": dict(desc="C=A*A, A R-MAT scale 20 ef 16 (0.57,0.19,0.19,0.05), FP64 U[0,1), rows shuffled, "
                        "unsorted output", sorted=False),
    "er20": dict(desc="C=A*A, A ER n=2^20, 16 distinct uniform cols/row, FP64 U[0,1), rows shuffled, "
                      "unsorted output", sorted=False),
    "rmat16": dict(desc="C=A*A, A R-MAT scale 16 ef 16 (0.57,0.19,0.19,0.05), FP64 U[0,1)", sorted=True),
    "er4096": dict(desc="C=A*A, A ER n=4096, 8 distinct uniform cols/row, FP64 U[0,1), sorted output",
                   sorted=True),
    "tri18": dict(desc="triangle count: symmetric R-MAT scale 18 ef 16 no self loops, C=L*U int64 sorted, "
                       "count=sum(C o A)/2", sorted=True),
    "bfs18": dict(desc="C=A*F, A R-MAT scale 18 ef 16 int64 ones, F n x 512 one nonzero per column, "
                       "unsorted output", sorted=False),
    "serve": dict(desc="served stream: Poisson arrivals, n log-uniform [256, 131072], nnz/row U{2..32}, "
                       "ER/R-MAT 50/50, sorted/unsorted 50/50, A and B independent, FP64", sorted=None),
    "tri18f": dict(desc="triangle count: symmetric R-MAT scale 18 ef 16 no self loops, natural order, "
                        "masked product of L*U over A's pattern without forming C, count=sum/2", sorted=None),
    "batch": dict(desc="small stratum of the served stream (n*d^2 <= 2^20): the products of one batch through "
                       "the batched path vs one launch sequence per product", sorted=None),
    "sweep_density": dict(desc="C=A*A at scale 16, ER (fixed degree) and G500 R-MAT, edge factor 2..64, sorted "
                               "and unsorted output (the density sweep of Section 5.4)", sorted=None),
    "sweep_size": dict(desc="C=A*A, ER scale 7..20 and G500 R-MAT scale 7..17, edge factor 16, sorted and "
                            "unsorted output (the size sweep of Section 5.4)", sorted=None),
    "tallskinny": dict(desc="C=A*B, A G500 R-MAT scale 18..20 ef 16, B = 2^10..2^16 columns of A drawn at "
                            "random, sorted and unsorted output (Section 5.5)", sorted=None),
    "stanza": dict(desc="stanza read probe: stanzas of 2^k consecutive 8-byte words (k = 0..13) from random "
                        "places of a 4 GiB array (HBM) and of a 64 MiB array (fits the 256 MB Infinity Cache)",
                   sorted=None),
}
SWEEPS = ("sweep_density", "sweep_size", "tallskinny")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def input_rows_sorted(srt: bool, input_order: str) -> bool:
    """Whether the input rows come sorted by column: with the output's order
    (the paper's unsorted runs shuffle the input rows, Section 5.1) unless
    --input-order fixes it."""
    return srt if input_order == "auto" else input_order == "sorted"


def make_inputs(name: str, seed: int, sorted_flag, input_order: str = "auto", degree_order: bool = False):
    from synth import (bfs_frontier, erdos_renyi_fixed_degree, rmat, shuffle_within_rows,
                       symmetric_rmat_graph, triangle_inputs, with_values)
    w = WORKLOADS[name]
    srt = w["sorted"] if sorted_flag is None else sorted_flag
    rows_sorted = input_rows_sorted(srt, input_order)
    if name == "rmat20":
        A = rmat(20, 16, seed, sorted_rows=rows_sorted)
        return dict(A=A, B=A, sorted=srt, rows_sorted=rows_sorted)
    if name == "er20":
        A = erdos_renyi_fixed_degree(1 << 20, 16, seed, sorted_rows=rows_sorted)
        return dict(A=A, B=A, sorted=srt, rows_sorted=rows_sorted)
    if name == "rmat16":
        A = rmat(16, 16, seed, sorted_rows=rows_sorted)
        return dict(A=A, B=A, sorted=srt, rows_sorted=rows_sorted)
    if name == "er4096":
        A = erdos_renyi_fixed_degree(4096, 8, seed, sorted_rows=True)
        return dict(A=A, B=A, sorted=srt)
    if name in ("tri18", "tri18f"):
        g = symmetric_rmat_graph(18, 16, seed)
        A, L, U = triangle_inputs(g, degree_order=degree_order)
        return dict(A=L, B=U, M=A, sorted=True)
    if name == "bfs18":
        A = with_values(rmat(18, 16, seed, values=""), 0, "ones")
        F = bfs_frontier(A.ncols, 512, seed + 5)
        return dict(A=A, B=F, sorted=srt)
    raise KeyError(name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat20", choices=sorted(WORKLOADS))
    ap.add_argument("--sorted", dest="sorted_flag", action="store_true", default=None)
    ap.add_argument("--unsorted", dest="sorted_flag", action="store_false")
    ap.add_argument("--input-order", default="auto", choices=("auto", "sorted", "shuffled"),
                    help="column order inside the input rows (rmat20, er20, rmat16); auto: sorted "
                         "for sorted output, shuffled for unsorted output")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--heap", action="store_true",
                    help="plan with the Heap accumulator for the rows in its envelope (sorted output only)")
    ap.add_argument("--bucket-slots", type=int, default=4, choices=(4, 8, 16),
                    help="slots per bucket of the LDS hash tables (8 and 16: the HashVector-style chunks)")
    ap.add_argument("--degree-order", action="store_true",
                    help="tri18: relabel the graph by ascending degree (Section 5.6) before splitting L and U")
    ap.add_argument("--no-small-stratum", action="store_true",
                    help="skip the small-stratum comparison in the headline line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target oracle time of the CPU baseline's row sample")
    ap.add_argument("--requests", type=int, default=4000, help="serve: requests in the stream")
    ap.add_argument("--small-requests", type=int, default=256, help="serve: requests of the small stratum")
    ap.add_argument("--budget-gb", type=float, default=128.0, help="serve: admission budget")
    ap.add_argument("--no-timing", action="store_true", help="skip per-kernel HIP events")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the row-parallel "
              "multi-GPU split is a design note, not part of this build.", file=sys.stderr)
        sys.exit(2)

    host_serve = None
    headline_small = args.workload == "rmat20" and not args.no_small_stratum
    if args.workload in ("serve", "batch") or headline_small:
        # operands are generated on a host process pool before anything touches the GPU
        host_serve = _generate_serve(args, small_only=args.workload != "serve")

    import torch
    import paper_1804_01698_amd as sp

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "serve":
        return bench_serve(args, sp, dev, *host_serve)
    if args.workload == "batch":
        return bench_batch(args, sp, dev, host_serve[1])
    if args.workload in SWEEPS:
        return bench_sweep(args, sp, dev)
    if args.workload == "stanza":
        return bench_stanza(args, sp, dev)

    t_gen = time.perf_counter()
    inp = make_inputs(args.workload, args.seed, args.sorted_flag, args.input_order, args.degree_order)
    if args.workload == "tri18f":
        return bench_tri_fused(args, sp, dev, inp)
    log(f"inputs {args.workload}: generated in {time.perf_counter() - t_gen:.1f}s; "
        f"A {inp['A'].shape} nnz {inp['A'].nnz}, B {inp['B'].shape} nnz {inp['B'].nnz}")
    dA = sp.DeviceCSR.from_host(inp["A"], device=dev)
    dB = dA if inp["B"] is inp["A"] else sp.DeviceCSR.from_host(inp["B"], device=dev)
    dM = sp.DeviceCSR.from_host(inp["M"], device=dev) if "M" in inp else None
    srt = inp["sorted"]
    torch.cuda.synchronize()

    # HBM copy probe (1 GiB each way), measured copy rate for context
    nbytes = 1 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    src.zero_()
    sp.stream_copy(dst, src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        sp.stream_copy(dst, src)
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * nbytes / (time.perf_counter() - t0) / 1e9
    del src, dst

    cfg = None
    if args.heap or args.bucket_slots != 4:
        cfg = dict(sp.default_config(), heap=1 if args.heap else 0, bucket_slots=args.bucket_slots)

    def step(timing: bool):
        p = sp.Plan([dA], [dB], sorted_output=srt, timing=timing, config=cfg)
        p.symbolic()
        C = p.numeric()[0]
        p.C = []                      # the plan keeps no reference to C
        extra = None
        if dM is not None:
            extra = sp.masked_sum_i64(C, dM)
        return p, C, extra

    for i in range(args.warmup):
        p, C, extra = step(False)
        torch.cuda.synchronize()
        st = p.stats(0)
        if st["status"] != 0:
            raise SystemExit(f"device check failed: {st}")
        log(f"warmup {i}: nnz(C) = {st['nnz_C']}, flop = {st['flop']}, windows = {st['windows']}")
        del C
        p.close()
        del p

    # the timed steps: plan through numeric, no per-kernel events.  Every step
    # drops its plan (and with it the workspace) and C before the next one
    # starts, so each step's buffers come from the allocator's cache of the
    # previous step's; the last plan is kept for its counters.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ms = []
    for i in range(args.steps):
        ts = time.perf_counter()
        p, C, extra = step(False)
        del C
        if i + 1 < args.steps:
            p.close()
            del p
        step_ms.append((time.perf_counter() - ts) * 1e3)     # host time to enqueue/return
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / max(args.steps, 1)
    log("step host ms: " + ", ".join(f"{x:.1f}" for x in step_ms))

    st = p.stats(0)
    p.close()
    del p
    if st["status"] != 0:
        raise SystemExit(f"device check failed: {st}")
    flop = st["flop"]
    nnz_c = st["nnz_C"]
    gflops = 2.0 * flop / (ms * 1e-3) / 1e9

    # per-kernel times: the same steps again with HIP events around every
    # launch on the library's stream (the events are read after each step)
    agg = {}
    if not args.no_timing:
        for i in range(args.steps):
            p, C, extra = step(True)
            del C
            for k in p.kernel_times():
                a = agg.setdefault(k["name"], dict(ms=0.0, launches=0, alg_bytes=0.0))
                a["ms"] += k["ms"]
                a["launches"] += k["launches"]
                a["alg_bytes"] += k["alg_bytes"]
            p.close()
            del p
    kernels = sorted(([n, v["ms"] / args.steps, v["launches"] // max(args.steps, 1),
                       v["alg_bytes"] / max(v["launches"], 1)] for n, v in agg.items()),
                     key=lambda r: -r[1])
    roofline = None
    if kernels:
        name, kms, nl, bytes_per_launch = kernels[0]
        avg_launch_ms = kms / max(nl, 1)
        achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
        traffic = counted_traffic(name, args.workload)
        roofline = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "avg_launch_ms": round(avg_launch_ms, 4), "alg_bytes_per_launch": bytes_per_launch}
    nnz_a, nnz_b, m = inp["A"].nnz, inp["B"].nnz, inp["A"].nrows
    path_bytes = path_alg_bytes(flop, nnz_c, nnz_a, m)
    out = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i64" if inp["A"].vals.dtype == np.int64 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]['desc']}",
                   "sorted_output": srt, "input_rows": ("sorted" if inp.get("rows_sorted") else "shuffled")
                   if "rows_sorted" in inp else None, "nrows": m, "nnz_A": nnz_a, "nnz_B": nnz_b, "flop": flop,
                   "nnz_C": nnz_c, "seed": args.seed},
        "roofline": roofline,
        "path_roofline": {"alg_bytes": path_bytes, "achieved": round(path_bytes / (ms * 1e-3) / 1e9, 1),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(path_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "copy_probe_GBs": round(copy_gbs, 1),
        "kernels_ms_per_step": {k[0]: round(k[1], 4) for k in kernels},
        "kernels": [{"kernel": k[0], "ms_per_step": round(k[1], 4), "launches": k[2],
                     "alg_bytes_per_launch": k[3],
                     "frac": round(k[3] / (k[1] / max(k[2], 1) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if k[1] > 0 else None}
                    for k in kernels],
    }
    if dM is not None:
        out["triangles"] = int(extra) // 2
    if args.heap:
        out["config"]["accumulator"] = "heap for rows in its envelope (heap_rows = %d)" % st["heap_rows"]
    if args.bucket_slots != 4:
        out["config"]["bucket_slots"] = args.bucket_slots
    if args.degree_order:
        out["config"]["vertex_order"] = "ascending degree"

    if host_serve is not None:
        # the served half of the metric: the small stratum through one launch
        # sequence per product, one batch and the server (inputs of the
        # headline product freed first)
        del dA, dB, dM
        torch.cuda.empty_cache()
        t_small = time.perf_counter()
        out["small_stratum"] = measure_small(args, sp, dev, host_serve[1])
        log(f"small stratum measured in {time.perf_counter() - t_small:.1f}s: {out['small_stratum']}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inp, args.cpu_seconds, srt, args.seed)
    print(json.dumps(out), flush=True)


def path_alg_bytes(flop, nnz_c, nnz_a, m):
    """Algorithmic bytes of one whole product (int32 indices, 8-byte values):
    16 per multiplication (4 for the symbolic key, 12 for the numeric key and
    value), 12 per output entry, 36 per entry of A (its column twice, its value,
    the B row-pointer pair twice) and 40 per row (pointers, flop, counts, scan)."""
    return 16.0 * flop + 12.0 * nnz_c + 36.0 * nnz_a + 40.0 * m


KERNEL_SOURCES = ("paper_1804_01698_amd/csrc/kernels.hip", "paper_1804_01698_amd/csrc/device.hpp",
                  "paper_1804_01698_amd/csrc/config.hpp")


def counted_traffic(kernel: str, workload: str):
    """HBM bytes per launch of ``kernel`` on ``workload`` from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when there is none or the
    kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", " ")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if fields.get("kernel") != kernel or fields.get("source_sha256") != h.hexdigest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(inp, seconds, srt, seed):
    """The oracle, as it is, on a seeded random sample of rows of the same
    product, streamed in row blocks of at most 1e9 multiplications whose results
    are dropped (the whole product's C does not fit host memory).  A first
    block measures the rate; the sample is then sized to about ``seconds``."""
    import oracle
    A, B = inp["A"], inp["B"]
    # step 1 of the oracle (operand validation) once; the row blocks skip it
    oracle.validate(A)
    if B is not A:
        oracle.validate(B)
    f = oracle.row_flop(A, B, validate_inputs=False).astype(np.int64)
    order = np.random.default_rng(seed + 99).permutation(A.nrows)
    csum = np.cumsum(f[order])
    threads = oracle.max_threads()

    def run(lo_flop, hi_flop):
        lo = int(np.searchsorted(csum, lo_flop, side="right"))
        hi = min(int(np.searchsorted(csum, hi_flop, side="right")) + 1, A.nrows)
        rows_all = order[lo:hi]
        t = 0.0
        done = 0
        i = 0
        while i < rows_all.size:
            j = i
            acc = 0
            while j < rows_all.size and (acc == 0 or acc + f[rows_all[j]] <= 1e9):
                acc += f[rows_all[j]]
                j += 1
            rows = np.sort(rows_all[i:j])
            t0 = time.perf_counter()
            C = oracle.spgemm(A, B, sorted_output=srt, rows=rows, validate_inputs=False)
            t += time.perf_counter() - t0
            del C
            done += acc
            i = j
        return hi - lo, done, t

    n1, fl1, t1 = run(0, 5e8)
    rate = fl1 / max(t1, 1e-9)
    target = min(float(csum[-1]), fl1 + rate * max(seconds - t1, 0.0))
    n2, fl2, t2 = run(fl1, target) if target > fl1 else (0, 0, 0.0)
    nrows, flop, dt = n1 + n2, fl1 + fl2, t1 + t2
    passes = 1
    if nrows >= A.nrows:
        # the whole product took less than the target: repeat it while one
        # more pass still fits the target
        total = int(csum[-1])
        per = dt
        while dt + per <= seconds:
            t0 = time.perf_counter()
            C = oracle.spgemm(A, B, sorted_output=srt, validate_inputs=False)
            dt += time.perf_counter() - t0
            del C
            flop += total
            passes += 1
    what = (f"the whole product x {passes}" if nrows >= A.nrows else
            f"{nrows} random rows of the same product ({flop / max(int(csum[-1]), 1):.3%} of the flop)")
    return {"value": round(float(2.0 * flop / dt / 1e9), 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{what}, {flop} multiplications in row blocks of <= 1e9, {dt:.1f} s"}


def _gen_request(r):
    from synth import serving_request_operands
    a, b = serving_request_operands(r)
    return r, a, b


SMALL_FLOP = 2 ** 20       # the small stratum: products of at most this many multiplications


def _generate_serve(args, small_only: bool = False):
    """Requests of the served stream and candidates for its small stratum, with
    their operands generated on a host process pool (16 workers at most).  The
    candidates are the stream generator's requests with n*d^2 <= 2^20 (a cheap
    pre-filter; R-MAT products often exceed it), four per stratum slot: the
    stratum itself is picked on the device by real flop (small_stratum)."""
    import multiprocessing as mp
    from synth import serving_stream
    t = time.perf_counter()
    reqs = [] if small_only else serving_stream(args.requests, args.seed)
    small = serving_stream(4 * args.small_requests, args.seed + 1000, max_flop=SMALL_FLOP)
    workers = max(1, min(16, os.cpu_count() or 1))
    # close() + join() rather than the with-block's terminate(): the workers
    # exit on their own instead of being sent SIGTERM
    pool = mp.get_context("spawn").Pool(workers)
    try:
        main_ops = pool.map(_gen_request, reqs, chunksize=4)
        small_ops = pool.map(_gen_request, small, chunksize=4)
    finally:
        pool.close()
        pool.join()
    log(f"serve: {len(reqs)} + {len(small)} requests generated in {time.perf_counter() - t:.1f}s "
        f"on {workers} processes")
    return main_ops, small_ops


def _upload(sp, ops, dev):
    from paper_1804_01698_amd.serve import Request
    return [Request(r.rid, r.arrival_s, sp.DeviceCSR.from_host(a, device=dev), sp.DeviceCSR.from_host(b, device=dev),
                    r.sorted_out) for r, a, b in ops]


def _sweep_points(name, seed):
    """(label, A, B, sorted, params) of a sweep workload, built lazily."""
    from synth import column_sample, erdos_renyi_fixed_degree, rmat
    if name == "sweep_density":
        for fam in ("er", "g500"):
            for ef in (2, 4, 8, 16, 32, 64):
                for srt in (False, True):
                    A = (erdos_renyi_fixed_degree(1 << 16, ef, seed, sorted_rows=srt) if fam == "er"
                         else rmat(16, ef, seed, sorted_rows=srt))
                    yield f"{fam} s16 ef{ef} {'sorted' if srt else 'unsorted'}", A, A, srt, dict(
                        family=fam, scale=16, ef=ef, sorted=srt)
    elif name == "sweep_size":
        for fam, scales in (("er", range(7, 21)), ("g500", range(7, 18))):
            for sc in scales:
                for srt in (False, True):
                    A = (erdos_renyi_fixed_degree(1 << sc, 16, seed, sorted_rows=srt) if fam == "er"
                         else rmat(sc, 16, seed, sorted_rows=srt))
                    yield f"{fam} s{sc} ef16 {'sorted' if srt else 'unsorted'}", A, A, srt, dict(
                        family=fam, scale=sc, ef=16, sorted=srt)
    elif name == "tallskinny":
        from synth import shuffle_within_rows
        for sc in (18, 19, 20):
            A_sorted = rmat(sc, 16, seed)
            for srt in (False, True):
                # rmat(..., sorted_rows=False) is this shuffle of the same matrix
                A = A_sorted if srt else shuffle_within_rows(A_sorted, seed + 2)
                for lk in (10, 12, 14, 16):
                    B = column_sample(A, 1 << lk, seed + 3)
                    yield f"g500 s{sc} x 2^{lk} {'sorted' if srt else 'unsorted'}", A, B, srt, dict(
                        family="g500", scale=sc, ef=16, k=1 << lk, sorted=srt)
    else:
        raise KeyError(name)


def bench_sweep(args, sp, dev):
    """Every point: plan + symbolic + allocation + numeric + free, timed over
    --steps runs after --warmup; GFLOP/s = 2*flop/t; roofline fraction from the
    algorithmic bytes 16*flop + 12*nnz(C) + 36*nnz(A) + 40*m over 8 TB/s."""
    import torch
    rows = []
    for label, A, B, srt, params in _sweep_points(args.workload, args.seed):
        dA = sp.DeviceCSR.from_host(A, device=dev)
        dB = dA if B is A else sp.DeviceCSR.from_host(B, device=dev)

        def run():
            p = sp.Plan([dA], [dB], sorted_output=srt)
            p.symbolic()
            C = p.numeric()[0]
            st = p.stats(0)
            p.close()
            return C, st

        for _ in range(max(args.warmup, 1)):
            C, st = run()
            del C
        torch.cuda.synchronize()
        if st["status"] != 0:
            raise SystemExit(f"device check failed at {label}: {st}")
        t0 = time.perf_counter()
        for _ in range(args.steps):
            C, st = run()
            del C
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
        flop, nnzc = int(st["flop"]), int(st["nnz_C"])
        alg = path_alg_bytes(flop, nnzc, A.nnz, A.nrows)
        rows.append(dict(point=label, **params, nnz_A=int(A.nnz), nnz_B=int(B.nnz), flop=flop, nnz_C=nnzc,
                         ms=round(ms, 4), gflops=round(2.0 * flop / (ms * 1e-3) / 1e9, 2),
                         roofline_frac=round(alg / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)))
        log(f"{label}: {ms:.3f} ms, {rows[-1]['gflops']} GFLOP/s, frac {rows[-1]['roofline_frac']}")
        del dA, dB
        torch.cuda.empty_cache()
    g = [r["gflops"] for r in rows if r["gflops"] > 0]
    geo = float(np.exp(np.mean(np.log(g)))) if g else 0.0
    out = {
        "metric": METRIC, "value": round(geo, 2), "unit": "GFLOP/s (geometric mean over the points)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(sum(r["ms"] for r in rows), 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]['desc']}", "points": len(rows),
                   "seed": args.seed},
        "points": rows,
    }
    print(json.dumps(out), flush=True)


def bench_stanza(args, sp, dev):
    """Stanza bandwidth against stanza length (Section 5's stanza benchmark):
    bytes of the stanzas read over the kernel time (HIP events), and the same
    with the 8-byte start of every stanza counted."""
    import torch
    rng = np.random.default_rng(args.seed)
    rows = []
    for arr_name, nbytes in (("hbm_4GiB", 4 << 30), ("mall_64MiB", 64 << 20)):
        nwords = nbytes // 8
        base = torch.ones(nwords, dtype=torch.int64, device=dev)
        out = torch.empty(2, dtype=torch.int64, device=dev)
        for lw in range(0, 14):
            L = 1 << lw
            nst = max(1 << 12, (1 << 27) >> lw)        # 1 GiB of stanza words per launch
            starts = torch.from_numpy(rng.integers(0, nwords - L + 1, size=nst, dtype=np.int64)).to(dev)
            for _ in range(max(args.warmup, 1)):
                sp.stanza_read(base, starts, lw, out)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                sp.stanza_read(base, starts, lw, out)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / max(args.steps, 1)
            got = out.cpu().tolist()
            if got[0] != nst * L or got[1] != 0:
                raise SystemExit(f"stanza probe read {got} at lw={lw}, expected {[nst * L, 0]}")
            data = 8.0 * nst * L
            rows.append(dict(array=arr_name, stanza_bytes=8 * L, stanzas=nst, ms=round(ms, 4),
                             gbs=round(data / (ms * 1e-3) / 1e9, 1),
                             gbs_with_starts=round((data + 8.0 * nst) / (ms * 1e-3) / 1e9, 1)))
            log(f"{arr_name} stanza {8 * L} B: {rows[-1]['gbs']} GB/s")
            del starts
        del base
        torch.cuda.empty_cache()
    ref = next(r for r in rows if r["array"] == "hbm_4GiB" and r["stanza_bytes"] == 64)
    out = {
        "metric": "stanza read GB/s against stanza length", "value": ref["gbs"], "unit": "GB/s (64-byte stanzas, 4 GiB array)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ref["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"stanza: {WORKLOADS['stanza']['desc']}", "seed": args.seed},
        "points": rows,
    }
    print(json.dumps(out), flush=True)


def bench_tri_fused(args, sp, dev, inp):
    """Triangle count by the masked product (products of L*U that land on A's
    pattern are counted as formed; C is never stored)."""
    import torch
    L, U, A = inp["A"], inp["B"], inp["M"]
    dL, dU, dA = (sp.DeviceCSR.from_host(x, device=dev) for x in (L, U, A))
    degU = np.diff(U.rpts)
    flop = int(degU[L.cols].sum())
    for _ in range(args.warmup):
        s = sp.masked_product_sum_i64(dL, dU, dA, ones=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        s = sp.masked_product_sum_i64(dL, dU, dA, ones=True)
    e1.record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
    kms = e0.elapsed_time(e1) / max(args.steps, 1)
    alg = 4.0 * flop + 12.0 * L.nnz + 8.0 * A.nnz + 16.0 * L.nrows
    achieved = alg / (kms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(2.0 * flop / (ms * 1e-3) / 1e9, 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"tri18f: {WORKLOADS['tri18f']['desc']}", "nrows": L.nrows, "nnz_L": L.nnz,
                   "nnz_A": A.nnz, "flop": flop, "seed": args.seed},
        "triangles": s // 2,
        "roofline": {"bound": "hbm", "kernel": "masked_product", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "avg_launch_ms": round(kms, 4), "alg_bytes_per_launch": alg},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inp, args.cpu_seconds, True, args.seed)
    print(json.dumps(out), flush=True)


def select_small(sp, dev, small_ops, count):
    """The small stratum: the first ``count`` candidate requests (stream order)
    whose product has at most SMALL_FLOP multiplications, counted on the
    device by the batched path's analysis (the row flop of Fig. 4)."""
    import torch
    cand = _upload(sp, small_ops, dev)
    an = sp.Batch([r.A for r in cand], [r.B for r in cand], [r.sorted_out for r in cand], allocate=False)
    flops = list(an.flop)
    del an
    torch.cuda.synchronize()
    sel = [r for r, f in zip(cand, flops) if f <= SMALL_FLOP][:count]
    fsel = [f for f in flops if f <= SMALL_FLOP][:count]
    return sel, fsel, len(cand)


def measure_small(args, sp, dev, small_ops):
    """The small stratum through (a) one launch sequence per product (plan,
    symbolic with its sync, allocation, numeric, sync, free: serial), (b) one
    batch as a caller runs it (upload of the batch description, analysis with
    its sync, arena, run, sync, result views) and (c) the server with every
    request queued at t = 0 (its batch worker does (b) plus admission and
    completion records).  Results of (b) are checked against (a) product by
    product.  Best of three rounds each."""
    import torch
    from paper_1804_01698_amd.serve import Server, serial_products
    budget = int(args.budget_gb * 1e9)
    reqs, flops, ncand = select_small(sp, dev, small_ops, args.small_requests)
    if not reqs:
        return None
    Server(budget).run(reqs[:16], realtime=False)
    serial_products(reqs[:16])

    def batched_direct():
        torch.cuda.synchronize()
        t = time.perf_counter()
        bt = sp.Batch([r.A for r in reqs], [r.B for r in reqs], [r.sorted_out for r in reqs])
        bt.run()
        outs = bt.outputs()
        torch.cuda.synchronize()
        return time.perf_counter() - t, bt, outs

    batched_direct()
    best = {}
    rb = None
    for _ in range(3):
        tb, bt, outs = batched_direct()
        r = Server(budget).run(reqs, realtime=False)
        tsv = max(c.done_s for c in r.completions)
        ts = serial_products(reqs)
        for k, v in (("batched", tb), ("server", tsv), ("serial", ts)):
            best[k] = min(best.get(k, v), v)
        if rb is None or tsv <= best["server"]:
            rb = r
    # results of the batch against the per-product path
    mism = 0
    for q, C in zip(reqs, outs):
        p = sp.Plan([q.A], [q.B], sorted_output=q.sorted_out)
        p.symbolic()
        R = p.numeric()[0]
        torch.cuda.synchronize()
        p.close()
        if C is None or C.nnz != R.nnz or not torch.equal(C.rpts, R.rpts):
            mism += 1
    sm = rb.summary()
    n = len(reqs)
    return {"products": n, "candidates": ncand, "flop_max": SMALL_FLOP, "flop_total": int(sum(flops)),
            "serial_products_per_s": round(n / best["serial"], 1),
            "batched_products_per_s": round(n / best["batched"], 1),
            "server_products_per_s": round(n / best["server"], 1),
            "speedup_batched": round(best["serial"] / best["batched"], 2),
            "speedup_server": round(best["serial"] / best["server"], 2),
            "server_p50_ms": round(sm["p50_ms"], 3), "server_p99_ms": round(sm["p99_ms"], 3),
            "server_batched": sm["batched"], "server_planned": sm["planned"],
            "row_count_mismatches": mism,
            "selection": f"first {n} of {ncand} seeded stream requests with n*d^2 <= 2^20 whose product has "
                         f"<= 2^20 multiplications (counted by the batch analysis on the device)"}


def bench_batch(args, sp, dev, small_ops):
    """The small stratum as one batch: analyse once, then K timed runs of the
    batch (kernels only, products outside the batched range go through the
    plan path on a second stream), against one launch sequence per product."""
    import torch
    from paper_1804_01698_amd.serve import serial_products
    reqs, _, ncand = select_small(sp, dev, small_ops, args.small_requests)
    As, Bs, fl = [r.A for r in reqs], [r.B for r in reqs], [r.sorted_out for r in reqs]
    bt = sp.Batch(As, Bs, fl)                      # first construction warms the allocator
    del bt
    torch.cuda.synchronize()
    t = time.perf_counter()
    bt = sp.Batch(As, Bs, fl)
    torch.cuda.synchronize()
    t_analyse = time.perf_counter() - t
    rest = [r for r, ok in zip(reqs, bt.supported) if not ok]
    side = torch.cuda.Stream()

    def step():
        # the batch runs on the current stream while the products outside its
        # range go through the plan path on a second stream
        bt.run()
        with torch.cuda.stream(side):
            for r in rest:
                p = sp.Plan([r.A], [r.B], sorted_output=r.sorted_out, stream=side)
                p.symbolic()
                p.numeric()
                side.synchronize()
                p.close()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(args.steps, 1)
    # the same batch again through its captured launch graph (shapes repeat)
    dt_replay = None
    if not rest:
        bt.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            bt.replay()
        torch.cuda.synchronize()
        dt_replay = (time.perf_counter() - t0) / max(args.steps, 1)
    serial_products(reqs[:8])
    ts = min(serial_products(reqs) for _ in range(2))
    flop = sum(bt.flop)
    out = {
        "metric": METRIC, "value": round(len(reqs) / dt, 1), "unit": "products/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch: {WORKLOADS['batch']['desc']}", "products": len(reqs),
                   "outside_batched_range": len(rest), "flop": flop, "seed": args.seed},
        "batched_gflops": round(2.0 * flop / dt / 1e9, 2),
        "analyse_ms": round(t_analyse * 1e3, 3),
        "serial_ms": round(ts * 1e3, 3),
        "speedup_vs_serial": round(ts / dt, 2),
        "speedup_incl_analyse": round(ts / (dt + t_analyse), 2),
        "graph_replay_ms": None if dt_replay is None else round(dt_replay * 1e3, 3),
        "speedup_graph_replay": None if dt_replay is None else round(ts / dt_replay, 2),
    }
    print(json.dumps(out), flush=True)


def bench_serve(args, sp, dev, main_ops, small_ops):
    """Served stream (request-level parallelism on one GPU).

    (i) saturation capacity mu: every request queued at t = 0; then the same
    stream replayed in real time at lambda = 0.5 mu and 0.9 mu (Poisson
    arrivals rescaled).  (ii) small stratum (requests with n*d^2 <= 2^20):
    the server's batched path against one launch sequence per product."""
    import torch
    from paper_1804_01698_amd.serve import Request, Server, serial_products
    budget = int(args.budget_gb * 1e9)
    t_gen = time.perf_counter()
    reqs = [r for r, _, _ in main_ops]
    dreqs = _upload(sp, main_ops, dev)
    del main_ops
    torch.cuda.synchronize()
    operand_bytes = sum(r.A.rpts.numel() * 4 + r.A.nnz * 12 + r.B.rpts.numel() * 4 + r.B.nnz * 12 for r in dreqs)
    log(f"serve: {len(dreqs)} requests uploaded in {time.perf_counter() - t_gen:.1f}s, "
        f"operands {operand_bytes / 1e9:.2f} GB")

    # warm-up: kernels loaded, allocator primed
    Server(budget).run(dreqs[:32], realtime=False)
    torch.cuda.empty_cache()
    sat = Server(budget).run(dreqs, realtime=False)
    ssum = sat.summary()
    mu = ssum["products_per_s"]
    log(f"serve saturation: {ssum}")
    base_rate = len(reqs) / max(reqs[-1].arrival_s, 1e-9)
    loads = {}
    for frac in (0.5, 0.9):
        lam = frac * mu
        scale = base_rate / lam
        rq = [Request(r.rid, r.arrival_s * scale, r.A, r.B, r.sorted_out) for r in dreqs]
        torch.cuda.empty_cache()                   # each run starts from a clean allocator
        rep = Server(budget).run(rq, realtime=True)
        loads[f"{frac}mu"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rep.summary().items()}
        loads[f"{frac}mu"]["lambda_per_s"] = round(lam, 1)
        slow = sorted(rep.completions, key=lambda c: -c.latency_s)[:5]
        loads[f"{frac}mu"]["slowest"] = [{"rid": c.rid, "path": c.path, "flop": c.flop,
                                          "latency_ms": round(c.latency_s * 1e3, 1)} for c in slow]
        log(f"serve at {frac} mu: {loads[f'{frac}mu']}")
    del dreqs

    small_stratum = measure_small(args, sp, dev, small_ops)
    out = {
        "metric": METRIC,
        "value": round(mu, 2),
        "unit": "products/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": round(sat.wall_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"serve: {WORKLOADS['serve']['desc']}", "requests": len(reqs), "seed": args.seed,
                   "budget_gb": args.budget_gb, "operand_gb": round(operand_bytes / 1e9, 3)},
        "saturation": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in ssum.items()},
        "load": loads,
        "small_stratum": small_stratum,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
