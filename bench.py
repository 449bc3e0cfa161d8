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
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_inputs(name: str, seed: int, sorted_flag):
    from synth import (bfs_frontier, erdos_renyi_fixed_degree, rmat, shuffle_within_rows,
                       symmetric_rmat_graph, triangle_inputs, with_values)
    w = WORKLOADS[name]
    srt = w["sorted"] if sorted_flag is None else sorted_flag
    if name == "rmat20":
        A = rmat(20, 16, seed, sorted_rows=srt)
        return dict(A=A, B=A, sorted=srt)
    if name == "er20":
        A = erdos_renyi_fixed_degree(1 << 20, 16, seed, sorted_rows=srt)
        return dict(A=A, B=A, sorted=srt)
    if name == "rmat16":
        A = rmat(16, 16, seed, sorted_rows=srt)
        return dict(A=A, B=A, sorted=srt)
    if name == "er4096":
        A = erdos_renyi_fixed_degree(4096, 8, seed, sorted_rows=True)
        return dict(A=A, B=A, sorted=srt)
    if name == "tri18":
        g = symmetric_rmat_graph(18, 16, seed)
        A, L, U = triangle_inputs(g, degree_order=False)
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
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-flop-budget", type=float, default=3e9,
                    help="multiplications in the oracle's row sample")
    ap.add_argument("--no-timing", action="store_true", help="skip per-kernel HIP events")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the row-parallel "
              "multi-GPU split is a design note, not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1804_01698_amd as sp

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    t_gen = time.perf_counter()
    inp = make_inputs(args.workload, args.seed, args.sorted_flag)
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

    def step(timing: bool):
        p = sp.Plan([dA], [dB], sorted_output=srt, timing=timing)
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

    timing = not args.no_timing
    plans = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        p, C, extra = step(timing)
        plans.append(p)
        del C
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / max(args.steps, 1)

    st = plans[-1].stats(0)
    if st["status"] != 0:
        raise SystemExit(f"device check failed: {st}")
    flop = st["flop"]
    nnz_c = st["nnz_C"]
    gflops = 2.0 * flop / (ms * 1e-3) / 1e9

    # per-kernel times (HIP events on the library's stream, timed region)
    agg = {}
    for p in plans:
        if timing:
            for k in p.kernel_times():
                a = agg.setdefault(k["name"], dict(ms=0.0, launches=0, alg_bytes=0.0))
                a["ms"] += k["ms"]
                a["launches"] += k["launches"]
                a["alg_bytes"] += k["alg_bytes"]
        p.close()
    kernels = sorted(([n, v["ms"] / args.steps, v["launches"] // max(args.steps, 1),
                       v["alg_bytes"] / max(v["launches"], 1)] for n, v in agg.items()),
                     key=lambda r: -r[1])
    roofline = None
    if kernels:
        name, kms, nl, bytes_per_launch = kernels[0]
        avg_launch_ms = kms / max(nl, 1)
        achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "avg_launch_ms": round(avg_launch_ms, 4), "alg_bytes_per_launch": bytes_per_launch}
    nnz_a, nnz_b, m = inp["A"].nnz, inp["B"].nnz, inp["A"].nrows
    path_bytes = 16.0 * flop + 12.0 * nnz_c + 44.0 * nnz_a + 40.0 * m
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
                   "sorted_output": srt, "nrows": m, "nnz_A": nnz_a, "nnz_B": nnz_b, "flop": flop,
                   "nnz_C": nnz_c, "seed": args.seed},
        "roofline": roofline,
        "path_roofline": {"alg_bytes": path_bytes, "achieved": round(path_bytes / (ms * 1e-3) / 1e9, 1),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(path_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "copy_probe_GBs": round(copy_gbs, 1),
        "kernels_ms_per_step": {k[0]: round(k[1], 4) for k in kernels},
    }
    if dM is not None:
        out["triangles"] = int(extra) // 2

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inp, args.cpu_flop_budget, srt, args.seed)
    print(json.dumps(out), flush=True)


def cpu_baseline(inp, budget, srt, seed):
    """The oracle, as it is, on a seeded random sample of rows of the same product."""
    import oracle
    A, B = inp["A"], inp["B"]
    f = oracle.row_flop(A, B)
    order = np.random.default_rng(seed + 99).permutation(A.nrows)
    csum = np.cumsum(f[order])
    k = int(np.searchsorted(csum, budget)) + 1
    rows = np.sort(order[:min(k, A.nrows)])
    sflop = int(f[rows].sum())
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.spgemm(A, B, sorted_output=srt, rows=rows)
    dt = time.perf_counter() - t0
    return {"value": round(2.0 * sflop / dt / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{rows.size} random rows of the same product ({sflop} multiplications, "
                      f"{sflop / max(int(f.sum()), 1):.3%} of the flop), {dt:.1f} s"}


if __name__ == "__main__":
    main()
