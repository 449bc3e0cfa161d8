"""Per-device tuning of the plan configuration (hash multiplier, bin limits, bucket width).

The paper's recipe (Section 5.7, Table 4) picks the SpGEMM variant by input
class -- uniform or skewed pattern, sparse (edge factor <= 8) or dense,
sorted or unsorted output -- and its cost analysis (Section 4.3, Eq. 2)
prices the hash variant at flop*c + sum_i nnz(c_i) log nnz(c_i), c being the
mean number of probes per insertion.  Here the same two ideas choose, per
input class, how full each bin's LDS table may get (a fuller table leaves
room for more blocks per CU but raises c), the hash multiplier and the
bucket width of the tables (4 slots, or the 8- and 16-slot chunks of the
HashVector variant, Section 4.2.2):

1. candidates: one load limit for the symbolic and one for the numeric
   tables (a fraction of every bin's table), times a few odd multipliers;
2. prior: an Eq. 2-style cost from the sample's row statistics (row flop from
   the CSR structure, exact row nnz from the library's symbolic phase):
   sum_i flop_i * c(load_i) + table slots initialised and scanned
   + the sort term when output is sorted, with c(load) the expected probes
   of linear probing (Knuth) at the row's actual table load;
3. the best-ranked candidates (and the defaults), and the best-ranked one
   and the defaults with 8- and 16-slot buckets, are timed end to end
   through the library; for sorted output, so are both with the Heap
   accumulator of Section 4.2.3 for the rows in its envelope (Eq. 1 prices
   it at flop*log nnz(a_i)); the fastest per class is stored in a JSON file
   keyed by device name and CU count.

All timing runs the library's kernels; this module only chooses arguments.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

SYM_TABLE = [64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384]
NUM_TABLE = [64, 128, 256, 512, 1024, 2048, 4096, 8192, 11264]
HEAVY = 8448
LOADS = (0.25, 0.5, 0.75, 1.0)
HASH_MULS = (2654435761, 0x85EBCA6B, 0xCC9E2D51)
BUCKETS = (4, 8, 16)       # slots per bucket: 4, and the HashVector-style 8 and 16 (Section 4.2.2)
HERE = os.path.dirname(os.path.abspath(__file__))
TUNED_DIR = os.path.join(HERE, "tuned")


# ---------------------------------------------------------------- classes

def classify(A, sorted_output: bool) -> str:
    """Input class of a product with left operand A (host CSR with rpts):
    '<uniform|skewed>-<sparse|dense>-<sorted|unsorted>' as in Table 4
    (skewed: the longest row is more than 8x the mean; dense: more than 8
    entries per row on average)."""
    deg = np.diff(np.asarray(A.rpts, dtype=np.int64))
    mean = float(deg.mean()) if deg.size else 0.0
    skew = deg.size > 0 and mean > 0 and float(deg.max()) > 8.0 * mean
    return "-".join(["skewed" if skew else "uniform", "dense" if mean > 8 else "sparse",
                     "sorted" if sorted_output else "unsorted"])


def limits_for(load: float, table: Sequence[int]) -> List[int]:
    """Bin limits filling every table up to ``load`` (non-decreasing, ninth at
    the heavy-row boundary)."""
    out = []
    prev = 0
    for b, t in enumerate(table):
        x = HEAVY if b == 8 else max(1, int(load * t))
        x = max(x, prev)
        out.append(x)
        prev = x
    return out


def make_config(sym_load: float, num_load: float, hash_mul: int, bucket_slots: int = 4) -> dict:
    return {"hash_mul": int(hash_mul), "sym_max": limits_for(sym_load, SYM_TABLE),
            "num_max": limits_for(num_load, NUM_TABLE), "bucket_slots": int(bucket_slots)}


# ---------------------------------------------------------------- prior (Eq. 2)

def _probes(load: np.ndarray) -> np.ndarray:
    """Expected probes per insertion of linear probing at load factor a:
    (1 + 1/(1-a)^2)/2 for a miss, (1 + 1/(1-a))/2 for a hit (Knuth); the mean
    of the two is used (a row mixes first insertions and accumulations)."""
    a = np.clip(load, 0.0, 0.95)
    return 0.25 * (2.0 + 1.0 / (1.0 - a) ** 2 + 1.0 / (1.0 - a))


def _table_of(x: np.ndarray, limits: Sequence[int], table: Sequence[int]) -> np.ndarray:
    lim = np.asarray(limits, dtype=np.int64)
    b = np.searchsorted(lim, x, side="left")        # first bin with x <= limit
    tab = np.asarray(list(table) + [0], dtype=np.int64)
    return tab[np.minimum(b, len(table))]


def prior_cost(flop: np.ndarray, key: np.ndarray, nnz: np.ndarray, cfg: dict, sorted_output: bool) -> float:
    """Eq. 2-style cost of a configuration on rows with the given row flop,
    key bound min(flop, ncols) and exact nnz (rows on the heavy path excluded:
    the configuration does not touch them)."""
    light = (key > 0) & (key <= HEAVY)
    f, x, z = flop[light].astype(np.float64), key[light], nnz[light]
    ts = _table_of(x, cfg["sym_max"], SYM_TABLE).astype(np.float64)
    tn = _table_of(z, cfg["num_max"], NUM_TABLE).astype(np.float64)
    zf = z.astype(np.float64)
    cost = float((f * _probes(zf / ts)).sum() + (f * _probes(zf / tn)).sum())   # flop * c, both phases
    cost += float(ts.sum() + 3.0 * tn.sum())                                     # init + scan of the tables
    if sorted_output:
        cost += float((zf * np.log2(np.maximum(zf, 2.0))).sum())
    return cost




# ---------------------------------------------------------------- timing

def _time_product(sp, dA, dB, sorted_output: bool, cfg: Optional[dict], reps: int) -> float:
    import torch
    best = math.inf
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t = time.perf_counter()
        try:
            p = sp.Plan([dA], [dB], sorted_output=sorted_output, config=cfg)
        except sp.SpgemmError:
            return math.inf                 # an arm the input does not admit (heap on unsorted B)
        p.symbolic()
        p.numeric()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        st = p.stats(0)
        p.close()
        if st["status"] != 0 or st["probe_overflow"]:
            return math.inf
        best = min(best, dt)
    return best


def tune_class(sp, A, B, sorted_output: bool, top: int = 6, reps: int = 3) -> dict:
    """Tune one input class on the sample product A*B (host CSRs)."""
    import torch
    dA = sp.DeviceCSR.from_host(A)
    dB = sp.DeviceCSR.from_host(B)
    p = sp.Plan([dA], [dB], sorted_output=sorted_output)
    p.symbolic()
    nnz = np.diff(p.rpts_C[0].cpu().numpy())
    flop = p.row_flop(0).astype(np.int64)          # the library's row flop (Fig. 4 part 1)
    p.close()
    key = np.minimum(flop, B.ncols)
    default = sp.default_config()
    cands = []
    for sl in LOADS:
        for nl in LOADS:
            for hm in HASH_MULS:
                cfg = make_config(sl, nl, hm)
                cands.append((prior_cost(flop, key, nnz, cfg, sorted_output), cfg))
    cands.sort(key=lambda c: c[0])
    # the bucket width is an arm the prior does not price: the defaults and the
    # best-ranked candidate are also timed with the 8- and 16-slot chunks
    arms = [(cands[0][0], dict(cands[0][1], bucket_slots=w)) for w in BUCKETS[1:]]
    arms += [(None, dict(default, bucket_slots=w)) for w in BUCKETS[1:]]
    if sorted_output:
        arms += [(None, dict(default, heap=1)), (cands[0][0], dict(cands[0][1], heap=1))]
    timed = [(None, default)] + [c for c in cands[:top]] + arms
    results = []
    for prior, cfg in timed:
        ms = _time_product(sp, dA, dB, sorted_output, cfg, reps) * 1e3
        results.append({"config": cfg, "prior": prior, "ms": ms})
    best = min(results, key=lambda r: r["ms"])
    torch.cuda.synchronize()
    return {"config": best["config"], "ms": best["ms"], "default_ms": results[0]["ms"],
            "flop": int(flop.sum()), "candidates": results}


def sample_inputs(scale: int = 16, seed: int = 1):
    """Sample products for the eight classes: ER (uniform) and R-MAT (skewed),
    edge factor 4 (sparse) and 16 (dense), sorted and unsorted output."""
    from synth import erdos_renyi_fixed_degree, rmat
    n = 1 << scale
    out = {}
    for ef in (4, 16):
        er = erdos_renyi_fixed_degree(n, ef, seed)
        rm = rmat(scale, ef, seed)
        for srt in (True, False):
            for A in (er, rm):
                out[classify(A, srt)] = (A, A, srt)
    return out


def device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    name = getattr(p, "gcnArchName", None) or p.name
    return f"{str(name).split(':')[0]}-{p.multi_processor_count}cu"


def tune(sp, classes: Optional[Dict[str, tuple]] = None, path: Optional[str] = None, top: int = 6,
         reps: int = 3) -> dict:
    """Tune every class and write the table (JSON) to ``path`` (default:
    tuned/<device>.json beside this module).  Returns the table."""
    if classes is None:
        classes = sample_inputs()
    table = {"device": device_key(), "created": time.strftime("%Y-%m-%d %H:%M:%S"), "classes": {}}
    for key, (A, B, srt) in classes.items():
        table["classes"][key] = tune_class(sp, A, B, srt, top=top, reps=reps)
    path = path or os.path.join(TUNED_DIR, table["device"] + ".json")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(table, f, indent=1)
    return table


def load(path: str) -> dict:
    with open(path) as f:
        table = json.load(f)
    if "classes" not in table or not isinstance(table["classes"], dict):
        raise ValueError(f"{path}: not a tuning table")
    for key, v in table["classes"].items():
        c = v["config"]
        if len(c["sym_max"]) != 9 or len(c["num_max"]) != 9:
            raise ValueError(f"{path}: class {key} has a malformed config")
    return table


def config_for(table: Optional[dict], A, sorted_output: bool) -> Optional[dict]:
    """The tuned configuration of A's class (None: use the library default)."""
    if not table:
        return None
    v = table["classes"].get(classify(A, sorted_output))
    return None if v is None else v["config"]


if __name__ == "__main__":
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    import paper_1804_01698_amd as _sp
    t = tune(_sp)
    for k, v in t["classes"].items():
        print(f"{k:28s} best {v['ms']:8.3f} ms (default {v['default_ms']:8.3f} ms) {v['config']}", flush=True)
