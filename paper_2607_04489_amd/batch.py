"""Autotuner of the batched join graph: per size bucket (floor(log2 build rows)),
pick the (load factor, probe tile) that makes that bucket's joins fastest, by
timing graph launches of the bucket's joins alone for every candidate."""
from __future__ import annotations

import json
import math
import os

import torch

import paper_2607_04489_amd as eg

TUNE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_tune.json")
CANDIDATES = [(lf, tile) for lf in (0.25, 0.5) for tile in (4096, 16384, 65536)]


def time_graph(joins, tune, reps=3):
    b = eg.Batch(joins, tune)
    b.launch()
    torch.cuda.synchronize()
    best = math.inf
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        b.launch()
        e.record()
        e.synchronize()
        best = min(best, s.elapsed_time(e))
    b.destroy()
    return best


def autotune(joins, candidates=CANDIDATES, reps=3, log=print):
    """joins: list of (bk, bp, pk, pp). Returns {bucket: (lf, tile)} and the timings."""
    by_bucket = {}
    for q in joins:
        by_bucket.setdefault(eg.batch_bucket(q[0].numel()), []).append(q)
    tune, table = {}, {}
    for b in sorted(by_bucket):
        times = {}
        for lf, tile in candidates:
            times[(lf, tile)] = time_graph(by_bucket[b], {b: (lf, tile)}, reps)
        best = min(times, key=times.get)
        tune[b] = best
        table[b] = {f"{lf}/{tile}": round(t, 4) for (lf, tile), t in times.items()}
        log(f"bucket 2^{b}: {len(by_bucket[b])} joins, best lf={best[0]} tile={best[1]} "
            f"({times[best]:.3f} ms vs default {times.get((0.5, 16384), float('nan')):.3f} ms)")
    return tune, table


def save(tune, path=TUNE_PATH, table=None):
    with open(path, "w") as f:
        json.dump({"format": "eiger-batch-tune-1",
                   "buckets": {str(b): {"load_factor": lf, "probe_tile": tile} for b, (lf, tile) in tune.items()},
                   "timings_ms": {str(b): t for b, t in (table or {}).items()}}, f, indent=1)


def load(path=TUNE_PATH):
    with open(path) as f:
        doc = json.load(f)
    return {int(b): (v["load_factor"], v["probe_tile"]) for b, v in doc["buckets"].items()}
