"""Autotuner of the batched join graph: per size bucket (floor(log2 build rows)),
pick the (load factor, probe tile, radix bits) that makes that bucket's joins
fastest, by timing graph launches of the bucket's joins alone for every
candidate. radix bits 0 keeps the per-join table choice on the device (DIRECT
or GLOBAL_HASH); > 0 runs the bucket through the partitioned join (fan-out
2^bits) inside the graph."""
from __future__ import annotations

import json
import math
import os

import torch

import paper_2607_04489_amd as eg

TUNE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_tune.json")
CANDIDATES = [(lf, tile, 0) for lf in (0.25, 0.5) for tile in (4096, 16384, 65536)]
RADIX_FROM_BUCKET = 14  # smaller joins: a partitioned join's ~20 launches outweigh its work


def candidates_for(bucket, base=CANDIDATES):
    """Hash/direct candidates, plus partitioned fan-outs around ~2^11 build rows
    per partition for buckets of 2^14 build rows and more."""
    out = list(base)
    if bucket >= RADIX_FROM_BUCKET:
        out += [(0.25, 16384, bits) for bits in sorted({max(1, min(16, bucket - d)) for d in (12, 11, 10)})]
    return out


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


def autotune(joins, candidates=None, reps=3, log=print, max_joins=64):
    """joins: list of (bk, bp, pk, pp). Returns {bucket: (lf, tile, bits)} and the
    timings; each bucket is timed on at most `max_joins` of its joins."""
    by_bucket = {}
    for q in joins:
        by_bucket.setdefault(eg.batch_bucket(q[0].numel()), []).append(q)
    tune, table = {}, {}
    for b in sorted(by_bucket):
        times = {}
        sub = by_bucket[b][:max_joins]  # the same joins for every candidate
        for c in (candidates or candidates_for(b)):
            times[tuple(c)] = time_graph(sub, {b: tuple(c)}, reps)
        best = min(times, key=times.get)
        tune[b] = best
        table[b] = {f"{lf}/{tile}/{bits}": round(t, 4) for (lf, tile, bits), t in times.items()}
        log(f"bucket 2^{b}: {len(sub)} of {len(by_bucket[b])} joins, best lf={best[0]} tile={best[1]} radix_bits={best[2]} "
            f"({times[best]:.3f} ms vs default {times.get((0.5, 16384, 0), float('nan')):.3f} ms)")
    return tune, table


def save(tune, path=TUNE_PATH, table=None):
    with open(path, "w") as f:
        json.dump({"format": "eiger-batch-tune-1",
                   "buckets": {str(b): {"load_factor": v[0], "probe_tile": v[1], "radix_bits": (tuple(v) + (0,))[2]}
                               for b, v in tune.items()},
                   "timings_ms": {str(b): t for b, t in (table or {}).items()}}, f, indent=1)


def load(path=TUNE_PATH):
    with open(path) as f:
        doc = json.load(f)
    return {int(b): (v["load_factor"], v["probe_tile"], v.get("radix_bits", 0)) for b, v in doc["buckets"].items()}
