"""Benchmark of the adaptive equi-join hot path on one MI355X.

One step = the whole path over one synthetic instance already resident in HBM:
statistics of both key columns (min/max + HLL registers), the plan, and the
join (build, probe, materialize the row-id pairs, payload aggregate).

Default workload: the large sparse join -- build 16,777,216 unique int64 keys
(full 64-bit range) with int64 payloads, probe 536,870,912 rows of which 90%
carry a build key, int64 payloads. Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--selector rule|fixed_hash]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "probe tuples/s + HBM GB/s % peak; learned/batched vs fixed hash join"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
CSRC = os.path.join(ROOT, "paper_2607_04489_amd", "csrc")
# Sources that define each timed kernel: a traffic record is valid only while they are unchanged.
KERNEL_SOURCES = {
    "hash_probe": ["join_hash.hip", "join_common.hpp", "common.hpp"],
    "hash_build": ["join_hash.hip", "join_common.hpp", "common.hpp"],
    "direct_probe": ["join_direct.hip", "join_common.hpp", "common.hpp"],
    "radix_scatter": ["join_radix.hip", "join_common.hpp", "common.hpp"],
    "radix_join": ["join_radix.hip", "join_common.hpp", "common.hpp"],
    "radix_hist": ["join_radix.hip", "common.hpp"],
    "cache_probe": ["join_radix.hip", "join_common.hpp", "common.hpp"],
    "stats_partial": ["stats.hip", "common.hpp"],
    "sort_scatter": ["sort.hip", "sort.hpp", "common.hpp"],
    "groupby_partition": ["groupby.hip", "common.hpp"],
}
# Kernel symbol fragments of each timed name (to find them in rocprofv3 output).
KERNEL_SYMBOLS = {
    "hash_probe": "k_probe<eiger::(anonymous namespace)::HashTab", "hash_build": "k_hash_build",
    "direct_probe": "k_probe<eiger::(anonymous namespace)::DirectTab", "radix_scatter": "k_part_scatter",
    "radix_join": "k_radix_join", "radix_hist": "k_part_hist", "cache_probe": "k_cache_probe",
    "stats_partial": "k_stats_partial", "sort_scatter": "k_sort_scatter", "groupby_partition": "k_gb_partition",
}


def sources_digest(name):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(name, []):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(name, workload, plan):
    """HBM bytes per launch of `name` from the committed rocprofv3 counter
    record, or None when there is none, or it was taken on another workload or
    plan, or the kernel's sources changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(name)
    except (OSError, ValueError):
        return None
    if (not rec or rec.get("workload") != workload or rec.get("plan") != plan
            or rec.get("sources_sha") != sources_digest(name)):
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def summarize_profile(d, workload, kernel, plan=None):
    """Read rocprofv3 CSV output under directory d (p_trace, p_fetch, p_write,
    p_cfetch, p_cwrite from the commands in the profile summary) and print the
    traffic record of `kernel` (largest launches) plus a kernel-time table."""
    import csv

    def rows(sub, fname):
        with open(os.path.join(d, sub, fname)) as f:
            return list(csv.DictReader(f))

    def scale(sub, counter):
        vals = [float(r["Counter_Value"]) for r in rows(sub, "run_counter_collection.csv")
                if "copy" in r["Kernel_Name"] and r["Counter_Name"] == counter]
        return (1 << 30) / 1024.0 / max(vals)  # KiB counted per KiB copied, inverted

    fs, ws_ = scale("p_cfetch", "FETCH_SIZE"), scale("p_cwrite", "WRITE_SIZE")
    sym = KERNEL_SYMBOLS[kernel]

    def biggest(sub, counter):
        v = [(int(r["Grid_Size"]), float(r["Counter_Value"])) for r in rows(sub, "run_counter_collection.csv")
             if sym in r["Kernel_Name"] and r["Counter_Name"] == counter]
        g = max(x for x, _ in v)
        sel = [c for x, c in v if x == g]
        return sum(sel) / len(sel) * 1024.0  # bytes

    fetch = biggest("p_fetch", "FETCH_SIZE") * fs
    write = biggest("p_write", "WRITE_SIZE") * ws_
    stats = rows("p_trace", "run_kernel_stats.csv")
    table = []
    for r in stats:
        n = r["Name"]
        if "eiger" not in n:
            continue
        head = n.replace("(anonymous namespace)::", "").split("(")[0]  # drop the argument list
        short = head.replace("void ", "").replace("eiger::", "")
        table.append((float(r["TotalDurationNs"]), short[:60], int(r["Calls"]), float(r["AverageNs"])))
    table.sort(reverse=True)
    rec = {"workload": workload, "kernel": kernel, "plan": plan, "sources_sha": sources_digest(kernel),
           "fetch_bytes_per_launch": int(fetch), "write_bytes_per_launch": int(write),
           "fetch_scale": round(fs, 4), "write_scale": round(ws_, 4)}
    print(json.dumps(rec))
    for tot, name, calls, avg in table[:12]:
        print(f"| {name} | {calls} | {avg / 1e6:.3f} ms | {tot / 1e6:.3f} ms |")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name, device, scale=1):
    import synth
    if name == "sparse_unique64":
        return synth.sparse_unique64(seed=42, n_build=(1 << 24) // scale, n_probe=(1 << 29) // scale,
                                     device=device)
    if name == "plain_dense":
        return synth.plain_dense(seed=42, device=device)
    if name.startswith("skewed_dup32"):
        s = float(name.split("_s")[-1]) if "_s" in name else 1.0
        return synth.skewed_dup32(seed=42, n_distinct=(1 << 24) // scale, n_probe=(1 << 28) // scale,
                                  zipf_s=s, device=device)
    raise SystemExit(f"unknown workload {name}")


def describe(name, inp):
    if name == "sparse_unique64":
        return (f"large sparse join: build {inp.n_build:,} unique int64 keys over the full 64-bit range "
                f"+ int64 payload; probe {inp.n_probe:,} rows, 90% keys drawn from the build keys, "
                f"10% absent; int64 payloads")
    if name == "plain_dense":
        return (f"plain join: build {inp.n_build:,} int32 keys = shuffled [0,65536), probe {inp.n_probe:,} "
                f"int32 keys U[0,81920), int32 payloads")
    return (f"skewed many-to-many join: build {inp.n_build:,} int32 rows over {inp.meta['n_distinct']:,} "
            f"distinct keys (geometric duplicates, mean 4), probe {inp.n_probe:,} Zipf(s={inp.meta['zipf_s']})")


def esize(t):
    return t.element_size()


def kernel_bytes(plan, inp, count):
    """Algorithmic bytes per step of each kernel: every input element the
    kernel's definition consumes is read once, every output element written once."""
    import paper_2607_04489_amd as eg
    nR, nS = inp.n_build, inp.n_probe
    K, PB, PS = esize(inp.build_keys), esize(inp.build_payload), esize(inp.probe_payload)
    b = {"stats_partial": (nR + nS) * K}
    if plan.variant == eg.DIRECT:
        b["direct_count"] = nR * K
        b["direct_fill"] = nR * (K + PB) + nR * (4 + PB)
        b["direct_probe"] = nS * (K + PS) + count * 8
    elif plan.variant == eg.GLOBAL_HASH:
        b["hash_build"] = nR * (K + PB)
        b["hash_probe"] = nS * (K + PS) + count * 8
    elif plan.variant == eg.RADIX_CACHE:
        b["radix_hist"] = (nR + nS) * K
        b["radix_scatter"] = nS * (K + PS) + nS * (K + PS + 4)
        b["cache_build"] = nR * (K + PB)
        b["cache_probe"] = nS * (K + PS + 4) + count * 8
    else:
        passes = 2 if plan.radix_bits > 10 else (1 if plan.radix_bits < 2 else plan.radix_passes)
        b["radix_hist"] = passes * (nR + nS) * K
        sc = (nR * (K + PB) + nS * (K + PS)) + (nR * (K + PB + 4) + nS * (K + PS + 4))
        if passes == 2:
            sc += 2 * (nR * (K + PB + 4) + nS * (K + PS + 4))
        b["radix_scatter"] = sc
        b["radix_join"] = nR * (K + PB + 4) + nS * (K + PS + 4) + count * 8
    return b


def batch_bytes(nb, npr, lf=0.5, radix_bits=0):
    """Device bytes one unique-key int32 join of a batch holds: its four input
    columns, its output range (one pair per probe row at most) and its table
    region (16-byte slots, sized as the library sizes them for load factor lf),
    or for a partitioned join its partitioned copies (key, payload, row id per
    row and pass) and counters."""
    if radix_bits:  # partitioned joins share one workspace region (counted by the caller)
        return 8 * nb + 8 * npr + 8 * npr + (1 << 22)
    slots = 64
    while slots < nb / lf + 1.0:
        slots <<= 1
    if slots < 2 * nb:
        slots <<= 1
    return 8 * nb + 8 * npr + 8 * npr + 16 * slots + 4096


def batch_waves(sizes, budget, tune=None):
    """Split joins (in index order) into the fewest consecutive groups whose
    batch_bytes sum stays within `budget` bytes."""
    import paper_2607_04489_amd as eg
    waves, cur, used = [], [], 0
    for j, (nb, npr) in enumerate(sizes):
        t = tuple((tune or {}).get(eg.batch_bucket(nb), (0.5, 0, 0))) + (0,)
        b = batch_bytes(nb, npr, t[0], t[2])
        if cur and used + b > budget:
            waves.append(cur)
            cur, used = [], 0
        cur.append(j)
        used += b
    if cur:
        waves.append(cur)
    return waves


def bench_batched(n_joins=4096, log2_lo=8.0, log2_hi=22.0, reps=3, autotune=False, seed=42, save_tune=None,
                  compare=True):
    """4,096 independent unique-key int32 joins of uneven sizes (build rows
    2^U(8,22), probe rows 4-16x, match rate U[0.1,1], half dense / half sparse).
    The batch does not fit HBM at once (inputs, outputs and tables of all joins
    are ~380 GB), so the joins are drawn and run in the fewest consecutive
    waves that fit: per wave one captured hipGraph (per-join plan on the
    device), timed, then one eiger_join call sequence per join (rule plan, and
    fixed GLOBAL_HASH) for comparison (skipped with compare=False, e.g. to
    trace the graph's kernels alone). Returns a summary dict."""
    import torch
    import paper_2607_04489_amd as eg
    import synth
    from paper_2607_04489_amd import batch as batchmod
    dev = torch.device("cuda:0")
    sizes = [synth.batched_join_params(seed, j, log2_lo, log2_hi)[:2] for j in range(n_joins)]
    max_np = max(n for _, n in sizes)
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    # the largest join's partitioned copies (the shared partitioned-join workspace)
    max_nb = max(n for n, _ in sizes)
    budget = int(free * 0.85) - 24 * max_np - 2 * 12 * (max_nb + max_np) - (1 << 30)
    tune = None
    if not autotune and os.path.exists(batchmod.TUNE_PATH):
        tune = batchmod.load()
    waves = batch_waves(sizes, budget, tune)
    graph_ms = rule_ms = fixed_ms = 0.0
    pairs = direct = radix = flagged = 0
    agree = True
    for w, idx in enumerate(waves):
        inputs = [synth.batched_join(seed, j, log2_lo, log2_hi, device=dev) for j in idx]
        joins = [(i.build_keys, i.build_payload, i.probe_keys, i.probe_payload) for i in inputs]
        if autotune and tune is None:
            tune, table = batchmod.autotune(joins, log=log)
            if save_tune:
                batchmod.save(tune, save_tune, table)
            import gc
            gc.collect()
            torch.cuda.empty_cache()
        b = eg.Batch(joins, tune)
        b.launch()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            st.record()
            b.launch()
            en.record()
            en.synchronize()
            times.append(st.elapsed_time(en))
        counts, sums, variants, flags = b.results()
        graph_ms += sum(times) / len(times)
        b.destroy()
        del b

        def per_join(selector):
            cap = max(i.n_probe for i in inputs)
            outs = (torch.empty(cap, dtype=torch.int32, device=dev), torch.empty(cap, dtype=torch.int32, device=dev))
            plans = [eg.join_plan(eg.stats(i.build_keys), eg.stats(i.probe_keys), selector) for i in inputs]
            need = max(eg.join_workspace_size(p, i.build_keys, i.build_payload, i.probe_keys, i.probe_payload)
                       for p, i in zip(plans, inputs))
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = [eg.join(i.build_keys, i.build_payload, i.probe_keys, i.probe_payload, p, workspace=ws,
                           outputs=outs) for p, i in zip(plans, inputs)]
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) * 1e3, [(r.count, r.checksum) for r in res]

        t_rule = t_fixed = 0.0
        if compare:
            t_rule, rres = per_join(eg.SEL_RULE)
            t_fixed, _ = per_join(eg.SEL_FIXED_HASH)
            agree = agree and all(r == (int(c), int(s_)) for r, c, s_ in zip(rres, counts, sums))
        rule_ms += t_rule
        fixed_ms += t_fixed
        pairs += int(counts.sum())
        direct += int((variants == eg.DIRECT).sum())
        radix += int((variants == eg.RADIX).sum())
        flagged += int((flags != 0).sum())
        log(f"  wave {w}: {len(idx)} joins, graph {sum(times) / len(times):.2f} ms, per-join rule {t_rule:.1f} ms")
        del inputs, joins
        torch.cuda.empty_cache()
    n_build = sum(n for n, _ in sizes)
    n_probe = sum(n for _, n in sizes)
    return {"joins": n_joins, "waves": len(waves), "wave_sizes": [len(x) for x in waves],
            "build_rows": n_build, "probe_rows": n_probe, "pairs": pairs,
            "graph_ms": round(graph_ms, 3), "graph_probe_tuples_per_s": n_probe / (graph_ms * 1e-3),
            "graph_alg_GBps": round((8 * n_build + 8 * n_probe + 8 * pairs) / (graph_ms * 1e-3) / 1e9, 1),
            "per_join_rule_ms": round(rule_ms, 3), "per_join_fixed_hash_ms": round(fixed_ms, 3),
            "speedup_vs_per_join_rule": round(rule_ms / graph_ms, 2) if compare else None,
            "speedup_vs_per_join_fixed_hash": round(fixed_ms / graph_ms, 2) if compare else None,
            "direct_joins": direct, "radix_joins": radix, "flagged": flagged,
            "agrees_with_single_joins": bool(agree) if compare else None, "tuned": tune is not None,
            "workload": (f"{n_joins} unique-key int32 joins, build rows 2^U({log2_lo:g},{log2_hi:g}), probe 4-16x "
                         f"build, match U[0.1,1], half dense / half sparse keys; drawn and run in "
                         f"{len(waves)} waves that fit HBM")}



def bench_groupby(n_log2=28, reps=3, seed=42, groups_log2=(2, 6, 10, 14, 16, 18, 20, 22, 24, 26), dtypes=None):
    """Group-by at the paper's microbenchmark shape (Section 5.3: 2^28 rows, two
    aggregated columns, g groups): HASH, PARTITION and the HLL-guided choice
    ("auto", which includes the statistics pass) for 4-byte and 8-byte keys and
    values. Each cell is the minimum of `reps` timed runs after one warm-up."""
    import torch
    import paper_2607_04489_amd as eg
    import synth
    dev = torch.device("cuda:0")
    n = 1 << n_log2
    rows = []
    for dt in dtypes or (torch.int32, torch.int64):
        name = "int32" if dt == torch.int32 else "int64"
        ws_stats = torch.empty(eg.lib().eiger_stats_workspace_size(n, eg.column(torch.empty(0, dtype=dt)).dtype),
                               dtype=torch.uint8, device=dev)
        for lg in groups_log2:
            g = 1 << lg
            keys, vals = synth.groupby_input(seed, n, g, key_dtype=dt, n_vals=2, val_dtype=dt, device=dev)
            torch.cuda.synchronize()
            cap = min(n, int(g * 1.25) + 1024)
            res, cell = {}, {"key": name, "groups_log2": lg}
            st0 = eg.stats(keys, workspace=ws_stats)
            fixed = {k: eg.groupby_plan(st0, eg.SEL_FORCED, eg.make_groupby_plan(v))
                     for k, v in (("hash", eg.GB_HASH), ("partition", eg.GB_PARTITION))}

            def run(kind):
                if kind == "auto":  # statistics and plan are part of the timed work
                    return eg.groupby(keys, vals, eg.groupby_plan(eg.stats(keys, workspace=ws_stats)), capacity=cap)
                return eg.groupby(keys, vals, fixed[kind], capacity=cap)

            for kind in ("hash", "partition", "auto"):
                best = None
                for r in range(reps + 1):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    out = run(kind)
                    torch.cuda.synchronize()
                    ms = (time.perf_counter() - t0) * 1e3
                    if r > 0:
                        best = ms if best is None else min(best, ms)
                res[kind] = out
                cell[kind + "_ms"] = round(best, 3)
                if kind == "auto":
                    cell["auto_choice"] = eg.GB_NAMES[out.plan.variant]
                    cell["auto_bits"] = int(out.plan.radix_bits)
                    cell["hll_groups"] = int(out.plan.predicted_groups)
                elif kind == "partition":
                    cell["partition_bits"] = int(out.plan.radix_bits)
            a, b, c = (res[k] for k in ("hash", "partition", "auto"))
            cell["groups"] = a.groups
            cell["agree"] = bool(a.groups == b.groups == c.groups
                                 and int(a.counts.sum()) == int(b.counts.sum()) == n
                                 and all(int(x.sum()) == int(y.sum()) for x, y in zip(a.sums, b.sums)))
            best_fixed = min(cell["hash_ms"], cell["partition_ms"])
            cell["auto_vs_best_fixed"] = round(best_fixed / cell["auto_ms"], 3)
            log(json.dumps(cell))
            rows.append(cell)
            del keys, vals, res, a, b, c
            torch.cuda.empty_cache()
    return {"metric": "group-by rows/s (2^28 rows, 2 sums): hash vs partition vs HLL-guided auto",
            "rows": n, "unit": "ms per group-by (statistics included for auto)", "cells": rows,
            "workload": "2^28 rows, keys uniform over g distinct values spread over the key type, two value "
                        "columns of the key's width uniform over the full range"}


# Table 4 of the paper (GH200, 2^28 rows, 4 int32 keys): the SKF + radix sort
# breakdown, for context only (another machine).
PAPER_SKF_SORT_GH200_MS = {"radix_sort": 12.224, "dictionary_encoding": 6.936, "fusing_keys": 3.393,
                           "hll": 1.061}


def bench_skf_sort(n_log2=28, reps=3, seed=42, configs=((4, "int32"), (2, "int32"), (4, "int64"), (2, "int64"))):
    """Multi-key sort through smart key fusion at the paper's sorting shape
    (Section 5.6: 2^28 rows, 2 or 4 keys of int32 or int64; half of the keys
    narrow -- frame of reference --, half sparse with few distinct values --
    dictionary). One step = statistics (min/max/HLL) of every key, the fusion
    plan, the dictionary encodings, the fusion kernel and the radix sort of the
    fused keys with the row ids (the sorting permutation). Per-kernel times come
    from the library's HIP-event timing on the launch stream."""
    import torch
    import paper_2607_04489_amd as eg
    import synth
    dev = torch.device("cuda:0")
    n = 1 << n_log2
    out = []
    for n_keys, dt_name in configs:
        dt = torch.int32 if dt_name == "int32" else torch.int64
        cols = synth.multikey_table(seed, n, n_keys, dt, narrow_bits=8, sparse_ndv=256, device=dev)
        torch.cuda.synchronize()

        def step():
            st = [eg.stats(c) for c in cols]
            return eg.sort_multikey(cols, plan=eg.skf_plan(st))

        perm, _, fin = step()
        torch.cuda.synchronize()
        # the result is a permutation and orders the rows by the key tuples
        ok = bool(torch.bincount(perm.long(), minlength=n).eq(1).all())
        srt = [c[perm.long()] for c in cols]
        diff = torch.zeros(n - 1, dtype=torch.int8, device=dev)   # 1: decided greater, -1: decided smaller
        for c in srt:
            undecided = diff == 0
            diff = torch.where(undecided & (c[1:] > c[:-1]), torch.ones_like(diff), diff)
            diff = torch.where(undecided & (c[1:] < c[:-1]), -torch.ones_like(diff), diff)
        ok = ok and bool((diff >= 0).all())
        del srt, diff
        best, prof = None, None
        for r in range(reps):
            torch.cuda.synchronize()
            eg.profile_enable(True)
            t0 = time.perf_counter()
            step()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            table = eg.profile_read()
            eg.profile_enable(False)
            if best is None or ms < best:
                best, prof = ms, table
        kb = 4 if fin.fused_bytes == 4 else 8
        scat = prof.get("sort_scatter", (0, 0.0))
        passes = max(1, (int(fin.total_bits) + 7) // 8)
        # sort_scatter algorithmic bytes of the row sort's passes: read key + value,
        # write key + value (the first pass generates the row ids instead of reading
        # them); the few small launches that sort the dictionaries' distinct values
        # are inside the measured time
        alg = n * (2 * kb + 8) * passes - n * 4
        cell = {"keys": n_keys, "dtype": dt_name, "rows": n, "ms": round(best, 3),
                "rows_per_s": n / (best * 1e-3), "fused_bytes": int(fin.fused_bytes),
                "total_bits": int(fin.total_bits), "codes": [k["code"] for k in fin.describe()["keys"]],
                "sorted_ok": ok,
                "kernels_ms": {k: round(v[1], 3) for k, v in sorted(prof.items(), key=lambda x: -x[1][1])},
                "sort_scatter": {"launches": scat[0], "ms": round(scat[1], 3),
                                 "alg_GBps": round(alg / (scat[1] * 1e-3) / 1e9, 1) if scat[1] else None}}
        log(json.dumps(cell))
        out.append(cell)
        del cols
        torch.cuda.empty_cache()
    return {"metric": "multi-key sort rows/s via smart key fusion + radix sort", "unit": "rows/s",
            "cells": out, "paper_gh200_4xi32_ms": PAPER_SKF_SORT_GH200_MS,
            "workload": "2^28 rows; even keys narrow (base + U[0, 2^8)), odd keys one of 256 values spread "
                        "over the type's range; all ascending"}


def bench_join_sweep(reps=3, seed=42):
    """The paper's narrow-join microbenchmarks (Section 5.2: |S| = 2^28 with |R|
    varied, and |R| = 2^16 with |S| varied; unique build keys, every probe row
    matching, a key and one payload column per side of the key's width), timed
    per plan: the hash join (GLOBAL_HASH lf 0.5), the partitioned hash join
    (RADIX, bits from the planner), the sort-merge join (SORT_MERGE) and the
    rule's own choice. Each cell is the minimum of `reps` runs after one
    warm-up; one run = one eiger_join call (statistics excluded, same for all)."""
    import torch
    import paper_2607_04489_amd as eg
    import synth
    dev = torch.device("cuda:0")
    shapes = [(16, s_) for s_ in (16, 18, 20, 22, 24, 26, 28)] + [(r_, 28) for r_ in (20, 22, 24, 26)]
    plans = {"hash": (eg.GLOBAL_HASH, 0, 0, 0.5), "radix": (eg.RADIX, 0, 0, 0.25), "sort_merge": (eg.SORT_MERGE, 0, 0, 0.0)}
    cells = []
    for dt_name, dt in (("int32", torch.int32), ("int64", torch.int64)):
        for r_log, s_log in shapes:
            inp = synth.wide_join(seed, 1 << r_log, 1 << s_log, 1000, n_cols=1, key_dtype=dt, col_dtype=dt, device=dev)
            sb, sp = eg.stats(inp.build_keys), eg.stats(inp.probe_keys)
            cell = {"key": dt_name, "R_log2": r_log, "S_log2": s_log}
            counts = set()
            chosen = {k: eg.join_plan(sb, sp, eg.SEL_FORCED, eg.make_plan(*v)) for k, v in plans.items()}
            chosen["rule"] = eg.join_plan(sb, sp, eg.SEL_RULE)
            cell["rule_plan"] = chosen["rule"].describe()
            for name, plan in chosen.items():
                best = None
                for r in range(reps + 1):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    res = eg.join(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload, plan)
                    torch.cuda.synchronize()
                    ms = (time.perf_counter() - t0) * 1e3
                    if r:
                        best = ms if best is None else min(best, ms)
                counts.add((res.count, res.checksum))
                cell[name + "_ms"] = round(best, 3)
                del res
            cell["agree"] = len(counts) == 1
            fastest = min(plans, key=lambda k: cell[k + "_ms"])
            cell["fastest_fixed"] = fastest
            cell["tuples_per_s_fastest"] = ((1 << r_log) + (1 << s_log)) / (cell[fastest + "_ms"] * 1e-3)
            log(json.dumps(cell))
            cells.append(cell)
            del inp
            torch.cuda.empty_cache()
    return {"metric": "narrow join ms per plan (hash / partitioned hash / sort-merge / rule)", "cells": cells,
            "workload": "unique build keys 2 * shuffle(|R|), every probe row copies a build key; one payload "
                        "column per side of the key's width; throughput = (|R| + |S|) / time"}


def host_cores():
    """Host CPUs this process may run on (its CPU affinity), at most 16."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_baseline(name):
    """The oracle, untuned, on a 1/32-scale instance of the same workload (same
    generator and distributions): statistics of both sides and the sort-merge
    join with canonical pairs, once on one thread and once with its sorts on
    every host core (the merge walk and the statistics stay single-threaded,
    as the oracle is written)."""
    import oracle
    scale = 32 if name in ("sparse_unique64",) or name.startswith("skewed") else 1
    inp = make_workload(name, "cpu", scale=scale)

    def once(threads):
        t0 = time.perf_counter()
        oracle.column_stats(inp.build_keys)
        oracle.column_stats(inp.probe_keys)
        _, cnt, _ = oracle.join_sortmerge(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload,
                                          threads=threads)
        return time.perf_counter() - t0, cnt

    cores = host_cores()
    dt1, cnt = once(1)
    dtn, _ = once(cores)
    return {"value": inp.n_probe / dtn, "unit": "probe tuples/s", "cores": cores, "kind": "oracle",
            "single_core_value": inp.n_probe / dt1,
            "sample": (f"1/{scale}-scale instance of the same generator: build {inp.n_build:,}, probe "
                       f"{inp.n_probe:,} rows ({cnt:,} pairs); stats of both sides + sort-merge join with "
                       f"canonical pairs; {dtn:.1f} s with the sorts on {cores} host threads, {dt1:.1f} s on "
                       f"one (os.cpu_count() = {os.cpu_count()})")}


def ceilings(dev):
    """Measured HBM ceilings beside the published 8 TB/s, with the library's
    calibration kernels (eiger_calibrate): a streaming copy of 4 GiB with
    16-byte loads and stores (read + write bytes per second), and 2^28 random
    32-byte reads from a 2 GiB table (8 in flight per thread), as reads per
    second and as GB/s of the 128-byte lines they fetch."""
    import ctypes
    import torch
    import paper_2607_04489_amd as eg
    n = 1 << 32
    a = torch.ones(n, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    ms = ctypes.c_double()
    s = eg._stream_ptr(None)

    def best(kind, x, y, nb, reads):
        t = []
        for _ in range(4):
            eg._check(eg.lib().eiger_calibrate(kind, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                               nb, reads, ctypes.byref(ms), s))
            t.append(ms.value)
        return min(t[1:])

    t_copy = best(0, a, b, n, 0)
    reads = 1 << 28
    sink = torch.empty(reads // 64, dtype=torch.int32, device=dev)
    t_rand = best(1, a, sink, 1 << 31, reads)
    del a, b, sink
    torch.cuda.empty_cache()
    return {"copy_GBps": round(2 * n / (t_copy * 1e-3) / 1e9, 1),
            "copy_frac_of_peak": round(2 * n / (t_copy * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
            "random_32B_reads_per_s": round(reads / (t_rand * 1e-3) / 1e9, 2) * 1e9,
            "random_read_line_GBps": round(reads * 128 / (t_rand * 1e-3) / 1e9, 1),
            "what": "eiger_calibrate: copy of 4 GiB (16-byte loads/stores); 2^28 random 32-byte reads from a "
                    "2 GiB table, 8 in flight per thread; min of 3 timed runs after one warm-up"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="sparse_unique64")
    ap.add_argument("--selector", default="learned", choices=["learned", "rule", "fixed_hash"],
                    help="plan selection (learned falls back to rule when no model file exists)")
    ap.add_argument("--force", default="", help="variant,bits,passes,lf (e.g. radix,14,2,0.5)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the fixed-hash comparison run")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (counter calibration) and exit")
    ap.add_argument("--calibrate-gather", action="store_true",
                    help="only run random 32-byte-row gathers from a 2 GiB table (counter check) and exit")
    ap.add_argument("--no-ceilings", action="store_true", help="skip the copy / random-read ceilings")
    ap.add_argument("--summarize-profile", default="", metavar="DIR",
                    help="summarize rocprofv3 CSV output under DIR for --kernel and exit (no GPU)")
    ap.add_argument("--kernel", default="hash_probe")
    ap.add_argument("--plan", default=None,
                    help="with --summarize-profile: the profiled run's plan as JSON (its 'plan {...}' log line)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-joins comparison")
    ap.add_argument("--no-learned", action="store_true", help="skip the rule-planner comparison of the learned plan")
    ap.add_argument("--autotune", action="store_true", help="autotune the batched graph before timing it")
    ap.add_argument("--save-tune", default="", metavar="PATH", help="batched: write the autotuned knobs here")
    ap.add_argument("--no-extras", action="store_true", help="skip the multi-key sort and group-by points")
    ap.add_argument("--skf-config", default="", help="skf_sort: one configuration KEYSxDTYPE, e.g. 4xint32")
    ap.add_argument("--gb-config", default="", help="groupby: one cell DTYPExLOG2GROUPS, e.g. int32x20")
    args = ap.parse_args()
    if args.summarize_profile:
        summarize_profile(args.summarize_profile, args.workload, args.kernel,
                          json.loads(args.plan.replace("'", '"')) if args.plan else None)
        return
    if args.workload == "batched":
        import torch  # noqa: F401
        print(json.dumps(bench_batched(autotune=args.autotune, save_tune=args.save_tune or None,
                                       compare=not args.no_compare)), flush=True)
        return
    if args.workload == "groupby":
        kw = {}
        if args.gb_config:
            import torch
            d, lg = args.gb_config.split("x")
            kw = {"groups_log2": (int(lg),), "dtypes": (getattr(torch, d),)}
        print(json.dumps(bench_groupby(reps=max(1, args.steps), **kw)), flush=True)
        return
    if args.workload == "join_sweep":
        print(json.dumps(bench_join_sweep(reps=max(1, args.steps))), flush=True)
        return
    if args.workload == "skf_sort":
        cfg = ((4, "int32"), (2, "int32"), (4, "int64"), (2, "int64"))
        if args.skf_config:
            k, d = args.skf_config.split("x")
            cfg = ((int(k), d),)
        print(json.dumps(bench_skf_sort(reps=max(1, args.steps), configs=cfg)), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(statistics would merge by all-reduce and the probe side would shard by row "
              "range); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2607_04489_amd as eg

    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": 3}), flush=True)
        return
    if args.calibrate_gather:
        # 2^24 random 32-byte rows of a 2 GiB table: 512 MiB of row bytes, 128 MiB
        # of ids read, 512 MiB written; FETCH_SIZE shows the lines the reads fetch
        rows, reads = 1 << 26, 1 << 24
        table = torch.zeros(rows, 4, dtype=torch.int64, device="cuda:0")
        idx = torch.randint(0, rows, (reads,), device="cuda:0",
                            generator=torch.Generator(device="cuda:0").manual_seed(1))
        out = torch.empty(reads, 4, dtype=torch.int64, device="cuda:0")
        for _ in range(3):
            torch.index_select(table, 0, idx, out=out)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_gather_reads": reads, "row_bytes": 32, "table_bytes": rows * 32,
                          "gathers": 3}), flush=True)
        return

    if not eg.available():
        import __graft_entry__
        __graft_entry__.build()
    dev = torch.device("cuda:0")
    log(f"generating {args.workload} on {dev}")
    inp = make_workload(args.workload, dev)
    torch.cuda.synchronize()

    from paper_2607_04489_amd import selector as selmod
    if args.selector == "learned":
        if os.path.exists(selmod.MODEL_PATH):
            selmod.load_model()
        else:
            args.selector = "rule"
    sel = {"learned": eg.SEL_LEARNED, "rule": eg.SEL_RULE, "fixed_hash": eg.SEL_FIXED_HASH}[args.selector]
    forced = None
    if args.force:
        v, bits, passes, lf = args.force.split(",")
        forced = eg.make_plan({"direct": eg.DIRECT, "hash": eg.GLOBAL_HASH, "radix": eg.RADIX,
                               "cache": eg.RADIX_CACHE}[v],
                              int(bits), int(passes), float(lf))
        sel = eg.SEL_FORCED

    # buffers allocated once, outside the timed region
    sb, sp = eg.stats(inp.build_keys), eg.stats(inp.probe_keys)
    plan = eg.join_plan(sb, sp, sel, forced)
    ws_stats = torch.empty(max(eg.lib().eiger_stats_workspace_size(inp.n_probe, eg.column(inp.probe_keys).dtype),
                               eg.lib().eiger_stats_workspace_size(inp.n_build, eg.column(inp.build_keys).dtype)),
                           dtype=torch.uint8, device=dev)

    def prepare(p):
        need = eg.join_workspace_size(p, inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload)
        cap = max(int(p.predicted_out * 1.25) + 1024, inp.n_probe)
        return (torch.empty(need, dtype=torch.uint8, device=dev),
                (torch.empty(cap, dtype=torch.int32, device=dev), torch.empty(cap, dtype=torch.int32, device=dev)))

    ws_join, outs = prepare(plan)

    def step(selector, forced_plan):
        b = eg.stats(inp.build_keys, workspace=ws_stats)
        p = eg.stats(inp.probe_keys, workspace=ws_stats)
        pl = eg.join_plan(b, p, selector, forced_plan)
        return pl, eg.join(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload, pl,
                           workspace=ws_join, outputs=outs)

    def timed(selector, forced_plan, warmup):
        """Mean ms per step over args.steps steps, with the library's per-kernel
        HIP-event timing on (for every plan alike, so comparisons carry the
        same overhead), plus the per-kernel table and the last result."""
        for _ in range(warmup):
            step(selector, forced_plan)
        torch.cuda.synchronize()
        eg.profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            last = step(selector, forced_plan)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        table = eg.profile_read()
        eg.profile_enable(False)
        return dt / args.steps * 1e3, table, last

    log(f"plan {plan.describe()}; warmup {args.warmup}")
    ms, prof, (pl, res) = timed(sel, forced, args.warmup)
    log(f"timed {args.steps} steps: {ms:.3f} ms/step, count={res.count}")

    # sanity against the generator's record (no oracle in the timed path)
    verified = None
    if args.workload == "sparse_unique64":
        src = inp.meta["source_row"]
        hit = src >= 0
        expect_cnt = int(hit.sum())
        expect_cs = int((inp.build_payload[src[hit]] * inp.probe_payload[hit]).sum())
        verified = (res.count == expect_cnt and res.checksum == expect_cs)

    kb = kernel_bytes(pl, inp, res.count)
    rows = []
    for name, (launches, total_ms) in prof.items():
        per_step_ms = total_ms / args.steps
        alg = kb.get(name)
        rows.append((per_step_ms, name, launches // args.steps, alg))
    rows.sort(reverse=True)
    for per_step_ms, name, l, alg in rows:
        gbs = (alg / (per_step_ms * 1e-3) / 1e9) if alg else None
        log(f"  {name:16s} {per_step_ms:8.3f} ms/step  launches/step={l}  "
            + (f"alg {alg/1e9:.3f} GB -> {gbs:.0f} GB/s" if alg else ""))
    dom_ms, dom, dom_launches, dom_bytes = rows[0]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9 if dom_bytes else None
    step_alg = sum(kb.values())

    compare = None
    if not args.no_compare and sel != eg.SEL_FIXED_HASH:
        fplan = eg.join_plan(sb, sp, eg.SEL_FIXED_HASH)
        ws_join, outs = prepare(fplan)
        fms, _, (_, r2) = timed(eg.SEL_FIXED_HASH, None, max(1, args.warmup))
        assert (r2.count, r2.checksum) == (res.count, res.checksum)
        compare = {"fixed_hash_ms_per_step": round(fms, 4), "speedup_vs_fixed_hash": round(fms / ms, 3),
                   "plan": fplan.describe()}
        log(f"fixed hash join: {fms:.3f} ms/step")

    rule_cmp = None
    if not args.no_learned and not args.force and sel == eg.SEL_LEARNED:
        rplan = eg.join_plan(sb, sp, eg.SEL_RULE)
        ws_join, outs = prepare(rplan)
        rms, _, (_, r3) = timed(eg.SEL_RULE, None, max(1, args.warmup))
        assert (r3.count, r3.checksum) == (res.count, res.checksum)
        rule_cmp = {"plan": rplan.describe(), "ms_per_step": round(rms, 4), "learned_speedup": round(rms / ms, 3)}
        log(f"rule planner: {rplan.describe()} {rms:.3f} ms/step")
    batched = None
    if not args.no_batched and args.workload == "sparse_unique64":
        log("batched joins")
        del ws_join, outs
        batched = bench_batched()

    out = {
        "metric": METRIC,
        "value": inp.n_probe / (ms * 1e-3),
        "unit": "probe tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64" if inp.build_keys.dtype == torch.int64 else "int32",
        "data": "synthetic (seeded counter-based generator, resident in HBM)",
        "config": {"workload": describe(args.workload, inp), "name": args.workload,
                   "n_build": inp.n_build, "n_probe": inp.n_probe, "pairs": res.count,
                   "plan": pl.describe(), "selector": args.selector if not args.force else "forced"},
        "effective_GBps": round(step_alg / (ms * 1e-3) / 1e9, 1),
        "effective_frac_of_peak": round(step_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "verified_vs_generator": verified,
        "kernels_ms_per_step": {n: round(t, 4) for t, n, _, _ in rows},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1) if achieved else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": (lambda t: round(t / 1e9, 3) if t else None)(traffic_for(dom, args.workload, pl.describe())),
                     "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "alg_bytes_per_launch": int(dom_bytes / max(dom_launches, 1)) if dom_bytes else None,
                     "avg_launch_ms": round(dom_ms / max(dom_launches, 1), 5)},
    }
    if compare:
        out["vs_fixed_hash"] = compare
    if rule_cmp:
        out["vs_rule_planner"] = rule_cmp
    if batched:
        out["batched"] = batched
    if not args.no_ceilings:
        log("measuring the copy and random-read ceilings")
        out["ceilings"] = ceilings(dev)
    if not args.no_extras and args.workload == "sparse_unique64":
        # one point each of the operators beyond the single join, at the paper's shapes
        del inp
        torch.cuda.empty_cache()
        log("multi-key sort (smart key fusion) and group-by points")
        sk = bench_skf_sort(reps=2, configs=((4, "int32"),))["cells"][0]
        gb = bench_groupby(reps=2, groups_log2=(4, 20), dtypes=(torch.int32,))["cells"]
        out["other_operators"] = {
            "skf_sort_4xint32_2p28": {k: sk[k] for k in ("ms", "rows_per_s", "total_bits", "sorted_ok")},
            "groupby_int32_2p28": [{k: c[k] for k in ("groups_log2", "hash_ms", "partition_ms", "auto_ms",
                                                      "auto_choice", "agree")} for c in gb],
        }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
