"""Measurement, training and evaluation of the learned variant selector.

The selector (an MLP in the C library, EIGER_SEL_LEARNED) predicts log2 of the
join time of each of the 16 plan classes from 16 features of the two sides'
statistics. This module produces what it learns from and checks what it gains:

  collect()   time every feasible class on generated instances (exhaustive
              timing; min over repeats, HIP events around eiger_join), append one
              JSON line per instance (resumable)
  train()     full-batch Adam on the GPU through eiger_mlp_train_step (80% split)
  evaluate()  regret t_chosen / t_best on the held-out 20% for the learned
              selector, the rule planner and the fixed hash join
  load_model() / save_model()  the model file (parameters, feature scaling)

Instances come from synth.selector_instance (seeded shapes only).
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np
import torch

import paper_2607_04489_amd as eg

MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_model.json")
DATA_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_data", "timings_mi355x.jsonl")
# family 2 (synth.selector_params): larger builds, wider probe ratios, misses
# inside the build range, full 64-bit key layouts
DATA_PATH_WIDE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_data",
                              "timings_mi355x_wide.jsonl")
# family 3: builds of 2^22..2^28 rows, probes up to 2^29 rows
DATA_PATH_LARGE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_data",
                               "timings_mi355x_large.jsonl")
# family 4: instances shaped like the large sparse and the skewed benchmark joins
# (other seeds and sizes than the benchmark's own instances)
DATA_PATH_SHAPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_data",
                                "timings_mi355x_shaped.jsonl")
DATA_PATHS = (DATA_PATH, DATA_PATH_WIDE, DATA_PATH_LARGE, DATA_PATH_SHAPED)
SHAPED = ([("sparse_unique64", dict(seed=100 + i, n_build=1 << b, n_probe=1 << p, match_per_mille=m))
           for i, (b, p, m) in enumerate([(23, 28, 900), (24, 28, 900), (24, 29, 800), (25, 29, 900),
                                          (22, 29, 900), (24, 27, 950), (23, 29, 700), (25, 28, 900)])] +
          [("skewed_dup32", dict(seed=120 + i, n_distinct=1 << d, n_probe=1 << p, zipf_s=z))
           for i, (d, p, z) in enumerate([(23, 28, 0.5), (24, 27, 1.0), (24, 28, 0.75), (24, 28, 1.25),
                                          (23, 27, 1.5), (22, 28, 1.0), (24, 28, 0.3), (23, 28, 1.1)])])


def _shaped_draws(n, seed=11):
    """More family-4 instances with sizes, match ratio and skew drawn at random
    around the two large shapes (alternating sparse and skewed)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        if i % 2 == 0:
            b, p = int(rng.integers(22, 26)), int(rng.integers(27, 30))
            m = 50 * int(rng.integers(12, 20))
            out.append(("sparse_unique64", dict(seed=200 + i, n_build=1 << b, n_probe=1 << p, match_per_mille=m)))
        else:
            d, p = int(rng.integers(22, 26)), int(rng.integers(27, 29))
            z = round(float(rng.uniform(0.3, 1.5)), 2)
            out.append(("skewed_dup32", dict(seed=200 + i, n_distinct=1 << d, n_probe=1 << p, zipf_s=z)))
    return out


SHAPED = SHAPED + _shaped_draws(48)
FIXED_HASH_CLASS = 2  # GLOBAL_HASH at load factor 0.5


def _time_join(inp, plan, ws, outs, reps, budget_ms):
    """Min over `reps` runs of eiger_join (HIP events on the current stream)."""
    best = math.inf
    res = None
    for r in range(reps):
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        res = eg.join(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload, plan,
                      workspace=ws, outputs=outs)
        stop.record()
        stop.synchronize()
        best = min(best, start.elapsed_time(stop))
        if best > budget_ms:
            break
    return best, res


def measure_instance(inp, reps=3, max_pairs=1 << 32):
    """Exhaustive timing of every feasible class plus the rule plan."""
    sb, sp = eg.stats(inp.build_keys), eg.stats(inp.probe_keys)
    feats = eg.selector_features(sb, sp).tolist()
    plans = [eg.selector_class_plan(c, sb, sp) for c in range(eg.SEL_CLASSES)]
    rule = eg.join_plan(sb, sp, eg.SEL_RULE)
    fixed = eg.join_plan(sb, sp, eg.SEL_FIXED_HASH)
    cnt = eg.join(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload, fixed, count_only=True)
    if cnt.count > max_pairs:
        return {"features": feats, "times_ms": [None] * eg.SEL_CLASSES, "rule_ms": None,
                "rule_plan": rule.describe(), "pairs": cnt.count, "all_variants_agree": None,
                "skipped": f"result above {max_pairs} pairs"}
    cap = max(cnt.count, 1)
    outs = (torch.empty(cap, dtype=torch.int32, device=inp.probe_keys.device),
            torch.empty(cap, dtype=torch.int32, device=inp.probe_keys.device))
    need = max(eg.join_workspace_size(p, inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload)
               for p in plans + [rule] if p is not None)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=inp.probe_keys.device)
    times = [None] * eg.SEL_CLASSES
    agree = True
    best = math.inf
    for c, p in enumerate(plans):
        if p is None:
            continue
        t, res = _time_join(inp, p, ws, outs, reps, budget_ms=max(20 * best, 5.0))
        times[c] = t
        best = min(best, t)
        agree &= (res.count, res.checksum) == (cnt.count, cnt.checksum)
    rule_ms, res = _time_join(inp, rule, ws, outs, reps, budget_ms=math.inf)
    agree &= (res.count, res.checksum) == (cnt.count, cnt.checksum)
    return {"features": feats, "times_ms": times, "rule_ms": rule_ms, "rule_plan": rule.describe(),
            "pairs": cnt.count, "all_variants_agree": bool(agree)}


def collect(path, n_instances, seed=7, reps=3, max_build_log2=22.0, max_probe_log2=25.0, log_every=25,
            device="cuda:0", time_limit_s=None, family=1, min_build_log2=10.0, max_pairs=1 << 32):
    """Append one JSON line per instance to `path`, skipping (seed, idx) pairs
    already there. Instances whose result exceeds `max_pairs` pairs are logged
    as skipped (no timings) rather than materialized."""
    import synth
    done = set()
    if os.path.exists(path):
        with open(path) as f:
            for line in f:
                r = json.loads(line)
                done.add((r["seed"], r["idx"]))
    t0 = time.time()
    kw = dict(max_build_log2=max_build_log2, max_probe_log2=max_probe_log2)
    if family != 1 or min_build_log2 != 10.0:
        kw.update(family=family, min_build_log2=min_build_log2)
    with open(path, "a") as f:
        for idx in range(n_instances):
            if (seed, idx) in done:
                continue
            if time_limit_s and time.time() - t0 > time_limit_s:
                print(f"time limit reached at instance {idx}", flush=True)
                break
            inp = synth.selector_instance(seed, idx, device=device, **kw)
            rec = measure_instance(inp, reps, max_pairs=max_pairs)
            rec.update({"idx": idx, "seed": seed, "params": inp.meta["params"],
                        "n_build": inp.n_build, "n_probe": inp.n_probe})
            f.write(json.dumps(rec) + "\n")
            f.flush()
            del inp
            torch.cuda.empty_cache()
            if idx % log_every == 0:
                ts = [t for t in rec["times_ms"] if t is not None]
                best = f"{min(ts):.3f} ms" if ts else "skipped"
                print(f"instance {idx}: best {best}, elapsed {time.time() - t0:.0f} s", flush=True)


def retime(path, family, classes, out, reps=3, device="cuda:0", log_every=10, time_limit_s=None):
    """Re-time `classes` and the rule plan on every timed instance of family
    `family`'s data file `path`, keeping the other classes' timings: for a kernel
    change that only affects those classes. Writes `out` in the order of `path`
    (skipped instances copied as they are), resuming after what `out` holds."""
    import synth
    kw = {k: v for k, v in FAMILIES[family].items() if k not in ("n_instances", "seed")}
    with open(path) as f:
        recs = [json.loads(line) for line in f]
    done = 0
    if os.path.exists(out):
        with open(out) as f:
            done = sum(1 for _ in f)
    t0 = time.time()
    with open(out, "a") as f:
        for k in range(done, len(recs)):
            rec = recs[k]
            if time_limit_s and time.time() - t0 > time_limit_s:
                print(f"time limit reached at record {k}", flush=True)
                break
            if not rec.get("skipped"):
                inp = synth.selector_instance(rec["seed"], rec["idx"], device=device, **kw)
                assert (inp.n_build, inp.n_probe) == (rec["n_build"], rec["n_probe"]), "instance drifted"
                sb, sp = eg.stats(inp.build_keys), eg.stats(inp.probe_keys)
                fixed = eg.join_plan(sb, sp, eg.SEL_FIXED_HASH)
                rule = eg.join_plan(sb, sp, eg.SEL_RULE)
                cnt = eg.join(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload, fixed,
                              count_only=True)
                cap = max(cnt.count, 1)
                outs = (torch.empty(cap, dtype=torch.int32, device=inp.probe_keys.device),
                        torch.empty(cap, dtype=torch.int32, device=inp.probe_keys.device))
                plans = {c: eg.selector_class_plan(c, sb, sp) for c in classes}
                need = max(eg.join_workspace_size(q, inp.build_keys, inp.build_payload, inp.probe_keys,
                                                  inp.probe_payload) for q in list(plans.values()) + [rule]
                           if q is not None)
                ws = torch.empty(max(need, 1), dtype=torch.uint8, device=inp.probe_keys.device)
                kept = [t for c, t in enumerate(rec["times_ms"]) if t is not None and c not in classes]
                best = min(kept) if kept else math.inf
                agree = rec["all_variants_agree"]
                for c, q in plans.items():
                    if q is None:
                        continue
                    t, res = _time_join(inp, q, ws, outs, reps, budget_ms=max(20 * best, 5.0))
                    rec["times_ms"][c] = t
                    agree &= (res.count, res.checksum) == (cnt.count, cnt.checksum)
                rec["rule_ms"], res = _time_join(inp, rule, ws, outs, reps, budget_ms=math.inf)
                rec["rule_plan"] = rule.describe()
                agree &= (res.count, res.checksum) == (cnt.count, cnt.checksum)
                rec["all_variants_agree"] = bool(agree)
                rec["retimed_classes"] = sorted(classes)
                del inp, outs, ws
                torch.cuda.empty_cache()
            f.write(json.dumps(rec) + "\n")
            f.flush()
            if k % log_every == 0:
                print(f"record {k}: elapsed {time.time() - t0:.0f} s", flush=True)


def load_records(paths=None):
    """Timed instances of every data file (skipped instances left out)."""
    if paths is None:
        paths = [p for p in DATA_PATHS if os.path.exists(p)]
    elif isinstance(paths, str):
        paths = [paths]
    out = []
    for path in paths:
        with open(path) as f:
            for line in f:
                r = json.loads(line)
                if not r.get("skipped"):
                    out.append(r)
    return out


def split(records, seed=0, train_frac=0.8):
    order = np.random.default_rng(seed).permutation(len(records))
    k = int(round(train_frac * len(records)))
    return [records[i] for i in order[:k]], [records[i] for i in order[k:]]


# Instance weight in the training loss: (best time / mean best time)^alpha,
# normalized to mean 1 (alpha 0: every instance alike). The regret that matters
# is summed over instances, where long joins dominate.
TRAIN_WEIGHT_ALPHA = 0.0


def _arrays(records, alpha=0.0):
    X = np.array([r["features"] for r in records], dtype=np.float32)
    T = np.zeros((len(records), eg.SEL_CLASSES), dtype=np.float32)
    M = np.zeros_like(T)
    best = np.array([min(t for t in r["times_ms"] if t is not None) for r in records], dtype=np.float64)
    w = (best / best.mean()) ** alpha if alpha else np.ones_like(best)
    w = w / w.mean()
    for i, r in enumerate(records):
        for c, t in enumerate(r["times_ms"]):
            if t is not None:
                T[i, c] = math.log2(max(t, 1e-3))
                M[i, c] = w[i]
    return X, T, M


def init_params(seed=0):
    """He-normal weights (std sqrt(2/fan_in)) and zero biases, on the CPU."""
    g = torch.Generator().manual_seed(seed)
    parts = []
    for fan_in, fan_out in ((16, 64), (64, 64), (64, 16)):
        parts.append(torch.randn(fan_in * fan_out, generator=g) * math.sqrt(2.0 / fan_in))
        parts.append(torch.zeros(fan_out))
    return torch.cat(parts).float()


def train(records, steps=3000, lr=3e-3, seed=0, device="cuda:0", alpha=None):
    """Full-batch Adam with the library's GPU kernels (loss weights: the mask
    carries each instance's weight, see TRAIN_WEIGHT_ALPHA); returns a model dict."""
    alpha = TRAIN_WEIGHT_ALPHA if alpha is None else alpha
    X, T, M = _arrays(records, alpha)
    mean = X.mean(axis=0)
    std = np.maximum(X.std(axis=0), 1e-3)
    Xn = (X - mean) / std
    dev = torch.device(device)
    tr = eg.MlpTrainer(init_params(seed).to(dev), batch=len(records))
    x, t, m = (torch.from_numpy(a).to(dev).contiguous() for a in (Xn, T, M))
    losses = []
    for s in range(steps):
        tr.step(x, t, m, lr)
        if s % 500 == 0 or s == steps - 1:
            losses.append(float(tr.loss.item()))
    return {"params": tr.params.cpu(), "mean": mean.astype(np.float32), "std": std.astype(np.float32),
            "lo": X.min(axis=0), "hi": X.max(axis=0),
            "losses": losses, "steps": steps, "lr": lr, "seed": seed, "alpha": alpha}


# GLOBAL_HASH classes in ascending load factor (0.25, 0.5, 0.75), and the
# near-tie margin of the library's choice: log2(1.01) in predicted log2 ms.
HASH_CLASSES = (1, 2, 3)
TIE_LOG2 = math.log2(1.01)


def choose(y):
    """The library's learned choice from one row of predictions (infeasible
    classes at +inf): the argmin, moved to the largest-load-factor GLOBAL_HASH
    class predicted within TIE_LOG2 of it when the argmin is a GLOBAL_HASH class."""
    first = int(np.argmin(y))
    best = first
    if first in HASH_CLASSES:
        for c in HASH_CLASSES:
            if c > best and np.isfinite(y[c]) and y[c] - y[first] <= np.float32(TIE_LOG2):
                best = c
    return best


def predict_classes(model, records, device="cuda:0"):
    """The learned choice (see choose) over the classes each record measured."""
    X, _, M = _arrays(records)
    Xn = (X - model["mean"]) / model["std"]
    dev = torch.device(device)
    y = eg.mlp_forward(model["params"].to(dev).contiguous(), torch.from_numpy(Xn.astype(np.float32)).to(dev).contiguous())
    y = y.cpu().numpy()
    y[M == 0] = np.inf
    return np.array([choose(row) for row in y], dtype=np.int64)


def evaluate(model, records, device="cuda:0"):
    """Regret t_chosen / t_best (per instance and summed) of the learned selector,
    the rule planner and the fixed hash join (GLOBAL_HASH, load factor 0.5)."""
    pick = predict_classes(model, records, device)
    best = np.array([min(t for t in r["times_ms"] if t is not None) for r in records])
    rule = np.array([r["rule_ms"] for r in records])
    # outside the training box the library returns the rule plan
    X = np.array([r["features"] for r in records], dtype=np.float32)
    ood = np.zeros(len(records), dtype=bool)
    if model.get("lo") is not None:
        ood = ((X < model["lo"]) | (X > model["hi"])).any(axis=1)
    learned = np.array([rr if o else r["times_ms"][c] for r, c, rr, o in zip(records, pick, rule, ood)])
    fixed = np.array([r["times_ms"][FIXED_HASH_CLASS] for r in records])

    def summary(t):
        ratio = t / best
        return {"sum_ratio": float(t.sum() / best.sum()), "geomean": float(np.exp(np.log(ratio).mean())),
                "p50": float(np.percentile(ratio, 50)), "p90": float(np.percentile(ratio, 90)),
                "p99": float(np.percentile(ratio, 99)), "mean": float(ratio.mean())}

    return {"n": len(records), "out_of_domain": int(ood.sum()), "learned": summary(learned), "rule": summary(rule),
            "fixed_hash": summary(fixed),
            "exhaustive_ms": float(best.sum())}


def save_model(model, path=MODEL_PATH, extra=None):
    doc = {"format": "eiger-selector-mlp-1", "features": eg.SEL_FEATURES, "classes": eg.SEL_CLASSES,
           "hidden": eg.MLP_HIDDEN, "params": [float(v) for v in model["params"].tolist()],
           "mean": [float(v) for v in model["mean"]], "std": [float(v) for v in model["std"]],
           "domain": {"lo": [float(v) for v in model["lo"]], "hi": [float(v) for v in model["hi"]]},
           "train": {"steps": model["steps"], "lr": model["lr"], "seed": model["seed"], "losses": model["losses"],
                     "weight_alpha": model.get("alpha", 0.0)}}
    if extra:
        doc.update(extra)
    with open(path, "w") as f:
        json.dump(doc, f)


def load_model(path=MODEL_PATH, install=True):
    """Read a model file and (by default) install it for EIGER_SEL_LEARNED."""
    with open(path) as f:
        doc = json.load(f)
    if doc.get("format") != "eiger-selector-mlp-1" or len(doc["params"]) != eg.mlp_param_count():
        raise eg.EigerError(eg.EIGER_ERR_MODEL, f"{path}: not a selector model of this library")
    model = {"params": torch.tensor(doc["params"], dtype=torch.float32),
             "mean": np.array(doc["mean"], dtype=np.float32), "std": np.array(doc["std"], dtype=np.float32),
             "steps": doc["train"]["steps"], "lr": doc["train"]["lr"], "seed": doc["train"]["seed"],
             "losses": doc["train"]["losses"],
             "lo": np.array(doc["domain"]["lo"], dtype=np.float32) if "domain" in doc else None,
             "hi": np.array(doc["domain"]["hi"], dtype=np.float32) if "domain" in doc else None}
    if install:
        eg.selector_load(model["params"], model["mean"], model["std"], model["lo"], model["hi"])
    return model


# The three instance families of the training data: collect() arguments.
FAMILIES = {
    1: dict(n_instances=4000, seed=7),
    2: dict(n_instances=771, seed=8, family=2, min_build_log2=16.0, max_build_log2=26.0, max_probe_log2=28.0),
    3: dict(n_instances=243, seed=9, family=3, min_build_log2=22.0, max_build_log2=28.0, max_probe_log2=29.0),
}
FAMILY_PATHS = {1: DATA_PATH, 2: DATA_PATH_WIDE, 3: DATA_PATH_LARGE, 4: DATA_PATH_SHAPED}


def collect_shaped(path, reps=3, device="cuda:0", log=print):
    """Family 4: time every class on the SHAPED instances (resumable by index)."""
    import synth
    done = set()
    if os.path.exists(path):
        with open(path) as f:
            done = {json.loads(line)["idx"] for line in f}
    with open(path, "a") as f:
        for idx, (gen, kw) in enumerate(SHAPED):
            if idx in done:
                continue
            inp = getattr(synth, gen)(device=device, **kw)
            rec = measure_instance(inp, reps)
            rec.update({"idx": idx, "seed": kw["seed"], "params": {"family": 4, "generator": gen, **kw},
                        "n_build": inp.n_build, "n_probe": inp.n_probe})
            f.write(json.dumps(rec) + "\n")
            f.flush()
            ts = [t for t in rec["times_ms"] if t is not None]
            log(f"shaped {idx} {gen} {kw}: best {min(ts):.3f} ms" if ts else f"shaped {idx}: skipped")
            del inp
            torch.cuda.empty_cache()


def main(argv=None):
    """python -m paper_2607_04489_amd.selector collect --family F [--out PATH] [--time-limit S]
       python -m paper_2607_04489_amd.selector retime --family F --classes 1,2,3 --out PATH
       python -m paper_2607_04489_amd.selector train [--out MODEL]
    collect resumes a partial file; train fits on the 80% split of every data
    file and prints the held-out evaluation."""
    import argparse
    ap = argparse.ArgumentParser(prog="paper_2607_04489_amd.selector")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--family", type=int, choices=sorted(FAMILIES) + [4], required=True)
    c.add_argument("--out", default=None)
    c.add_argument("--time-limit", type=float, default=None)
    rt = sub.add_parser("retime")
    rt.add_argument("--family", type=int, choices=sorted(FAMILIES), required=True)
    rt.add_argument("--classes", default="1,2,3", help="comma-separated class indices")
    rt.add_argument("--out", required=True)
    rt.add_argument("--time-limit", type=float, default=None)
    t = sub.add_parser("train")
    t.add_argument("--out", default=MODEL_PATH)
    t.add_argument("--steps", type=int, default=2000)
    t.add_argument("--alpha", type=float, default=None, help="instance weight exponent (default TRAIN_WEIGHT_ALPHA)")
    args = ap.parse_args(argv)
    if args.cmd == "collect":
        if args.family == 4:
            collect_shaped(args.out or DATA_PATH_SHAPED)
            return
        kw = dict(FAMILIES[args.family])
        n = kw.pop("n_instances")
        collect(args.out or FAMILY_PATHS[args.family], n, time_limit_s=args.time_limit, log_every=10, **kw)
        return
    if args.cmd == "retime":
        retime(FAMILY_PATHS[args.family], args.family, [int(c) for c in args.classes.split(",")], args.out,
               time_limit_s=args.time_limit)
        return
    recs = load_records()
    train_set, test_set = split(recs, seed=0)
    model = train(train_set, steps=args.steps, lr=3e-3, seed=0, alpha=args.alpha)
    ev = evaluate(model, test_set)
    by_family = {}
    for f in sorted(FAMILIES) + [4]:
        part = [r for r in test_set if r.get("params", {}).get("family", 1) == f]
        if part:
            by_family[f"family{f}"] = evaluate(model, part)
    save_model(model, args.out, extra={"eval_holdout": ev, "eval_holdout_by_family": by_family,
                                       "records": len(recs)})
    print(json.dumps({"eval_holdout": ev, "eval_holdout_by_family": by_family}), flush=True)


if __name__ == "__main__":
    main()
