"""Host-side logic of bench.py that decides what it reports: a counter record
is attached to a bench line only when it was taken on the same workload, the
same plan and the kernel's current sources."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

PLAN = {"variant": "global_hash", "predicted_out": 1000, "load_factor": 0.25}


def write_record(path, **over):
    rec = {"workload": "w", "kernel": "hash_probe", "plan": PLAN,
           "sources_sha": bench.sources_digest("hash_probe"),
           "fetch_bytes_per_launch": 3000, "write_bytes_per_launch": 500}
    rec.update(over)
    with open(path, "w") as f:
        json.dump({"hash_probe": rec}, f)


def test_traffic_needs_same_workload_plan_and_sources(tmp_path, monkeypatch):
    path = str(tmp_path / "traffic.json")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", path)
    write_record(path)
    assert bench.traffic_for("hash_probe", "w", PLAN) == 3500
    assert bench.traffic_for("hash_probe", "other", PLAN) is None
    assert bench.traffic_for("hash_probe", "w", dict(PLAN, load_factor=0.5)) is None
    assert bench.traffic_for("radix_join", "w", PLAN) is None
    write_record(path, sources_sha="0" * 16)
    assert bench.traffic_for("hash_probe", "w", PLAN) is None
    write_record(path, plan=None)
    assert bench.traffic_for("hash_probe", "w", PLAN) is None


def test_missing_or_broken_record_file(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.json"))
    assert bench.traffic_for("hash_probe", "w", PLAN) is None
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(bad))
    assert bench.traffic_for("hash_probe", "w", PLAN) is None


def test_committed_records_name_their_plan():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        recs = json.load(f)
    for name, rec in recs.items():
        assert rec["kernel"] == name and isinstance(rec.get("plan"), dict) and rec["plan"]["variant"]
