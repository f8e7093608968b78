"""Host logic of bench.py that needs no GPU: the per-launch HBM traffic it
reports is read from the committed counter summary only while the decide
kernels' source is the one the counters were taken on."""
from __future__ import annotations

import importlib.util
import os
import shutil

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_at(root):
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.ROOT = root
    return mod


def _tree(tmp_path, src_suffix=b""):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_1304_4453_amd" / "csrc").mkdir(parents=True)
    shutil.copy(os.path.join(ROOT, "profiles", "decide_traffic_rmat26.md"), tmp_path / "profiles")
    src = open(os.path.join(ROOT, "paper_1304_4453_amd", "csrc", "move.hip"), "rb").read()
    (tmp_path / "paper_1304_4453_amd" / "csrc" / "move.hip").write_bytes(src + src_suffix)
    return str(tmp_path)


def test_traffic_follows_the_source_hash(tmp_path):
    import hashlib
    import json
    text = open(os.path.join(ROOT, "profiles", "decide_traffic_rmat26.md")).read()
    blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    src = open(os.path.join(ROOT, "paper_1304_4453_amd", "csrc", "move.hip"), "rb").read()
    matches = blob["move_hip_sha256"] == hashlib.sha256(src).hexdigest()
    b = _bench_at(_tree(tmp_path))
    level = blob.get("level", 0)
    tr = b.counter_traffic("k_hub_part+k_hub_agg", level)
    if matches:
        k = [k for k in blob["kernels"] if k["kernel"] == "k_hub_part+k_hub_agg"][0]
        assert tr is not None and tr["bytes_per_launch"] == k["traffic_bytes_per_launch"]
        assert tr["bytes_per_launch"] >= tr["algorithmic_bytes_per_launch_same_sweep"]
    else:
        assert tr is None
    # counters of one level are not reported for another
    assert b.counter_traffic("k_hub_part+k_hub_agg", level + 1) is None
    assert b.counter_traffic("no_such_kernel", level) is None


def test_traffic_is_null_once_the_source_changes(tmp_path):
    b = _bench_at(_tree(tmp_path, b"\n// changed\n"))
    assert b.counter_traffic("k_hub_part+k_hub_agg") is None
    assert b.counter_traffic("k_decide_wave") is None


def test_traffic_is_null_without_a_summary(tmp_path):
    root = _tree(tmp_path)
    os.remove(os.path.join(root, "profiles", "decide_traffic_rmat26.md"))
    assert _bench_at(root).counter_traffic("k_hub_part+k_hub_agg") is None
