"""Host logic of bench.py (CPU): the measured-traffic tables it reports from and
its refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _records(path):
    with open(path) as fh:
        t = json.load(fh)
    recs = []
    for key, val in t.items():
        if isinstance(val, dict) and "bytes_per_launch" in val:
            recs.append((key, val))
    for key, alts in t.get("alternates", {}).items():
        recs.extend((key, a) for a in alts)
    return t, recs


TABLES = [bench.TRAFFIC_FILE, bench.BATCH_TRAFFIC_FILE]


@pytest.mark.parametrize("path", TABLES, ids=os.path.basename)
def test_traffic_table_resolves_every_recorded_launch(path):
    t, recs = _records(path)
    assert recs
    if t["kernel_source_sha"] != bench.kernel_sha():
        pytest.skip("kernel sources changed since the counters were taken: the bench reports traffic null")
    for key, rec in recs:
        assert bench.measured_traffic(key, rec["launch"], path) in [r["bytes_per_launch"] for k, r in recs if k == key]


@pytest.mark.parametrize("path", TABLES, ids=os.path.basename)
def test_traffic_is_null_for_other_sources_or_launches(path, monkeypatch):
    _, recs = _records(path)
    key, rec = recs[0]
    other = dict(rec["launch"], steps_per_launch=2, fused_tile=[64, 4])
    assert bench.measured_traffic(key, other, path) is None
    monkeypatch.setattr(bench, "kernel_sha", lambda: "0" * 16)
    assert bench.measured_traffic(key, rec["launch"], path) is None


@pytest.mark.parametrize("path", TABLES, ids=os.path.basename)
def test_recorded_traffic_is_at_least_the_compulsory_bytes(path):
    # a launch of s steps reads and writes every population at least once: 1/s of
    # the algorithmic bytes of s single steps (less only through a counting error)
    _, recs = _records(path)
    for key, rec in recs:
        spl = rec["launch"]["steps_per_launch"]
        assert rec["bytes_per_launch"] >= 0.98 * rec["algorithmic_bytes_per_launch"] / spl, (key, rec["launch"])
        assert abs(rec["bytes_per_launch"] - (rec["fetch_bytes"] + rec["write_bytes"])) <= 1.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
