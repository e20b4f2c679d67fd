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
    # a launch of any number of steps reads and writes every population at least
    # once (less only through a counting error), the roofline's bytes per launch
    _, recs = _records(path)
    for key, rec in recs:
        es = 8 if "double" in rec["kernels"][0]["kernel"] else 4
        assert rec["compulsory_bytes_per_launch"] == 26 * es * rec["nodes"]
        assert rec["bytes_per_launch"] >= 0.98 * rec["compulsory_bytes_per_launch"], (key, rec["launch"])
        assert abs(rec["bytes_per_launch"] - (rec["fetch_bytes"] + rec["write_bytes"])) <= 1.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("steps,diag_every", [(20, 1000), (2040, 1000), (3000, 1000), (7, 3), (5, 0)])
def test_diagnostics_run_at_their_stated_rate(steps, diag_every):
    """Timed chunks cover the steps exactly; diagnostics follow only the chunks
    that end on a multiple of diag_every (none in a run shorter than that)."""
    done, diags = 0, 0
    while done < steps:
        k, d = bench.next_chunk(done, steps, diag_every)
        assert k > 0
        done += k
        diags += d
        if d:
            assert done % diag_every == 0
    assert done == steps
    assert diags == (steps // diag_every if diag_every > 0 else 0)


@pytest.mark.parametrize("precision,spl", [(1, 1), (1, 3), (0, 2), (0, 3)])
def test_roofline_fraction_is_a_fraction(precision, spl):
    """The HBM roofline of a k-step launch counts one read and one write of the
    state per launch: a launch as fast as the peak allows gives frac 1, and
    k does not enter the bytes."""
    nodes = 4096 * 4096
    ideal_ms = bench.BYTES_PER_LU[precision] * nodes / (bench.HBM_PEAK_GBPS * 1e9) * 1e3
    r = bench.roofline(nodes, ideal_ms, precision, spl=spl)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["frac"] == pytest.approx(1.0, rel=1e-3)
    assert r["alu"]["frac"] < 1.0
    slower = bench.roofline(nodes, 2 * ideal_ms, precision, spl=spl,
                            counters={"SQ_INSTS_VALU": 1.0e8, "file": "x"})
    assert slower["frac"] == pytest.approx(0.5, rel=1e-3)
    cap = bench.SIMDS * bench.CLOCK_GHZ * 1e9 * 2 * ideal_ms * 1e-3 / 4
    assert slower["valu_issue"]["frac"] == pytest.approx(1.0e8 / cap, rel=1e-3)
    assert bench.ALU_PEAK_TFLOPS == pytest.approx(78.6, abs=0.1)


@pytest.mark.parametrize("graph_k,steps,spl,expect", [(120, 2040, 3, 120), (120, 20, 3, 18), (120, 5, 3, 0),
                                                      (120, 20, 1, 20), (0, 2040, 3, 0), (120, 11, 2, 8)])
def test_graph_length_is_whole_even_launches(graph_k, steps, spl, expect):
    gk = bench.graph_length(graph_k, steps, spl)
    assert gk == expect
    if gk:
        assert gk % spl == 0 and (gk // spl) % 2 == 0 and gk <= steps


@pytest.mark.parametrize("gk,spl,expect", [(120, 3, 240), (18, 3, 252), (0, 3, 240), (0, 2, 240), (0, 1, 240),
                                           (4096, 3, 4096)])
def test_settle_steps_are_whole_replays(gk, spl, expect):
    """The set-up before timing runs whole graph replays (or whole launches
    without a graph), at least SETTLE_STEPS steps."""
    k = bench.settle_steps(gk, spl)
    assert k == expect and k >= bench.SETTLE_STEPS
    assert k % (gk if gk else spl) == 0
