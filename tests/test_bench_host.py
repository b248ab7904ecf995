"""Host logic of bench.py (no GPU): the captured-solve budgets taken from the
warm-up, the traffic record's source check, and the one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def interleave(src, cpl):
    out = []
    for a, b in zip(src, cpl):
        out += [a, b]
    return out


def test_budgets_from_the_last_warmup_steps():
    # five warm-up steps: the first, from rest, is never in the window
    its = interleave([3, 1, 0, 0, 0], [280, 40, 25, 22, 20])
    assert bench.graph_budgets(its, 5) == [2, 22]          # medians of steps 3..5
    assert bench.graph_budgets(its, 5, cap=12) == [2, 12]
    # forty steps: the last twenty
    src = [5] * 20 + [0] * 20
    cpl = [100] * 20 + [9, 10, 11, 12] * 5
    assert bench.graph_budgets(interleave(src, cpl), 40, cap=24) == [2, 10]
    # one or two warm-up steps: all of them
    assert bench.graph_budgets(interleave([4], [30]), 1) == [4, 30]
    assert bench.graph_budgets(interleave([0, 0], [7, 9]), 2) == [2, 8]


def test_traffic_record_follows_the_kernel_sources(monkeypatch, tmp_path):
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    ent = rec["k_cg_iter@48^3"]
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: ent["sources"])
    assert bench.traffic_record("k_cg_iter", "48^3") == ent["bytes_per_launch"]
    assert bench.traffic_record("k_cg_iter", "64^3") is None          # not recorded
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "0" * 16)
    assert bench.traffic_record("k_cg_iter", "48^3") is None          # sources changed
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: ent["sources"])
    assert bench.traffic_record("k_cg_iter", "48^3") is None          # no record file


def test_traffic_record_matches_its_summary():
    """Each record's bytes are its counters scaled by the copy calibration."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for ent in rec.values():
        b = 1024.0 * (ent["fetch_kib_per_launch"] * ent["fetch_scale"] +
                      ent["write_kib_per_launch"] * ent["write_scale"])
        assert abs(b - ent["bytes_per_launch"]) <= 1e-5 * b
        assert ent["bytes_per_launch"] >= ent["algorithmic_bytes_per_launch"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "1 GPU" in r.stderr or "--gpus 1" in r.stderr
    assert r.stdout.strip() == ""


def test_budget_cap_per_method():
    """Every start method the bench runs has a cap entry; only the SPE
    windows (whose needs fall once the window fills) are capped."""
    import bench
    for name in ("spe", "cspe", "pod", "prev", "zero"):
        assert name in bench.METHOD_BUDGET_CAP
    assert bench.METHOD_BUDGET_CAP["spe"] == bench.BUDGET_CAP_NODE
    assert bench.METHOD_BUDGET_CAP["cspe"] == bench.BUDGET_CAP_NODE
    assert all(bench.METHOD_BUDGET_CAP[m] is None for m in ("pod", "prev", "zero"))
