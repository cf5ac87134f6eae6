"""Host-side logic of the measurement tools (no GPU): the work-item trace
report, the benchmark's confidence interval and its counter-record lookup."""
import json
import os
import sys
import types

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1402_6601_amd import trace_report  # noqa: E402


def _trace(items):
    """items: (claim, start, end, workgroup, task) in 100 MHz ticks."""
    words = []
    for claim, start, end, wg, task in items:
        words += [claim, start, end, (wg << 32) | task]
    return torch.tensor(words, dtype=torch.int64)


def test_trace_report_hand_computed():
    # two workgroups over 40 us: wg 1 runs task 1 (kind B) for the whole
    # span; wg 0 claims task 0 (kind A) at 0, waits 10 us, runs 20 us
    tc = types.SimpleNamespace(KIND_NAMES=["A", "B"])
    plan = {"kind": np.array([0, 1], dtype=np.int32)}
    tr = _trace([(0, 1000, 3000, 0, 0), (0, 0, 4000, 1, 1)])
    lines = []
    trace_report.report(tc, plan, tr, "t", out=lines.append)
    assert lines[0] == "[t] makespan 0.04 ms, workgroups 2, busy 0.750, waiting 0.125"
    row_a = lines[2].split()
    row_b = lines[3].split()
    assert row_a[0] == "A" and int(row_a[1]) == 1
    assert float(row_a[2]) == pytest.approx(20.0) and float(row_a[6]) == pytest.approx(10.0)
    assert row_b[0] == "B" and float(row_b[2]) == pytest.approx(40.0) and float(row_b[6]) == pytest.approx(0.0)
    util = [float(x) for x in lines[4].split(":")[1].split()]
    assert len(util) == 20
    # buckets of 2 us: wg 0 runs over [10, 30) us, wg 1 over the whole span
    expect = [1.0 if 5 <= b < 15 else 0.5 for b in range(20)]
    assert util == pytest.approx(expect)


def test_trace_report_skips_absent_kinds():
    tc = types.SimpleNamespace(KIND_NAMES=["A", "B", "C"])
    plan = {"kind": np.array([2, 2], dtype=np.int32)}
    tr = _trace([(0, 0, 500, 0, 0), (500, 500, 1000, 0, 1)])
    lines = []
    trace_report.report(tc, plan, tr, "t", out=lines.append)
    kinds = [l.split()[0] for l in lines[2:-1]]
    assert kinds == ["C"]
    assert lines[0].endswith("busy 1.000, waiting 0.000")


def test_ci95_student_t():
    # n = 5: t(0.975, 4) = 2.776 (tables); s = sqrt(2.5)
    r = bench.ci95([1.0, 2.0, 3.0, 4.0, 5.0])
    assert r["reps"] == 5 and r["mean"] == 3.0 and r["min"] == 1.0 and r["max"] == 5.0
    assert r["ci95_half_width"] == pytest.approx(2.776 * np.sqrt(2.5) / np.sqrt(5), abs=2e-3)
    assert bench.ci95([7.0])["ci95_half_width"] == 0.0
    assert bench.ci95([]) is None


def test_traffic_record_only_for_current_source():
    path = os.path.join(ROOT, "profiles", "traffic_factor_solve_n32768_nb512.json")
    with open(path) as f:
        d = json.load(f)
    got = bench.load_traffic(32768, 512)
    if d["device_source_sha256_16"] == bench.device_source_hash():
        assert got == d["hbm_bytes_per_launch"]
        # at least the algorithmic bytes the record states
        assert got >= d["algorithmic_bytes"]["bytes"]
    else:
        assert got is None
    assert bench.load_traffic(1000, 128) is None
