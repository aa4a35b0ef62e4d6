"""The benchmark's host-side bookkeeping, without a GPU: the counter records in
profiles/ parse into the traffic bench.py reports, stale records are refused,
and the flop counts match their closed forms on a small plan."""
import hashlib
import json
import os
import re

import numpy as np
import pytest

import bench
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def records():
    out = []
    for name in sorted(os.listdir(PROFILES)):
        if not name.endswith("_hbm_counters.md"):
            continue
        for line in open(os.path.join(PROFILES, name)):
            if line.startswith("traffic-record:"):
                out.append((name, json.loads(line.split(":", 1)[1])))
    return out


def test_every_counter_summary_carries_a_wellformed_record():
    recs = records()
    assert len(recs) >= 2
    for name, r in recs:
        assert set(r) >= {"kernel", "source", "source_sha256", "fetch_kib", "fetch_factor", "write_kib",
                          "write_factor"}, name
        assert re.fullmatch(r"[0-9a-f]{64}", r["source_sha256"]), name
        assert os.path.exists(os.path.join(ROOT, r["source"])), name
        assert r["fetch_kib"] > 0 and r["write_kib"] > 0, name
        assert r["fetch_factor"] > 0 and r["write_factor"] > 0, name
        # the summary's name says which kernel and workload it covers
        m = re.fullmatch(r"cheb_step_(\w+?)_(bulk|sheet)_hbm_counters\.md", name)
        assert m, name


def test_counter_traffic_scales_the_record(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"kernel": "k", "source": "k.hip", "source_sha256": sha, "fetch_kib": 1000.0, "fetch_factor": 2.0,
           "write_kib": 10.0, "write_factor": 1.0}
    (prof / "cheb_step_f64_bulk_hbm_counters.md").write_text("text\ntraffic-record: " + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    nbytes, where = bench.counter_traffic("cheb_step_f64", "bulk")
    assert nbytes == pytest.approx(1000.0 * 1024 * 2.0 + 10.0 * 1024)
    assert where.endswith("cheb_step_f64_bulk_hbm_counters.md")
    # the kernel source changed since the counters were taken: no traffic
    src.write_text("kernel source, edited\n")
    nbytes, where = bench.counter_traffic("cheb_step_f64", "bulk")
    assert nbytes is None and "stale" in where
    # no summary for this workload
    assert bench.counter_traffic("cheb_step_f64", "sheet") == (None, None)


def test_flop_counts_match_their_closed_forms():
    P = synth.make_problem(synth.TINY)
    ns = 48
    # one H application: 2 ns times the stored block entries; uniform J = 32 on a
    # 2x2x2 grid with the 7-block stencil: 8 elements x 7 blocks x 32 x 32
    assert bench.filter_flops_per_step(P, ns) == 2.0 * ns * 8 * 7 * 32 * 32
    f1 = bench.sweep_flops(P, ns, 10, 1.0, 20)
    f2 = bench.sweep_flops(P, ns, 10, 2.0, 20)
    assert f1["filter"] == 10 * bench.filter_flops_per_step(P, ns)
    # the second Cholesky-QR pass adds the triangular product and its Gram
    # matrix (2 N ns^2) and a second factor and inverse (2 ns^3 / 3)
    assert f2["orthonormalize"] - f1["orthonormalize"] == pytest.approx(2.0 * P.N * ns * ns + 2.0 * ns ** 3 / 3.0)
    assert f1["rayleigh_ritz"] == f2["rayleigh_ritz"]
