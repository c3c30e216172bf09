"""Host logic of bench.py (no GPU): the one-GPU refusal, the algorithmic
bytes the roofline is priced on, and the traffic record lookup."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_pagerank_algorithmic_bytes():
    # offsets (N+1) words, one 4-byte message per vertex, per message a 4-byte
    # target and an 8-byte mailbox read-modify-write
    assert bench.pr_scatter_bytes(10, 100, 8) == 11 * 8 + 40 + 1200
    assert bench.pr_scatter_bytes(10, 100, 4) == 11 * 4 + 40 + 1200
    n, m = 1 << 26, 1060380725  # R-MAT scale 26, edge factor 16, after deduplication
    assert bench.pr_scatter_bytes(n, m, 8) == 13529875076


def test_traffic_record_is_used_only_for_its_own_source_and_run(monkeypatch):
    rec = bench.measured_traffic("sssp-s26@s26", "blocked", 16)
    if rec is None:
        pytest.skip("the blocked kernels changed since their counters were taken")
    assert rec > bench.pr_scatter_bytes(1 << 26, 1060380725, 8)  # counters see more than the algorithmic bytes
    assert bench.measured_traffic("sssp-s26@s26", "blocked", 0) is None  # other message type
    assert bench.measured_traffic("cc-s22@s22", "blocked", 16) is None  # other workload
    monkeypatch.setattr(bench, "kernel_source_hash", lambda form: "0" * 16)
    assert bench.measured_traffic("sssp-s26@s26", "blocked", 16) is None  # kernel source changed


def test_whole_pagerank_superstep_adds_the_rank_write():
    n, m = 1 << 26, 1060380725
    assert bench.pr_superstep_bytes(n, m, 8) == bench.pr_scatter_bytes(n, m, 8) + 4 * n


def test_min_superstep_bytes_formula():
    # SSSP on 10 vertices, int64 offsets, weighted: a source with 3 out-edges
    # reaching 3 receivers, 2 of which improve; then those 2 send 5 messages
    # to 4 receivers, 0 improve
    got = bench.min_superstep_bytes(10, 8, True, [1, 2, 0], [3, 5, 0], [3, 4, 0], dense0=False)
    assert got == [1 * 24 + 3 * 16 + 3 * 12 + 2 * 8, 2 * 24 + 5 * 16 + 4 * 12 + 0, 0]
    # CC, int32 offsets, unweighted, superstep 0 dense: N (4 + o) for the senders
    got = bench.min_superstep_bytes(10, 4, False, [10, 4], [30, 7], [9, 5], dense0=True)
    assert got == [10 * 8 + 30 * 12 + 9 * 12 + 4 * 8, 4 * 16 + 7 * 12 + 5 * 12]
