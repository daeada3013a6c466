"""CPU checks of bench.py's host logic: the one-GPU guard, and the committed
HBM-traffic summaries it reads (a summary counts only for the kernel sources
it was taken on)."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

M, N = bench.M, bench.N
ALGORITHMIC = {
    # A once, the input vector once, the float64 output once
    "gemv_n": M * N * 4 + N * 4 + M * 8,
    "gemv_t": M * N * 4 + M * 4 + N * 8,
    # A once, p once, w and A^T w written once
    "gemv_fused": M * N * 4 + N * 4 + M * 8 + N * 8,
}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("kernel", sorted(ALGORITHMIC))
def test_traffic_summary_within_a_few_percent_of_algorithmic(kernel):
    v = bench.measured_traffic(kernel)
    if v is None:
        pytest.skip(f"the {kernel} counter summary was taken on other sources")
    assert 1.0 <= v / ALGORITHMIC[kernel] < 1.05, v / ALGORITHMIC[kernel]


def test_traffic_is_null_for_other_sources(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_digest", lambda kernel="gemv_n": "0" * 16)
    for kernel in ALGORITHMIC:
        assert bench.measured_traffic(kernel) is None


def test_traffic_digest_covers_the_listed_sources():
    for kernel, (summary, sources) in bench.TRAFFIC.items():
        assert os.path.exists(os.path.join(ROOT, "profiles", summary)), summary
        for rel in sources:
            assert os.path.exists(os.path.join(ROOT, rel)), rel
