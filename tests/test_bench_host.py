"""Host-side logic of bench.py (no GPU): the one-GPU contract and the stored HBM traffic
records of the two streaming sweeps of the block step."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

# Algorithmic bytes per launch of the two sweeps at n = 1e6, r = 4, k = 10, FP64, both spaces:
# update (k + 2) n r 8 per space, window products (k + 1) n r 8 per space.
ALGORITHMIC = {"update": 2 * 12 * 10**6 * 4 * 8, "dots": 2 * 11 * 10**6 * 4 * 8}


def test_more_than_one_gpu_is_refused():
    proc = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                          text=True, timeout=120)
    assert proc.returncode != 0
    assert "one GPU" in proc.stderr


def _records():
    with open(bench.TRAFFIC_RECORD) as f:
        return [json.loads(l.split(":", 1)[1]) for l in f if l.startswith("traffic-record:")]


def test_traffic_records_are_consistent():
    recs = _records()
    assert {r["kernel"] for r in recs} == {"update", "dots"}
    for r in recs:
        assert r["fetch_bytes"] + r["write_bytes"] == r["bytes_per_launch"]
        # a sweep cannot move fewer bytes than its definition; more than 1.5x would be a
        # measurement (or scaling) error, not re-reads this design has
        ratio = r["bytes_per_launch"] / ALGORITHMIC[r["kernel"]]
        assert 0.99 <= ratio <= 1.5, (r["kernel"], ratio)
        assert len(r["sources_sha256"]) == 64


def test_traffic_record_follows_the_kernel_sources(monkeypatch):
    recs = {r["kernel"]: r for r in _records()}
    monkeypatch.setattr(bench, "kernel_sources_digest", lambda: recs["dots"]["sources_sha256"])
    got = bench.measured_traffic("dots", "fp64")
    assert got is not None and got["bytes_per_launch"] == recs["dots"]["bytes_per_launch"]
    assert bench.measured_traffic("dots", "mixed") is None
    monkeypatch.setattr(bench, "kernel_sources_digest", lambda: "0" * 64)
    assert bench.measured_traffic("dots", "fp64") is None
    assert bench.measured_traffic("update", "fp64") is None


@pytest.mark.parametrize("name", bench.KERNEL_SOURCES)
def test_digest_covers_existing_sources(name):
    assert os.path.isfile(os.path.join(ROOT, "paper_2311_16019_amd", "csrc", name))
