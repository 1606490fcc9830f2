"""The benchmark's host-side contract (no GPU): it refuses more than one GPU
before touching one, its algorithmic byte counts are the per-ray and per-hit
figures of the forward and backward (ray, outputs, one surfel record per
composited hit; the backward reads the record and writes its gradient), and
the measured traffic it reports is taken only from counters recorded on the
same forward kernel sources."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env={**os.environ, "HIP_VISIBLE_DEVICES": ""})
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("F", [3, 8])
def test_algorithmic_bytes(F):
    n_hits = np.array([0, 1, 43, 256])
    H = n_hits.sum()
    R = n_hits.size
    # F = 8: 64 + 72 H per ray forward, 108 + 144 H backward
    assert bench.fwd_bytes(n_hits, F) == R * (24 + 4 * (2 + F)) + H * (40 + 4 * F)
    assert bench.bwd_bytes(n_hits, F) == R * (24 + 8 * (2 + F) + 4) + H * 2 * (40 + 4 * F)
    if F == 8:
        assert bench.fwd_bytes(np.array([10]), 8) == 64 + 72 * 10
        assert bench.bwd_bytes(np.array([10]), 8) == 108 + 144 * 10
    # composited channels other than F (SH colour: 3) change only the outputs
    assert bench.fwd_bytes(n_hits, 48, FO=3) == R * (24 + 4 * 5) + H * (40 + 4 * 48)


def test_traffic_needs_matching_kernel_sources(monkeypatch):
    d = None
    with open(bench.TRAFFIC_FILE) as fh:
        for ln in fh:
            if ln.startswith("traffic-data: "):
                import json
                d = json.loads(ln[len("traffic-data: "):])
    assert d is not None, "the committed traffic summary carries its data line"
    monkeypatch.setattr(bench, "forward_fingerprint", lambda: d["kernel_fingerprint"])
    got = bench.measured_traffic()
    want = (d["fetch_kib"] * 1024 * d["copy_bytes"] / (d["copy_fetch_kib"] * 1024)
            + d["write_kib"] * 1024 * d["copy_bytes"] / (d["copy_write_kib"] * 1024))
    assert got == pytest.approx(want, rel=1e-9)
    assert 0.0 < bench.measured_l2_hit_rate() < 1.0
    monkeypatch.setattr(bench, "forward_fingerprint", lambda: "0" * 16)
    assert bench.measured_traffic() is None
    assert bench.measured_l2_hit_rate() is None


def test_committed_traffic_matches_the_current_sources():
    """The summary under profiles/ was taken on the forward kernel as it is
    in this tree (else the bench line would report traffic as null)."""
    assert bench.measured_traffic() is not None
