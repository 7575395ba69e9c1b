"""Host-side pieces of bench.py (no GPU): the algorithmic bytes per row of
each pass, the counter-traffic lookup against the committed profile, and the
one-GPU guard."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bytes_per_row_match_the_row_layout():
    # FP64 values and vector: 12 attitude values 96 B + int32 local start +
    # u read and written; the other 12 values + int64 star + 6 int32
    # instrumental indices + u read and written; the attitude pass reads u once
    b = bench.bytes_per_row(8, 8)
    assert b["attitude_dot"] == 96 + 4 + 16
    assert b["fused_rest"] == 96 + 8 + 24 + 16
    assert b["attitude"] == 96 + 4 + 8
    assert b["aprod1"] == 192 + 40 + 16 and b["aprod2"] == 192 + 40 + 8
    f = bench.bytes_per_row(4, 4)  # the FP32 inner solve
    assert (f["attitude_dot"], f["fused_rest"], f["attitude"]) == (60, 88, 56)


def test_counter_traffic_follows_the_profiled_sources(tmp_path, monkeypatch):
    # the committed profile carries the hash of the kernel sources it was
    # taken with; a profile of other sources gives no traffic figure
    with open(bench.TRAFFIC_PROFILE) as fh:
        text = fh.read()
    lines = [w.split() for w in text.splitlines()]
    rec = {w[1]: float(w[2]) for w in lines if len(w) == 3 and w[0] == "traffic_bytes_per_launch"}
    assert {"attitude_dot", "fused_rest", "attitude"} <= set(rec)
    fake = tmp_path / "profile.txt"
    fake.write_text(text.replace("sources_sha256 ", "sources_sha256 0"))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(fake))
    assert bench.counter_traffic("fused_rest") is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
