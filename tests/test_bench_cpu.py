"""Host-side checks of bench.py (no GPU): the multi-GPU guard, the
algorithmic-bytes models behind its roofline figures, and the counter
summary's source check."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_vcycle_bytes_model():
    """Per field and level above the 4,096-cell tail: down 24 + 16/2^d and up
    24 + 8/2^d bytes per cell; the tail's levels cost nothing."""
    # 256^2: levels 256^2 and 128^2 are above the tail (64^2 = 4096 is in it)
    want = 2 * sum(c * (24 + 4 + 24 + 2) for c in (256 ** 2, 128 ** 2))
    assert bench.rd_vcycle_bytes(2, 256) == want == 8847360
    # 128^3: 128^3, 64^3, 32^3 above the tail (16^3 = 4096 is in it)
    want3 = 2 * sum(c * (24 + 2 + 24 + 1) for c in (128 ** 3, 64 ** 3, 32 ** 3))
    assert bench.rd_vcycle_bytes(3, 128) == want3
    assert bench.rd_vcycle_bytes(2, 64) == 0.0  # all in the tail


def test_counter_summary_is_tied_to_the_kernel_sources(tmp_path, monkeypatch):
    """measured_counters returns the committed counters only while the stage
    kernel sources hash to the recorded value."""
    got = bench.measured_counters("blast")
    if got:
        assert set(got) == {"traffic_bytes_per_launch", "valu_issue_frac", "fp64_issue_frac"}
        assert got["traffic_bytes_per_launch"] > 8e9  # above the 8.47 GB algorithmic bytes
    assert bench.measured_counters("kh") == {}
    # counters of the van Leer combined-variant kernel belong to no other stage kernel
    assert bench.measured_counters("blast", "koren", 1) == {}
    assert bench.measured_counters("blast", "vanleer", 1) == {}
    assert bench.measured_counters("blast", "mc", 0) == {}
