"""bench.py's host logic (no GPU): the one-GPU refusal and the committed
HBM traffic table that the timing line quotes."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "one MI355X" in r.stderr
    assert r.stdout == ""


def test_traffic_table_was_taken_on_the_current_kernels():
    # the counters in profiles/traffic.json belong to the kernel sources they
    # were measured on; the timing line reports them only while that holds
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        data = json.load(fh)
    assert data["kernel_source_hash"] == bench.kernel_source_hash()
    for prec, eb in (("fp64", 8), ("fp32", 4)):
        for kind, per_point in (("z", 3), ("xab", 5), ("yba", 4)):
            ent = data["entries"][f"{prec}:{kind}"]
            # algorithmic bytes: fields read and written per grid point of 256^3
            assert ent["algorithmic_bytes_per_launch"] == per_point * eb * 256 ** 3
            # what reached memory: at least the algorithmic bytes, at most 10% more
            assert 0.999 <= ent["ratio"] <= 1.10, (prec, kind, ent["ratio"])
            assert bench.traffic_for(kind, prec) == pytest.approx(ent["hbm_bytes_per_launch"])
