"""Host-side logic of bench.py (no GPU): the one-GPU guard and the rule that
the committed HBM byte counters are used only for the kernel source they were
taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _counter_fields():
    fields = {}
    for line in open(bench.COUNTERS_FILE):
        if "=" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split("=", 1)
            fields[k.strip()] = v.strip().strip("`")
    return fields


def test_counters_summary_is_machine_readable():
    f = _counter_fields()
    assert len(f["source_sha256_16"]) == 16
    traffic = float(f["traffic_bytes_per_launch"])
    # one read and one write of 2^27 4-byte keys is the least a round can move
    assert traffic >= 2 * (1 << 27) * 4
    assert 0.5 < float(f["fetch_scale"]) < 4 and 0.5 < float(f["write_scale"]) < 4


def test_traffic_only_for_the_profiled_source(monkeypatch):
    f = _counter_fields()
    if f["source_sha256_16"] != bench.source_sha():
        pytest.skip("kernel source changed since the counters were taken (bench reports null)")
    assert bench.committed_traffic() == float(f["traffic_bytes_per_launch"])
    monkeypatch.setattr(bench, "source_sha", lambda: "0" * 16)
    assert bench.committed_traffic() is None


def test_source_hash_covers_the_round_kernels():
    h = bench.source_sha()
    assert len(h) == 16 and int(h, 16) >= 0
    assert h == bench.source_sha()
