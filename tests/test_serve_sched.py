"""Host-only tests of the sort server's admission and batching policy: the
policy header is compiled with g++ into a harness that drives it with a
simulated device (no GPU, no HIP)."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def harness():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tempfile.mkdtemp(prefix="serve_sched_")
    exe = os.path.join(d, "harness")
    src = os.path.join(HERE, "serve_sched_harness.cpp")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror", src, "-o", exe], check=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_policy_and_simulated_streams(harness):
    p = subprocess.run([harness], capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stderr
    lines = p.stdout.strip().splitlines()
    assert lines[-1] == "OK"
    assert sum(1 for ln in lines if ln.startswith("stream ")) == 3
