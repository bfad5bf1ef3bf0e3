"""Host-only tests of the segmented tuner's cache file format: the header is
compiled with g++ into a harness (no GPU, no HIP) that writes, damages and
reads back cache files in a scratch directory."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_tune_cache_format_and_lookup():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tempfile.mkdtemp(prefix="tune_cache_")
    try:
        exe = os.path.join(d, "harness")
        subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror",
                        os.path.join(HERE, "tune_cache_harness.cpp"), "-o", exe], check=True)
        p = subprocess.run([exe, d], capture_output=True, text=True, timeout=60)
        assert p.returncode == 0, p.stderr
        assert p.stdout.strip().splitlines()[-1] == "OK"
    finally:
        shutil.rmtree(d, ignore_errors=True)
