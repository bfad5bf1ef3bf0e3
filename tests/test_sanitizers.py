"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the oracle
(oracle/sr4.c, every entry point on small inputs and edge cases, driven by
tests/oracle_sanitize_driver.c) and the sort server's admission and batching
policy (tests/serve_sched_harness.cpp) and the segmented tuner's cache file
format (tests/tune_cache_harness.cpp).  Any report fails the run."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]


@pytest.fixture(scope="module")
def tmp():
    d = tempfile.mkdtemp(prefix="rsort_san_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def build_and_run(cmd, exe, args=()):
    try:
        subprocess.run(cmd, check=True, capture_output=True, text=True)
    except subprocess.CalledProcessError as e:
        if "asan" in e.stderr.lower() and "cannot find" in e.stderr.lower():
            pytest.skip("sanitizer runtime not installed")
        raise
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    p = subprocess.run([exe] + list(args), capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "Sanitizer" not in p.stderr, p.stderr[-4000:]
    assert p.stdout.strip().splitlines()[-1] == "OK"


def test_oracle_under_asan_ubsan(tmp):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = os.path.join(tmp, "oracle_san")
    build_and_run(["gcc", "-std=c11", "-Wall", "-Werror"] + SAN +
                  [os.path.join(HERE, "oracle_sanitize_driver.c"),
                   os.path.join(ROOT, "oracle", "sr4.c"), "-o", exe], exe)


def test_serve_policy_under_asan_ubsan(tmp):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = os.path.join(tmp, "serve_san")
    build_and_run(["g++", "-std=c++17", "-Wall", "-Werror"] + SAN +
                  [os.path.join(HERE, "serve_sched_harness.cpp"), "-o", exe], exe)


def test_tune_cache_under_asan_ubsan(tmp):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = os.path.join(tmp, "tune_san")
    work = os.path.join(tmp, "tune_files")
    os.makedirs(work, exist_ok=True)
    build_and_run(["g++", "-std=c++17", "-Wall", "-Werror"] + SAN +
                  [os.path.join(HERE, "tune_cache_harness.cpp"), "-o", exe], exe, [work])
