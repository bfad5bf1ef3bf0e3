"""The built library exports every function include/rsort.h declares, and the
Python binding lists exactly those names.  No GPU call is made."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsort.h")
LIB = os.path.join(ROOT, "paper_1808_10292_amd", "librsort.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsort_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        pytest.fail("librsort.so is not built (run __graft_entry__.build())")
    return LIB


def test_every_declared_symbol_is_exported(lib_path):
    out = subprocess.check_output(["nm", "-D", "--defined-only", lib_path], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [s for s in declared() if s not in exported]
    assert not missing, missing
    assert len(declared()) >= 8


def test_binding_names_match_header(lib_path):
    from paper_1808_10292_amd import rsort
    assert sorted(rsort.EXPORTED) == declared()
    lib = rsort.load_library()
    for name in rsort.EXPORTED:
        assert hasattr(lib, name)


def test_status_strings_without_gpu(lib_path):
    from paper_1808_10292_amd import rsort
    lib = rsort.load_library()
    assert lib.rsort_status_string(0) == b"success"
    assert lib.rsort_status_string(-1) == b"invalid argument"
    assert lib.rsort_status_string(-99) == b"unknown status"
    # NULL handles are rejected, not dereferenced
    assert lib.rsort_destroy(None) == rsort.RSORT_EINVAL
    assert lib.rsort_sort(None, 0, None, None, None, None, 0, 0, 32, 0, None, 0, None) == rsort.RSORT_EINVAL
    assert lib.rsort_last_error(None) == b""

