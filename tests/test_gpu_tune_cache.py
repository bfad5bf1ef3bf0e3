"""The segmented tuner's persisted choices (rsort_set_tune_cache) and the
out-of-memory paths forced from the host (rsort_debug_fail_alloc), through the
C ABI.  Every sort is checked against the oracle or numpy's stable sort."""
import ctypes
import json

import numpy as np
import pytest

import keygen
import oracle
from tests.gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1808_10292_amd import rsort
    rsort.load_library()
    return rsort


def reset(rs):
    rs.rsort_segmented_set_split(8192)
    rs.rsort_segmented_set_small_sort("radix")
    rs.rsort_segmented_set_tile(0)
    rs.rsort_segmented_set_launch("rounds")


def lines(path):
    with open(path) as f:
        return [ln for ln in f.read().splitlines() if ln.strip()]


def test_tune_cache_miss_hit_and_bad_entries(rs, tmp_path):
    import torch
    path = str(tmp_path / "tune.jsonl")
    sizes = keygen.lognormal_sizes(200, seed=91)
    off = keygen.offsets_from_sizes(sizes)
    n = int(off[-1])
    keys = keygen.uniform_u32(n, 92)
    want, _ = oracle.segmented(keys, None, off)
    dk = dev(keys)
    rs.rsort_set_tune_cache(path)
    try:
        # miss: tunes, appends one line with the choice it left on the context
        announce("tune cache miss", n)
        ko = torch.zeros_like(dk)
        split, ms = rs.rsort_segmented_tune(dk, ko, off, reps=1)
        assert np.array_equal(host(ko), want)
        got = lines(path)
        assert len(got) == 1
        e = json.loads(got[0])
        cfg = rs.rsort_segmented_get_config()
        assert e["arch"].startswith("gfx") and ":" not in e["arch"]
        assert (e["key_type"], e["payload"]) == (0, 0)
        assert e["log2_keys"] == int(np.ceil(np.log2(n))) and e["log2_segs"] == 8
        assert e["split"] == split == cfg["split"]
        assert e["tile_threads"] == cfg["tile_threads"]
        assert abs(e["ms"] - ms) < 1e-5

        # hit: another configuration set first; the stored one comes back, the
        # batch is sorted once with it and the file is unchanged
        rs.rsort_segmented_set_split(0)
        rs.rsort_segmented_set_tile(256 if cfg["tile_threads"] != 256 else 1024)
        announce("tune cache hit", n)
        ko = torch.zeros_like(dk)
        split2, ms2 = rs.rsort_segmented_tune(dk, ko, off, reps=1)
        assert (split2, ms2) == (e["split"], e["ms"])
        assert rs.rsort_segmented_get_config() == cfg
        assert np.array_equal(host(ko), want)
        assert len(lines(path)) == 1

        # a damaged line and a later entry the library cannot apply (a tile of
        # 300 threads): both ignored, so the batch is tuned again and appended
        bad = dict(e, tile_threads=300)
        with open(path, "a") as f:
            f.write('{"arch": "gfx950", "key_type": 0,\n')
            f.write(json.dumps(bad) + "\n")
        announce("tune cache bad entry", n)
        ko = torch.zeros_like(dk)
        rs.rsort_segmented_tune(dk, ko, off, reps=1)
        assert np.array_equal(host(ko), want)
        got = lines(path)
        assert len(got) == 4 and json.loads(got[-1])["tile_threads"] in (256, 512, 1024)

        # another size class (payloads move) is another key: a miss
        vals = np.arange(n, dtype=np.uint32)
        announce("tune cache payload key", n)
        ko, vo = torch.zeros_like(dk), torch.zeros_like(dev(vals))
        rs.rsort_segmented_tune(dk, ko, off, vals_in=dev(vals), vals_out=vo, reps=1)
        wk, wv = oracle.segmented(keys, vals, off)
        assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)
        got = lines(path)
        assert len(got) == 5 and json.loads(got[-1])["payload"] == 1
    finally:
        rs.rsort_set_tune_cache(None)
        reset(rs)


def test_unwritable_cache_is_not_an_error(rs, tmp_path):
    import torch
    path = str(tmp_path / "no_such_dir" / "tune.jsonl")
    sizes = [5000, 20000, 3, 70001]
    off = keygen.offsets_from_sizes(sizes)
    keys = keygen.uniform_u32(int(off[-1]), 93)
    dk = dev(keys)
    rs.rsort_set_tune_cache(path)
    try:
        announce("tune cache unwritable", int(off[-1]))
        ko = torch.zeros_like(dk)
        rs.rsort_segmented_tune(dk, ko, off, reps=1)
        want, _ = oracle.segmented(keys, None, off)
        assert np.array_equal(host(ko), want)
    finally:
        rs.rsort_set_tune_cache(None)
        reset(rs)


def test_forced_allocation_failures(rs):
    """The k-th device allocation fails: context creation, a first sort's
    workspace and a first sample sort's statistics each return RSORT_ENOMEM,
    leave nothing half made, and the same call succeeds afterwards."""
    import torch
    lib = rs.load_library()
    h = ctypes.c_void_p()
    try:
        rs.rsort_debug_fail_alloc(1)   # the context's error word
        assert lib.rsort_create(0, ctypes.byref(h)) == rs.RSORT_ENOMEM and not h.value
        assert lib.rsort_create(0, ctypes.byref(h)) == 0 and h.value

        n = 1 << 18
        keys = keygen.uniform_u32(n, 94)
        dk = dev(keys)
        ko = torch.zeros_like(dk)
        args = (h, 0, ctypes.c_void_p(dk.data_ptr()), ctypes.c_void_p(ko.data_ptr()), None, None,
                n, 0, 32, rs.RSORT_LSD_R8, None, 0, None)
        rs.rsort_debug_fail_alloc(1)   # the context's first workspace
        announce("fail alloc workspace", n)
        assert lib.rsort_sort(*args) == rs.RSORT_ENOMEM
        assert b"workspace" in lib.rsort_last_error(h)
        assert lib.rsort_sort(*args) == 0
        assert lib.rsort_synchronize(h, None) == 0
        assert np.array_equal(host(ko), np.sort(keys, kind="stable"))

        vals = np.arange(n, dtype=np.uint32)
        dv = dev(vals)
        ko2, vo = torch.zeros_like(dk), torch.zeros_like(dv)
        sargs = (h, 0, ctypes.c_void_p(dk.data_ptr()), ctypes.c_void_p(ko2.data_ptr()),
                 ctypes.c_void_p(dv.data_ptr()), ctypes.c_void_p(vo.data_ptr()), n, 64, 8,
                 None, 0, None)
        rs.rsort_debug_fail_alloc(1)   # the sample sort's statistics
        announce("fail alloc sample stats", n)
        assert lib.rsort_sample_sort(*sargs) == rs.RSORT_ENOMEM
        assert lib.rsort_sample_sort(*sargs) == 0
        assert lib.rsort_synchronize(h, None) == 0
        order = np.argsort(keys, kind="stable")
        assert np.array_equal(host(ko2), keys[order]) and np.array_equal(host(vo), order)
    finally:
        rs.rsort_debug_fail_alloc(0)
        if h.value:
            lib.rsort_destroy(h)
    with pytest.raises(rs.RsortError):
        rs.rsort_debug_fail_alloc(-1)


def test_forced_allocation_failure_in_server_create(rs):
    import torch
    lib = rs.load_library()
    sv = ctypes.c_void_p()
    try:
        rs.rsort_debug_fail_alloc(1)
        assert lib.rsort_server_create(0, 1 << 30, 2, ctypes.byref(sv)) == rs.RSORT_ENOMEM
        assert not sv.value
    finally:
        rs.rsort_debug_fail_alloc(0)
    announce("server after failed create")
    srv = rs.Server(1 << 30, num_streams=2)
    try:
        keys = keygen.uniform_u32(100003, 95)
        dk = dev(keys)
        ko = torch.zeros_like(dk)
        srv.wait(srv.submit(dk, ko))
        assert np.array_equal(host(ko), np.sort(keys, kind="stable"))
    finally:
        srv.destroy()


def test_tune_cache_path_from_environment(rs, tmp_path, monkeypatch):
    """A context made while RSORT_TUNE_CACHE is set writes its tuner's choice there."""
    import torch
    path = str(tmp_path / "env_tune.jsonl")
    lib = rs.load_library()
    sizes = [3000, 9000, 40000, 1, 0, 12345]
    off = keygen.offsets_from_sizes(sizes)
    n = int(off[-1])
    keys = keygen.uniform_u64(n, 96)
    want, _ = oracle.segmented(keys, None, off)
    dk = dev(keys)
    ko = torch.zeros_like(dk)
    monkeypatch.setenv("RSORT_TUNE_CACHE", path)
    h = ctypes.c_void_p()
    assert lib.rsort_create(0, ctypes.byref(h)) == 0
    try:
        split, ms = ctypes.c_uint32(), ctypes.c_double()
        offs = np.ascontiguousarray(off, dtype=np.uint64)
        announce("tune cache from environment, u64", n)
        rc = lib.rsort_segmented_tune(h, 1, ctypes.c_void_p(dk.data_ptr()),
                                      ctypes.c_void_p(ko.data_ptr()), None, None,
                                      ctypes.c_void_p(offs.ctypes.data), len(sizes), 1, None,
                                      ctypes.byref(split), ctypes.byref(ms))
        assert rc == 0
        assert np.array_equal(host(ko), want)
        got = lines(path)
        assert len(got) == 1
        e = json.loads(got[0])
        assert (e["key_type"], e["payload"], e["split"]) == (1, 0, split.value)
    finally:
        lib.rsort_destroy(h)


def test_fault_alloc_from_environment():
    """RSORT_FAULT_ALLOC=1 in a fresh process: its first device allocation (the
    context's error word) fails as out of memory, the next context works."""
    import os
    import subprocess
    import sys
    code = (
        "from paper_1808_10292_amd import rsort\n"
        "try:\n"
        "    rsort.Context(0)\n"
        "    print('created')\n"
        "except rsort.RsortError as e:\n"
        "    print('status', e.status)\n"
        "c = rsort.Context(0)\n"
        "print('second ok', bool(c.handle))\n"
    )
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, RSORT_FAULT_ALLOC="1")
    announce("fault alloc from environment (subprocess)")
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                       env=env, cwd=root)
    assert p.returncode == 0, p.stderr[-2000:]
    out = p.stdout.split()
    assert "status" in out and out[out.index("status") + 1] == "-2", p.stdout
    assert "second" in out and out[-1] == "True", p.stdout
