"""GPU parity of the batched segmented sort against the oracle's per-segment SR4.

Segments cover every size class boundary of the in-LDS path (1024 / 4096 /
8192 keys), the tiled path (longer segments, ragged last tiles), empty and
one-key segments, constant segments (identity rounds), u64 keys, payloads,
in-place sorting, the all-tiled split, the lognormal 4096-segment batch, and
the BTN / OET small-segment sorters.  Every comparison is bit-exact.
"""
import numpy as np
import pytest

import keygen
import oracle
from tests.gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu

BOUNDARY_SIZES = [0, 1, 2, 31, 32, 33, 1023, 1024, 1025, 4095, 4096, 4097, 8191, 8192,
                  8193, 16384, 16385, 100001, 0, 7]


@pytest.fixture(scope="module")
def rs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1808_10292_amd import rsort
    rsort.load_library()
    yield rsort
    rsort.rsort_segmented_set_split(8192)
    rsort.rsort_segmented_set_tile(0)
    rsort.rsort_segmented_set_launch("rounds")


def run_case(rs, keys, sizes, with_vals, in_place=False):
    off = keygen.offsets_from_sizes(np.asarray(sizes))
    n = keys.size
    vals = np.arange(n, dtype=np.uint32)
    wk, wv = oracle.segmented(keys, vals if with_vals else None, off)
    dk = dev(keys)
    dv = dev(vals) if with_vals else None
    if in_place:
        rs.rsort_segmented_sort(dk, dk, off, dv, dv)
        ko, vo = dk, dv
    else:
        import torch
        ko = torch.empty_like(dk)
        vo = torch.empty_like(dv) if with_vals else None
        rs.rsort_segmented_sort(dk, ko, off, dv, vo)
    rs.rsort_synchronize()
    assert np.array_equal(host(ko), wk)
    if with_vals:
        assert np.array_equal(host(vo), wv)


@pytest.mark.parametrize("with_vals", [False, True])
def test_boundary_sizes_u32(rs, with_vals):
    n = int(sum(BOUNDARY_SIZES))
    announce("seg boundaries u32", with_vals)
    keys = keygen.uniform_u32(n, 31)
    run_case(rs, keys, BOUNDARY_SIZES, with_vals)


@pytest.mark.parametrize("with_vals", [False, True])
def test_boundary_sizes_u64(rs, with_vals):
    n = int(sum(BOUNDARY_SIZES))
    announce("seg boundaries u64", with_vals)
    keys = keygen.uniform_u64(n, 32)
    keys[::3] = keys[5]
    run_case(rs, keys, BOUNDARY_SIZES, with_vals)


@pytest.mark.parametrize("dist", keygen.KV_DISTRIBUTIONS)
def test_distributions(rs, dist):
    sizes = [3000, 9000, 700, 20000, 8192, 1]
    announce("seg dist", dist)
    keys = keygen.kv_keys(dist, int(sum(sizes)))
    run_case(rs, keys, sizes, True)


def test_in_place(rs):
    sizes = [5000, 50000, 100, 9000]
    announce("seg in place")
    keys = keygen.zipf_keys(int(sum(sizes)), 8)
    run_case(rs, keys, sizes, True, in_place=True)
    run_case(rs, keys, sizes, False, in_place=True)


def test_all_tiled_split(rs):
    sizes = [1, 100, 5000, 8192, 30000]
    announce("seg split 0")
    keys = keygen.uniform_u32(int(sum(sizes)), 9)
    rs.rsort_segmented_set_split(0)
    try:
        run_case(rs, keys, sizes, True)
    finally:
        rs.rsort_segmented_set_split(8192)


def test_lognormal_batch(rs):
    """The batched workload: 4096 lognormal segments (median 2^12, sigma 1.5,
    clipped to [16, 2^20]), uniform 32-bit keys."""
    sizes = keygen.lognormal_sizes(4096)
    n = int(sizes.sum())
    announce("seg lognormal", n)
    keys = keygen.uniform_u32(n, keygen.SEED_SEGMENTS)
    run_case(rs, keys, sizes, False)


def test_offsets_not_starting_at_zero_and_errors(rs):
    import torch
    keys = keygen.uniform_u32(1000, 3)
    off = np.array([100, 300, 300, 900], dtype=np.uint64)
    dk = dev(keys)
    ko = dev(keys.copy())
    rs.rsort_segmented_sort(dk, ko, off)
    got = host(ko)
    want = keys.copy()
    for a, b in zip(off[:-1], off[1:]):
        want[a:b] = np.sort(keys[a:b], kind="stable")
    assert np.array_equal(got, want)
    with pytest.raises(rs.RsortError):
        rs.rsort_segmented_sort(dk, ko, np.array([0, 500, 400], dtype=np.uint64))
    e = torch.empty(0, dtype=torch.uint32, device="cuda")
    rs.rsort_segmented_sort(e, e, np.array([0], dtype=np.uint64))


# ---------------------------------------------------------------------------
# BTN and OET as the sorters of the small segments (32-bit keys, <= 4096 keys;
# other small segments keep the radix rounds): same bit-exact result.

NETWORK_SIZES = [1, 2, 3, 4, 5, 31, 255, 256, 257, 1000, 1023, 1024, 1025, 2048, 3001, 4095,
                 4096, 4097, 8192, 20000, 0, 9]


@pytest.mark.parametrize("sorter", ["btn", "oet"])
@pytest.mark.parametrize("with_vals,in_place", [(True, False), (False, False), (True, True)])
def test_network_small_sorters_u32(rs, sorter, with_vals, in_place):
    n = int(sum(NETWORK_SIZES))
    announce("seg network", sorter, with_vals, in_place)
    keys = keygen.uniform_u32(n, 41)
    keys[::3] = keys[1::3][: keys[::3].size]        # duplicates: ties resolved by position
    rs.rsort_segmented_set_small_sort(sorter)
    try:
        assert rs.rsort_segmented_get_small_sort() == rs.SMALL_SORTS[sorter]
        run_case(rs, keys, NETWORK_SIZES, with_vals, in_place)
        run_case(rs, keygen.zipf_keys(n, 42), NETWORK_SIZES, with_vals, in_place)
    finally:
        rs.rsort_segmented_set_small_sort("radix")


@pytest.mark.parametrize("sorter", ["btn", "oet"])
def test_network_small_sorters_u64_and_device_offsets(rs, sorter):
    """64-bit keys take the radix rounds whatever the setting; the
    device-offset entry point uses the setting too."""
    import torch
    n = int(sum(NETWORK_SIZES))
    announce("seg network u64 / device", sorter)
    rs.rsort_segmented_set_small_sort(sorter)
    try:
        run_case(rs, keygen.uniform_u64(n, 43), NETWORK_SIZES, True)
        keys = keygen.uniform_u32(n, 44)
        vals = np.arange(n, dtype=np.uint32)
        off = keygen.offsets_from_sizes(np.asarray(NETWORK_SIZES))
        doff = torch.from_numpy(off.astype(np.uint32).view(np.int32)).cuda()
        dk, dv = dev(keys), dev(vals)
        ko, vo = torch.empty_like(dk), torch.empty_like(dv)
        rs.rsort_segmented_sort_device(dk, ko, doff, dv, vo)
        rs.rsort_synchronize()
        wk, wv = oracle.segmented(keys, vals, off)
        assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)
    finally:
        rs.rsort_segmented_set_small_sort("radix")
    with pytest.raises(rs.RsortError):
        rs.rsort_segmented_set_small_sort(3)


def test_tuner_picks_a_split_and_stays_exact(rs):
    import torch
    sizes = keygen.lognormal_sizes(512, seed=77)
    off = keygen.offsets_from_sizes(sizes)
    n = int(off[-1])
    announce("seg tune", n)
    keys = keygen.uniform_u32(n, 78)
    dk = dev(keys)
    ko = torch.empty_like(dk)
    split, ms = rs.rsort_segmented_tune(dk, ko, off, reps=2)
    assert split in (0, 1024, 4096, 8192) and ms > 0
    assert rs.rsort_segmented_get_small_sort() in (0, 1, 2)
    cfg = rs.rsort_segmented_get_config()
    assert cfg["split"] == split and cfg["tile_threads"] in (256, 512, 1024)
    assert cfg["radix_bits"] == 8
    rs.rsort_segmented_sort(dk, ko, off)
    want, _ = oracle.segmented(keys, None, off)
    assert np.array_equal(host(ko), want)
    rs.rsort_segmented_set_split(8192)
    rs.rsort_segmented_set_small_sort("radix")
    rs.rsort_segmented_set_tile(0)
    rs.rsort_segmented_set_launch("rounds")


@pytest.mark.parametrize("tile_threads", [256, 512, 1024])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_tile_shapes_exact(rs, tile_threads, dtype):
    """Every tile shape the tuner searches (tiles of 256 / 512 / 1024 threads x
    16 or 8 keys), through the tiled path alone (split 0) and mixed with the
    in-LDS path, with payloads and in place, with per-segment identity
    rounds: bit-exact against the oracle."""
    sizes = [1, 100, 5000, 8192, 8193, 16384, 16385, 30000, 70001, 0, 100003, 4097]
    rs.rsort_segmented_set_tile(tile_threads)
    try:
        assert rs.rsort_segmented_get_config()["tile_threads"] == tile_threads
        for kind in (4, 0, 3):   # uniform, segment-constant high half, all equal
            keys = shaped_segments(kind, sizes, 200 + kind, dtype)
            for split in (0, 8192):
                announce("seg tile", tile_threads, dtype.__name__, kind, split)
                rs.rsort_segmented_set_split(split)
                run_case(rs, keys, sizes, True)
                run_case(rs, keys, sizes, False, in_place=True)
    finally:
        rs.rsort_segmented_set_split(8192)
        rs.rsort_segmented_set_tile(0)
    with pytest.raises(rs.RsortError):
        rs.rsort_segmented_set_tile(384)


def test_graph_capture_replays(rs):
    """The segmented sort captured into a HIP graph: every replay, with eager
    work in between, equals the eager result, and follows new input data."""
    import torch
    sizes = keygen.lognormal_sizes(300, seed=5)
    off = keygen.offsets_from_sizes(sizes)
    n = int(off[-1])
    announce("seg graph", n)
    keys = keygen.uniform_u32(n, 6)
    vals = np.arange(n, dtype=np.uint32)
    dk, dv = dev(keys), dev(vals)
    ko, vo = torch.empty_like(dk), torch.empty_like(dv)
    need = rs.rsort_segmented_workspace_bytes(torch.uint32, True, off)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rs.rsort_segmented_sort(dk, ko, off, dv, vo, workspace=ws)
    torch.cuda.synchronize()
    wk, wv = oracle.segmented(keys, vals, off)
    assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rs.rsort_segmented_sort(dk, ko, off, dv, vo, workspace=ws)
    for rep in range(3):
        ko.view(torch.int32).fill_(rep)
        vo.view(torch.int32).fill_(rep)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(ko), wk), rep
        assert np.array_equal(host(vo), wv), rep
    keys2 = keygen.uniform_u32(n, 7)
    dk.copy_(torch.from_numpy(keys2).cuda())
    g.replay()
    torch.cuda.synchronize()
    assert np.array_equal(host(ko), oracle.segmented(keys2, vals, off)[0])
    # a capture without the preceding identical eager call is refused
    off2 = keygen.offsets_from_sizes(sizes[::-1].copy())
    g2 = torch.cuda.CUDAGraph()
    with pytest.raises(rs.RsortError):
        with torch.cuda.graph(g2):
            rs.rsort_segmented_sort(dk, ko, off2, dv, vo, workspace=ws)


def test_device_offsets_match_and_capture(rs):
    """Offsets in device memory: same result as the host-offset call and the
    oracle; capturable with no preceding eager call; replays follow new data."""
    import torch
    sizes = keygen.lognormal_sizes(700, seed=15)
    sizes[::50] = 0
    off = keygen.offsets_from_sizes(sizes)
    n = int(off[-1]) + 33   # a tail outside every segment stays untouched
    announce("seg device offsets", n)
    keys = keygen.uniform_u32(n, 16)
    vals = np.arange(n, dtype=np.uint32)
    end = int(off[-1])

    def expect(k, v):
        wk, wv = oracle.segmented(k, v, off)
        wk[end:] = k[end:]            # the oracle leaves elements outside segments unset
        if v is not None:
            wv[end:] = v[end:]
        return wk, wv

    wk, wv = expect(keys, vals)
    doff = torch.from_numpy(off.astype(np.int64)).to(torch.int32).cuda()
    dk, dv = dev(keys), dev(vals)
    ko, vo = dev(keys.copy()), dev(vals.copy())
    rs.rsort_segmented_sort_device(dk, ko, doff, dv, vo)
    rs.rsort_synchronize()
    assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)
    need = rs.rsort_segmented_device_workspace_bytes(torch.uint32, True, off.size - 1, n)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rs.rsort_segmented_sort_device(dk, ko, doff, dv, vo, workspace=ws)
    for rep in range(3):
        ko.copy_(dk)
        vo.copy_(dv)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(ko), wk), rep
        assert np.array_equal(host(vo), wv), rep
    keys2 = keygen.zipf_keys(n, 17)
    dk.copy_(dev(keys2))
    ko.copy_(dk)
    g.replay()
    torch.cuda.synchronize()
    assert np.array_equal(host(ko), expect(keys2, vals)[0])
    # u64 keys, keys only
    k64 = keygen.uniform_u64(n, 18)
    d64 = dev(k64)
    o64 = dev(k64.copy())
    rs.rsort_segmented_sort_device(d64, o64, doff)
    rs.rsort_synchronize()
    assert np.array_equal(host(o64), expect(k64, None)[0])


def test_device_offsets_invalid_are_reported(rs):
    """Decreasing offsets, or offsets past the arrays: nothing is written and
    the next synchronize reports a device error."""
    import torch
    n = 5000
    keys = keygen.uniform_u32(n, 21)
    dk = dev(keys)
    for bad in ([0, 3000, 2000, 5000], [0, 1000, 6000]):
        announce("seg device offsets invalid", bad)
        ko = dev(keys.copy())
        doff = torch.tensor(bad, dtype=torch.int32, device="cuda")
        rs.rsort_segmented_sort_device(dk, ko, doff)
        with pytest.raises(rs.RsortError) as e:
            rs.rsort_synchronize()
        assert e.value.status == rs.RSORT_EDEVICE
        assert np.array_equal(host(ko), keys)
    rs.rsort_synchronize()   # the error word was cleared


def shaped_segments(kind, sizes, seed, dtype=np.uint32):
    """Keys whose digits are constant inside a segment in different ways, so
    that segments skip different rounds: a per-segment high half, a constant
    low byte, a constant interior byte, all-equal segments, and uniform ones."""
    parts = []
    for i, s in enumerate(sizes):
        if dtype == np.uint32:
            u = keygen.uniform_u32(int(s), seed + i)
        else:
            u = keygen.uniform_u64(int(s), seed + i)
        k = (i + kind) % 5
        if k == 0:      # only the low 16 bits vary; the rest is the segment's own
            base = dtype(((i * 0x9E3779B1) & 0xFFFF) << 16)
            u = (u & dtype(0xFFFF)) | base
        elif k == 1:    # low byte constant
            u = (u & ~dtype(0xFF)) | dtype(0x5A)
        elif k == 2:    # an interior byte constant
            u = (u & ~dtype(0xFF00)) | dtype(0x3C00)
        elif k == 3:    # all equal
            u = np.full(int(s), u[0] if s else 0, dtype=dtype)
        parts.append(u.astype(dtype))
    return np.concatenate(parts) if parts else np.zeros(0, dtype=dtype)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("with_vals", [False, True])
@pytest.mark.parametrize("in_place", [False, True])
def test_per_segment_identity_rounds(rs, dtype, with_vals, in_place):
    """Large segments skip the rounds whose digit is constant inside them (each
    segment its own plan, ending in the output); bit-exact against the
    oracle, tiled path only (split 0) and mixed with in-LDS segments."""
    sizes = [20000, 8193, 70001, 16384, 30000, 9000, 100003, 5000, 8192, 65536, 12345, 0, 40000]
    for kind in range(5):
        keys = shaped_segments(kind, sizes, 90 + kind, dtype)
        for split in (0, 8192):
            announce("seg identity", dtype.__name__, with_vals, in_place, kind, split)
            rs.rsort_segmented_set_split(split)
            run_case(rs, keys, sizes, with_vals, in_place)
    rs.rsort_segmented_set_split(8192)


@pytest.mark.parametrize("with_vals", [False, True])
def test_per_segment_identity_rounds_device_offsets(rs, with_vals):
    """The same through the device-planned path (offsets in device memory)."""
    import torch
    sizes = [20000, 8193, 70001, 16384, 30000, 9000, 100003, 5000, 8192, 65536, 12345, 0, 40000]
    for kind in range(5):
        keys = shaped_segments(kind, sizes, 120 + kind)
        off = keygen.offsets_from_sizes(np.asarray(sizes))
        n = keys.size
        vals = np.arange(n, dtype=np.uint32)
        announce("seg identity device", with_vals, kind)
        wk, wv = oracle.segmented(keys, vals if with_vals else None, off)
        dk = dev(keys)
        dv = dev(vals) if with_vals else None
        ko = torch.empty_like(dk)
        vo = torch.empty_like(dv) if with_vals else None
        doff = dev(off.astype(np.uint32))
        rs.rsort_segmented_sort_device(dk, ko, doff, dv, vo)
        rs.rsort_synchronize()
        assert np.array_equal(host(ko), wk)
        if with_vals:
            assert np.array_equal(host(vo), wv)
