"""GPU parity of the radix-2^8 LSD path (PR4) against the CPU oracle.

Every comparison is bit-exact: the stable sort is unique, and so are the digit
counts.  Sizes span one to many tiles with ragged tails (a tile is 8192 uint32
or 4096 uint64 keys), all six key distributions, keys-only and key-value,
in-place and out-of-place, partial bit ranges and repeated runs.
"""
import numpy as np
import pytest

import keygen
import oracle
from tests.gpu_util import announce, check_kv_invariants, dev, host

pytestmark = pytest.mark.gpu

# One to a few hundred 8192-key tiles, ragged tails, powers of two; 2^21 keys
# (256 tiles) is the largest sort whose scatter sums the tile counts itself,
# 2^21 + 1 the smallest with the tile-scan kernel.
SIZES = [1, 2, 63, 64, 65, 1000, 2047, 2048, 2049, 8191, 8192, 8193, 3 * 8192 + 17, 100003,
         1 << 20, 1 << 21, (1 << 21) + 1, 3 * (1 << 20) + 4097]


@pytest.fixture(scope="module")
def rs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1808_10292_amd import rsort
    rsort.load_library()
    return rsort


@pytest.mark.parametrize("dist", keygen.KV_DISTRIBUTIONS)
def test_histogram_8bit_matches_oracle(rs, dist):
    for n in (1, 8193, 300001):
        announce("hist8", dist, n)
        keys = keygen.kv_keys(dist, n)
        got = host(rs.rsort_histogram(dev(keys), 8)).astype(np.uint64)
        for d in range(4):
            assert np.array_equal(got[d], oracle.digit_counts(keys, 8 * d, 8)), (dist, n, d)


def test_histogram_16bit_and_ranges(rs):
    keys = keygen.zipf_keys(250001, 3)
    announce("hist16")
    got = host(rs.rsort_histogram(dev(keys), 16)).astype(np.uint64)
    for d in range(2):
        assert np.array_equal(got[d], oracle.digit_counts(keys, 16 * d, 16))
    got = host(rs.rsort_histogram(dev(keys), 8, 5, 27)).astype(np.uint64)
    assert got.shape[0] == 3
    assert np.array_equal(got[0], oracle.digit_counts(keys, 5, 8))
    assert np.array_equal(got[2][:64], oracle.digit_counts(keys, 21, 6))
    k64 = keygen.uniform_u64(70001, 4)
    got = host(rs.rsort_histogram(dev(k64), 8)).astype(np.uint64)
    for d in range(8):
        assert np.array_equal(got[d], oracle.digit_counts(k64, 8 * d, 8))


@pytest.mark.parametrize("n", SIZES)
def test_keys_only_sizes(rs, n):
    announce("keys u32", n)
    keys = keygen.uniform_u32(n, 100 + n)
    ko, _ = rs.sort(dev(keys))
    want, _ = oracle.sr4(keys)
    assert np.array_equal(host(ko), want)


@pytest.mark.parametrize("n", [200003, 2500009])
@pytest.mark.parametrize("dist", keygen.KV_DISTRIBUTIONS)
def test_kv_distributions(rs, dist, n):
    announce("kv u32", dist, n)
    keys = keygen.kv_keys(dist, n)
    vals = np.arange(n, dtype=np.uint32)
    ko, vo = rs.sort(dev(keys), dev(vals))
    ko, vo = host(ko), host(vo)
    wk, wv = oracle.sr4(keys, vals)
    assert np.array_equal(ko, wk) and np.array_equal(vo, wv)
    check_kv_invariants(keys, ko, vo)


@pytest.mark.parametrize("n", [5, 4096, 4097, 77777])
def test_u64_keys(rs, n):
    announce("u64", n)
    keys = keygen.uniform_u64(n, 7 + n)
    keys[::5] = keys[1]
    vals = np.arange(n, dtype=np.uint32)
    ko, vo = rs.sort(dev(keys), dev(vals))
    wk, wv = oracle.sr4(keys, vals)
    assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)
    ko, _ = rs.sort(dev(keys))
    assert np.array_equal(host(ko), wk)


@pytest.mark.parametrize("d", [0, 1, 2, 3])
def test_state_after_each_round(rs, d):
    """Sorting on [0, 8(d+1)) is the array after round d (oracle's round-d state)."""
    n = 50001
    announce("round", d)
    keys = keygen.uniform_u32(n, 55)
    vals = np.arange(n, dtype=np.uint32)
    ko, vo = rs.sort(dev(keys), dev(vals), end_bit=8 * (d + 1))
    wk, wv = oracle.lsd_sort(keys, vals, 8, 0, 8 * (d + 1))
    assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)


@pytest.mark.parametrize("lo,hi", [(0, 24), (4, 28), (3, 10), (16, 32), (0, 0), (31, 32)])
def test_bit_ranges_in_and_out_of_place(rs, lo, hi):
    import torch
    n = 30011
    announce("bits", lo, hi)
    keys = keygen.zipf_keys(n, 5)
    vals = np.arange(n, dtype=np.uint32)
    wk, wv = oracle.lsd_sort(keys, vals, 8, lo, hi)
    ko, vo = rs.sort(dev(keys), dev(vals), begin_bit=lo, end_bit=hi)
    assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)
    k, v = dev(keys), dev(vals)
    rs.rsort_sort(k, k, v, v, lo, hi)
    torch.cuda.synchronize()
    assert np.array_equal(host(k), wk) and np.array_equal(host(v), wv)


@pytest.mark.parametrize("dist", ["low16", "equal", "presorted", "reverse"])
def test_in_place_with_identity_rounds(rs, dist):
    """Identity rounds are skipped; in place the running count is made even."""
    n = 65537
    announce("inplace", dist)
    keys = keygen.kv_keys(dist, n)
    vals = np.arange(n, dtype=np.uint32)
    wk, wv = oracle.sr4(keys, vals)
    k, v = dev(keys), dev(vals)
    rs.rsort_sort(k, k, v, v)
    assert np.array_equal(host(k), wk) and np.array_equal(host(v), wv)
    k = dev(keys)
    rs.rsort_sort(k, k)
    assert np.array_equal(host(k), wk)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("tile", [0, 1, 63, 64, 100, 129])
def test_one_key_differs(rs, dtype, tile):
    """All keys equal but one, in the given tile: only that tile's workgroup
    sees a difference, so the round plan must take it from wherever round 0's
    count recorded it; every other round is the identity."""
    tile_keys = 8192 if dtype == np.uint32 else 4096
    n = 129 * tile_keys + 5              # the last tile holds 5 keys
    announce("one-differs", np.dtype(dtype).name, tile)
    same = dtype(0x5A5A5A5A) if dtype == np.uint32 else dtype(0x5A5A5A5A5A5A5A5A)
    keys = np.full(n, same, dtype=dtype)
    pos = min(tile * tile_keys + 3, n - 1)
    keys[pos] = same - dtype(0x00010000)     # differs in the third digit, sorts first
    vals = np.arange(n, dtype=np.uint32)
    wk, wv = oracle.sr4(keys, vals)
    assert wk[0] == keys[pos] and wv[0] == pos
    ko, vo = rs.sort(dev(keys), dev(vals))
    assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)
    k = dev(keys)
    rs.rsort_sort(k, k)
    assert np.array_equal(host(k), wk)


def test_repeatable(rs):
    n = (1 << 20) + 3
    keys = keygen.zipf_keys(n, 77)
    vals = np.arange(n, dtype=np.uint32)
    announce("repeat")
    dk, dv = dev(keys), dev(vals)
    first = None
    for _ in range(5):
        ko, vo = rs.sort(dk, dv)
        cur = (host(ko), host(vo))
        if first is None:
            first = cur
            wk, wv = oracle.sr4(keys, vals)
            assert np.array_equal(cur[0], wk) and np.array_equal(cur[1], wv)
        else:
            assert np.array_equal(cur[0], first[0]) and np.array_equal(cur[1], first[1])
    rs.rsort_synchronize()


def test_caller_workspace(rs):
    import torch
    n = 123457
    keys = keygen.uniform_u32(n, 9)
    need = rs.rsort_workspace_bytes(torch.uint32, False, n)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    announce("caller workspace", need)
    ko = torch.empty(n, dtype=torch.uint32, device="cuda")
    rs.rsort_sort(dev(keys), ko, workspace=ws)
    assert np.array_equal(host(ko), oracle.sr4(keys)[0])
    with pytest.raises(rs.RsortError):
        rs.rsort_sort(dev(keys), ko, workspace=ws[: need // 2])


def test_argument_errors(rs):
    import torch
    k = dev(keygen.uniform_u32(1000, 1))
    with pytest.raises(rs.RsortError):
        rs.rsort_sort(k, torch.empty(1000, dtype=torch.uint32, device="cuda"), begin_bit=4, end_bit=40)
    # partial overlap of input and output
    big = torch.zeros(2000, dtype=torch.uint32, device="cuda")
    with pytest.raises(rs.RsortError):
        rs.rsort_sort(big[:1000], big[500:1500])
    # n = 0 is a no-op
    e = torch.empty(0, dtype=torch.uint32, device="cuda")
    rs.rsort_sort(e, e)
    rs.rsort_synchronize()


def test_profile_counts_and_period(rs):
    """Kernel timing: every round launch of a 4-round sort is timed; with a
    period of 5 only launches 0, 5, 10, ... of the kind are; period 0 and a
    disabled profiler are errors."""
    import torch
    announce("profiler")
    keys = keygen.uniform_u32(1 << 20, 41)
    dk = dev(keys)
    out = torch.empty_like(dk)
    rs.rsort_profile_enable(True, kinds=[rs.RSORT_KERNEL_ROUND])
    for _ in range(3):
        rs.rsort_sort(dk, out, algo="lsd8")
    launches, ms = rs.rsort_profile_read(rs.RSORT_KERNEL_ROUND)
    assert launches == 12 and ms > 0
    assert rs.rsort_profile_read(rs.RSORT_KERNEL_COUNT) == (0, 0.0)   # kind not timed
    rs.rsort_profile_enable(True, kinds=[rs.RSORT_KERNEL_ROUND])
    rs.rsort_profile_set_period(5)
    for _ in range(6):
        rs.rsort_sort(dk, out, algo="lsd8")
    launches, ms = rs.rsort_profile_read(rs.RSORT_KERNEL_ROUND)
    assert launches == 5 and ms > 0                                   # 0, 5, 10, 15, 20 of 24
    with pytest.raises(rs.RsortError):
        rs.rsort_profile_set_period(0)
    rs.rsort_profile_enable(False)
    with pytest.raises(rs.RsortError):
        rs.rsort_profile_set_period(2)
    rs.rsort_synchronize()
    assert np.array_equal(host(out), np.sort(keys))


@pytest.mark.slow
def test_full_size_2p27_keys_only(rs):
    """The benchmark workload itself: 2^27 uniform 32-bit keys, bit-exact."""
    n = 1 << 27
    announce("2^27 keys")
    keys = keygen.uniform_u32(n, keygen.SEED_LARGE)
    ko, _ = rs.sort(dev(keys))
    got = host(ko)
    want, _ = oracle.sr4(keys)
    assert np.array_equal(got, want)
    rs.rsort_synchronize()


def test_graph_capture_replays(rs):
    """The plain sort enqueues kernels only: captured once into a HIP graph,
    every replay (with eager work between) equals the eager result and follows
    new input data."""
    import torch
    n = (1 << 20) + 77
    announce("graph", n)
    keys = keygen.zipf_keys(n, 19)
    vals = np.arange(n, dtype=np.uint32)
    dk, dv = dev(keys), dev(vals)
    ko, vo = torch.empty_like(dk), torch.empty_like(dv)
    need = rs.rsort_workspace_bytes(torch.uint32, True, n)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rs.rsort_sort(dk, ko, dv, vo, workspace=ws)
    torch.cuda.synchronize()
    wk, wv = oracle.sr4(keys, vals)
    assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rs.rsort_sort(dk, ko, dv, vo, workspace=ws)
    for rep in range(3):
        ko.view(torch.int32).fill_(rep)
        vo.view(torch.int32).fill_(rep)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(ko), wk), rep
        assert np.array_equal(host(vo), wv), rep
    keys2 = keygen.uniform_u32(n, 20)
    dk.copy_(dev(keys2))
    g.replay()
    torch.cuda.synchronize()
    assert np.array_equal(host(ko), oracle.sr4(keys2)[0])


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("case", ["equal", "range_agrees", "one_round"])
@pytest.mark.parametrize("alias", ["vals", "keys"])
def test_one_array_in_place(rs, dtype, case, alias):
    """Only one of keys / payloads sorted in place (keys_in != keys_out but
    vals_in == vals_out, or the reverse), also when every round is the
    identity: the array that is not its own input must still be written."""
    import torch
    n = 3 * 8192 + 11
    announce("one array in place", np.dtype(dtype).name, case, alias)
    keys = keygen.uniform_u32(n, 91).astype(dtype)
    lo, hi = 0, 8 * keys.itemsize
    if case == "equal":
        keys[:] = keys[0]
    elif case == "range_agrees":
        keys = (keys & dtype(0xFF)) | dtype(0xA500)     # bits [8, 24) agree
        lo, hi = 8, 24
    else:
        keys = keys & dtype(0xFF)                        # one running round
    vals = np.arange(n, dtype=np.uint32)
    wk, wv = oracle.lsd_sort(keys, vals, 8, lo, hi)
    k, v = dev(keys), dev(vals)
    if alias == "vals":
        ko = torch.empty_like(k)
        rs.rsort_sort(k, ko, v, v, lo, hi)
        vo = v
    else:
        vo = torch.empty_like(v)
        rs.rsort_sort(k, k, v, vo, lo, hi)
        ko = k
    rs.rsort_synchronize()
    assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)


@pytest.mark.parametrize("dist", ["uniform", "zipf", "presorted"])
def test_kv_2p21_pairs_xcd_sliced_tiles(rs, dist):
    """2^21 pairs = 256 tiles, a multiple of 8: the scatter deals the tiles to
    the XCDs in contiguous slices, which the other key-value sizes here do not
    reach; bit-exact against the oracle."""
    n = 1 << 21
    announce("kv 2^21", dist)
    keys = keygen.kv_keys(dist, n, 77)
    vals = np.arange(n, dtype=np.uint32)
    ko, vo = rs.sort(dev(keys), dev(vals))
    wk, wv = oracle.sr4(keys, vals)
    assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)


@pytest.mark.slow
@pytest.mark.parametrize("dist", keygen.KV_DISTRIBUTIONS)
def test_full_size_kv_pr4(rs, dist):
    """The key-value workload at full size through PR4: 2^28 (key, input index)
    pairs per distribution.  The four invariants of check_kv_invariants
    determine the stable sort uniquely, so they stand in for the oracle at this
    size."""
    import torch
    n = 1 << 28
    announce("pr4 kv full", dist, n)
    keys = keygen.kv_keys(dist, n)
    dk = dev(keys)
    dv = torch.arange(n, dtype=torch.int32, device="cuda")
    ko, vo = torch.empty_like(dk), torch.empty_like(dv)
    rs.rsort_sort(dk, ko, dv, vo, algo="lsd8")
    rs.rsort_synchronize()
    del dk, dv
    check_kv_invariants(keys, host(ko), host(vo).view(np.uint32))


@pytest.mark.parametrize("dtype,n", [(np.uint32, 1 << 20), (np.uint32, (1 << 20) + 1),
                                     (np.uint32, 1 << 21), (np.uint32, (1 << 21) + 1),
                                     (np.uint64, 1 << 20), (np.uint64, (1 << 20) + 1)])
@pytest.mark.parametrize("in_place", [False, True])
def test_tile_shape_and_inline_scan_limits(rs, dtype, n, in_place):
    """Both sides of each size limit of the few-tile forms: 32-bit sorts of at
    most 2^20 keys (4096-key tiles), at most 256 tiles (no tile-scan kernel,
    16-bit tile counts summed by every scatter workgroup), and the tile-scan
    form beyond; with payloads, in and out of place, against the oracle."""
    import torch
    announce("tile limits", np.dtype(dtype).name, n, in_place)
    keys = (keygen.uniform_u32(n, 300 + n) if dtype == np.uint32
            else keygen.uniform_u64(n, 300 + n))
    keys[::9] = keys[4]                       # runs of equal keys across tiles
    vals = np.arange(n, dtype=np.uint32)
    wk, wv = oracle.sr4(keys, vals)
    dk, dv = dev(keys), dev(vals)
    if in_place:
        rs.rsort_sort(dk, dk, dv, dv)
        ko, vo = dk, dv
    else:
        ko, vo = torch.empty_like(dk), torch.empty_like(dv)
        rs.rsort_sort(dk, ko, dv, vo)
    rs.rsort_synchronize()
    assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)
