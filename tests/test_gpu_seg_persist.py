"""GPU parity of the segmented sort's persistent launch (RSORT_SEG_PERSISTENT:
one cooperative launch, phases separated by grid-wide barriers) against the
oracle's per-segment SR4, bit-exact.

The cases reach every phase: whole small segments of both in-LDS forms, tiles
of large segments (one tile, ragged last tiles, hundreds of tiles per
segment), empty and one-key segments, segments whose rounds are skipped
(per-segment plans, including all-equal segments that are copied), u32 / u64
keys, payloads, in place, the all-tiled split, the lognormal 4096-segment
batch, repeated launches, the refusal inside a graph capture, and the tuner
choosing between the launch modes.
"""
import numpy as np
import pytest

import keygen
import oracle
from tests.gpu_util import announce, dev, host
from tests.test_gpu_segmented import BOUNDARY_SIZES, run_case, shaped_segments

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1808_10292_amd import rsort
    rsort.load_library()
    rsort.rsort_segmented_set_launch("persistent")
    yield rsort
    rsort.rsort_segmented_set_launch("rounds")
    rsort.rsort_segmented_set_split(8192)
    rsort.rsort_segmented_set_tile(0)


def test_config_reports_persistent(rs):
    cfg = rs.rsort_segmented_get_config()
    assert cfg["launch"] == "persistent" and cfg["tile_threads"] == 512
    assert cfg["small_sort"] == "radix" and cfg["radix_bits"] == 8
    with pytest.raises(rs.RsortError):
        rs.rsort_segmented_set_launch(2)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("with_vals", [False, True])
def test_boundary_sizes(rs, dtype, with_vals):
    n = int(sum(BOUNDARY_SIZES))
    announce("persist boundaries", dtype.__name__, with_vals)
    keys = keygen.uniform_u32(n, 51) if dtype == np.uint32 else keygen.uniform_u64(n, 52)
    keys[::7] = keys[3]
    run_case(rs, keys, BOUNDARY_SIZES, with_vals)


@pytest.mark.parametrize("dist", keygen.KV_DISTRIBUTIONS)
def test_distributions(rs, dist):
    sizes = [3000, 9000, 700, 20000, 8192, 1, 300001, 0, 65537]
    announce("persist dist", dist)
    keys = keygen.kv_keys(dist, int(sum(sizes)))
    run_case(rs, keys, sizes, True)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("with_vals", [False, True])
@pytest.mark.parametrize("in_place", [False, True])
def test_per_segment_plans(rs, dtype, with_vals, in_place):
    """Segments that skip different rounds (constant high half, low byte,
    interior byte, all equal), all tiled (split 0) and mixed with small ones."""
    sizes = [20000, 8193, 70001, 16384, 30000, 9000, 100003, 5000, 8192, 65536, 12345, 0, 40000]
    try:
        for kind in range(5):
            keys = shaped_segments(kind, sizes, 190 + kind, dtype)
            for split in (0, 8192):
                announce("persist plans", dtype.__name__, with_vals, in_place, kind, split)
                rs.rsort_segmented_set_split(split)
                run_case(rs, keys, sizes, with_vals, in_place)
    finally:
        rs.rsort_segmented_set_split(8192)


def test_long_chains(rs):
    """A few segments of hundreds of tiles: long look-back chains, many
    workgroups waiting on the same segment's rounds."""
    sizes = [3 * (1 << 20) + 11, 5, (1 << 21) + 4097, 1 << 20]
    n = int(sum(sizes))
    announce("persist long chains", n)
    keys = keygen.uniform_u32(n, 61)
    run_case(rs, keys, sizes, True)
    run_case(rs, keygen.zipf_keys(n, 62), sizes, False, in_place=True)


def test_lognormal_batch(rs):
    """The batched workload: 4096 lognormal segments (median 2^12, sigma 1.5,
    clipped to [16, 2^20]), uniform 32-bit keys."""
    sizes = keygen.lognormal_sizes(4096)
    n = int(sizes.sum())
    announce("persist lognormal", n)
    keys = keygen.uniform_u32(n, keygen.SEED_SEGMENTS)
    run_case(rs, keys, sizes, False)


def test_repeat_and_capture_refused(rs):
    """Twenty launches in a row give the same result; a graph capture of the
    persistent launch is refused (it is a cooperative launch)."""
    import torch
    sizes = keygen.lognormal_sizes(300, seed=5)
    off = keygen.offsets_from_sizes(sizes)
    n = int(off[-1])
    keys = keygen.uniform_u32(n, 63)
    want, _ = oracle.segmented(keys, None, off)
    dk = dev(keys)
    ko = torch.empty_like(dk)
    announce("persist repeat", n)
    for r in range(20):
        ko.fill_(0)
        rs.rsort_segmented_sort(dk, ko, off)
        rs.rsort_synchronize()
        assert np.array_equal(host(ko), want), r
    need = rs.rsort_segmented_workspace_bytes(torch.uint32, False, off)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rs.rsort_segmented_sort(dk, ko, off, workspace=ws)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(rs.RsortError) as e:
        with torch.cuda.graph(g):
            rs.rsort_segmented_sort(dk, ko, off, workspace=ws)
    assert e.value.status == rs.RSORT_EUNSUPPORTED
    torch.cuda.synchronize()
    rs.rsort_segmented_sort(dk, ko, off)
    rs.rsort_synchronize()
    assert np.array_equal(host(ko), want)


def test_tuner_searches_launch_modes(rs):
    import torch
    sizes = keygen.lognormal_sizes(512, seed=79)
    off = keygen.offsets_from_sizes(sizes)
    n = int(off[-1])
    keys = keygen.uniform_u32(n, 80)
    dk = dev(keys)
    ko = torch.empty_like(dk)
    announce("persist tune", n)
    try:
        split, ms = rs.rsort_segmented_tune(dk, ko, off, reps=2)
        cfg = rs.rsort_segmented_get_config()
        assert cfg["launch"] in ("rounds", "persistent") and ms > 0
        rs.rsort_segmented_sort(dk, ko, off)
        want, _ = oracle.segmented(keys, None, off)
        assert np.array_equal(host(ko), want)
    finally:
        rs.rsort_segmented_set_launch("persistent")
        rs.rsort_segmented_set_split(8192)
        rs.rsort_segmented_set_small_sort("radix")
        rs.rsort_segmented_set_tile(0)
