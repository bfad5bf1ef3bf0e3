"""Repeat stress: each sort path run 20 times in a row over grids of
different sizes (tile counts that are and are not multiples of the 8 XCD
slices, one partial tile, hundreds of tiles) and, for the segmented sort, each
tile workgroup shape.  Every repeat must equal the oracle bit for bit; the test
stops at the first repeat that differs and names it."""
import numpy as np
import pytest

import keygen
import oracle
from tests.gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu

REPEATS = 20
# 8192-key tiles: 1, 7, 8, 9, 64, 257 (+ a ragged tail) and 1029 tiles
SIZES = [5000, 7 * 8192 + 3, 8 * 8192, 9 * 8192 + 1, 64 * 8192, 257 * 8192 + 4095,
         1029 * 8192 + 17]


@pytest.fixture(scope="module")
def rs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1808_10292_amd import rsort
    rsort.load_library()
    yield rsort
    rsort.rsort_set_pr4_rounds("counted")
    rsort.rsort_segmented_set_tile(0)


def repeat_sort(rs, keys, vals, algo, tag):
    import torch
    wk, wv = oracle.sr4(keys, vals) if algo != "lsd16" else oracle.lsd_sort(keys, vals, 16)
    dk, dv = dev(keys), dev(vals)
    ko, vo = torch.empty_like(dk), torch.empty_like(dv)
    for r in range(REPEATS):
        ko.fill_(0)
        vo.fill_(0)
        rs.rsort_sort(dk, ko, dv, vo, algo=algo)
        rs.rsort_synchronize()
        assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv), \
            "%s: repeat %d of %d differs" % (tag, r, REPEATS)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("rounds", ["counted", "single_read"])
def test_pr4_repeats(rs, rounds, n):
    announce("stress pr4", rounds, n)
    rs.rsort_set_pr4_rounds(rounds)
    try:
        keys = keygen.kv_keys("zipf" if n % 2 else "uniform", n, 90 + n)
        repeat_sort(rs, keys, np.arange(n, dtype=np.uint32), "lsd8", "pr4 %s n=%d" % (rounds, n))
    finally:
        rs.rsort_set_pr4_rounds("counted")


@pytest.mark.parametrize("n", [SIZES[1], SIZES[5]])
def test_pr2_repeats(rs, n):
    announce("stress pr2", n)
    keys = keygen.uniform_u32(n, 91 + n)
    repeat_sort(rs, keys, np.arange(n, dtype=np.uint32), "lsd16", "pr2 n=%d" % n)


@pytest.mark.parametrize("tile_threads", [256, 512, 1024])
def test_segmented_repeats(rs, tile_threads):
    import torch
    sizes = keygen.lognormal_sizes(300, seed=tile_threads)
    off = keygen.offsets_from_sizes(sizes)
    n = int(off[-1])
    keys = keygen.uniform_u32(n, 92)
    vals = np.arange(n, dtype=np.uint32)
    wk, wv = oracle.segmented(keys, vals, off)
    rs.rsort_segmented_set_tile(tile_threads)
    try:
        dk, dv = dev(keys), dev(vals)
        ko, vo = torch.empty_like(dk), torch.empty_like(dv)
        announce("stress segmented", tile_threads)
        for r in range(REPEATS):
            ko.fill_(0)
            rs.rsort_segmented_sort(dk, ko, off, dv, vo)
            rs.rsort_synchronize()
            assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv), \
                "segmented tile %d: repeat %d differs" % (tile_threads, r)
    finally:
        rs.rsort_segmented_set_tile(0)
