"""GPU parity of the single-read PR4 rounds (RSORT_PR4_SINGLE_READ) against the
CPU oracle, bit-exact.

The single-read rounds split the tiles of each round into chains: the counting
pass's chunks for the first round that runs, the ranges sharing the top four
bits of the previous digit for a round that follows a round that ran, and one
chain for a round that follows a skipped one.  The cases below reach every
kind: uniform keys (chunk then joint chains), a constant low byte (the first
round that runs is round 1, chunk chains over digit 1), a constant interior
byte (a single chain after a skipped round), partial bit ranges, in-place
sorts with an odd number of running rounds, payloads, and sizes from one key to
hundreds of tiles with ragged chunk and chain ends.
"""
import numpy as np
import pytest

import keygen
import oracle
from tests.gpu_util import announce, check_kv_invariants, dev, host

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 100, 8191, 8192, 8193, 65537, 100003, (1 << 20) + 17, 3 * (1 << 21) + 5]


@pytest.fixture(scope="module")
def rs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1808_10292_amd import rsort
    rsort.load_library()
    rsort.rsort_set_pr4_rounds("single_read")
    yield rsort
    rsort.rsort_set_pr4_rounds("counted")


def shaped(name, n, seed):
    u = keygen.uniform_u32(n, seed)
    if name == "uniform":
        return u
    if name == "low_byte_constant":
        return (u << np.uint32(8)) | np.uint32(0x5A)
    if name == "low_half_constant":
        return (u << np.uint32(16)) | np.uint32(0x5A5A)
    if name == "interior_byte_constant":
        return (u & np.uint32(0xFFFF00FF)) | np.uint32(0x3C00)
    if name == "small_range":
        return u & np.uint32(0xFF)
    return keygen.kv_keys(name, n, seed)


SHAPES = ["uniform", "low_byte_constant", "low_half_constant", "interior_byte_constant",
          "small_range"] + [d for d in keygen.KV_DISTRIBUTIONS if d != "uniform"]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("shape", SHAPES)
def test_keys_and_pairs(rs, shape, n):
    announce("single-read", shape, n)
    keys = shaped(shape, n, 7 + n)
    want, _ = oracle.sr4(keys)
    ko, _ = rs.sort(dev(keys), key_type="u32")
    assert np.array_equal(host(ko), want)
    vals = np.arange(n, dtype=np.uint32)
    ko, vo = rs.sort(dev(keys), dev(vals), key_type="u32")
    wk, wv = oracle.sr4(keys, vals)
    ko, vo = host(ko), host(vo)
    assert np.array_equal(ko, wk) and np.array_equal(vo, wv)
    check_kv_invariants(keys, ko, vo)


@pytest.mark.parametrize("shape", ["uniform", "low_byte_constant", "equal", "low16"])
def test_in_place(rs, shape):
    n = (1 << 20) + 33
    keys = shaped(shape, n, 3)
    vals = np.arange(n, dtype=np.uint32)
    wk, wv = oracle.sr4(keys, vals)
    for mode in ("both", "keys", "vals"):
        announce("single-read in place", shape, mode)
        dk, dv = dev(keys), dev(vals)
        ko = dk if mode in ("both", "keys") else dev(np.zeros_like(keys))
        vo = dv if mode in ("both", "vals") else dev(np.zeros_like(vals))
        rs.rsort_sort(dk, ko, dv, vo, key_type="u32")
        assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv), mode


@pytest.mark.parametrize("bits", [(4, 28), (0, 12), (8, 32), (3, 30), (0, 8), (24, 32)])
def test_bit_ranges(rs, bits):
    b, e = bits
    n = (1 << 20) + 5
    keys = keygen.uniform_u32(n, 11)
    announce("single-read bits", b, e)
    ko = dev(np.zeros_like(keys))
    rs.rsort_sort(dev(keys), ko, begin_bit=b, end_bit=e, key_type="u32")
    mask = np.uint32(((1 << (e - b)) - 1) << b)
    field = (keys & mask) >> np.uint32(b)
    # a stable sort on the field: the oracle sorts the field values, then the
    # keys are gathered by a second stable sort of (field, index) pairs
    _, order = oracle.sr4(field, np.arange(n, dtype=np.uint32))
    assert np.array_equal(host(ko), keys[order])


def test_u64_keys_fall_back(rs):
    n = 70001
    keys = keygen.uniform_u64(n, 5)
    announce("single-read u64 fallback")
    ko, _ = rs.sort(dev(keys))
    want, _ = oracle.sr4(keys)
    assert np.array_equal(host(ko), want)


def test_full_size_keys(rs):
    """2^27 uniform keys: the headline size, every chunk and chain full."""
    n = 1 << 27
    keys = keygen.uniform_u32(n, keygen.SEED_LARGE)
    announce("single-read 2^27")
    ko, _ = rs.sort(dev(keys), key_type="u32")
    got = host(ko)
    assert np.all(got[1:] >= got[:-1])
    want, _ = oracle.sr4(keys)
    assert np.array_equal(got, want)
