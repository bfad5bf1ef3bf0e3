"""GPU parity of the radix-2^16 LSD path (PR2) against the CPU oracle.

The oracle's LSD sort with 16-bit digits is the serial form of PR2's rounds;
every comparison is bit-exact.  Sizes span one tile (8192 uint32 / 4096 uint64
keys) to many chunks (up to 256 chunks, ragged last chunk and tile), all six
key distributions, keys only and with payloads, 64-bit keys (four rounds),
partial bit ranges (narrow last digit, an odd number of rounds in place), the
state after the first round, and the full benchmark size.
"""
import numpy as np
import pytest

import keygen
import oracle
from tests.gpu_util import announce, check_kv_invariants, dev, host

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 63, 1000, 8191, 8192, 8193, 3 * 8192 + 17, 100003, 1 << 20, 3000017]


@pytest.fixture(scope="module")
def rs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1808_10292_amd import rsort
    rsort.load_library()
    return rsort


@pytest.mark.parametrize("n", SIZES)
def test_keys_only_sizes(rs, n):
    announce("pr2 keys", n)
    keys = keygen.uniform_u32(n, 300 + n)
    ko, _ = rs.sort(dev(keys), algo="lsd16")
    want, _ = oracle.lsd_sort(keys, None, 16)
    assert np.array_equal(host(ko), want)


@pytest.mark.parametrize("dist", keygen.KV_DISTRIBUTIONS)
def test_kv_distributions(rs, dist):
    n = 1000003
    announce("pr2 kv", dist, n)
    keys = keygen.kv_keys(dist, n)
    vals = np.arange(n, dtype=np.uint32)
    ko, vo = rs.sort(dev(keys), dev(vals), algo="lsd16")
    ko, vo = host(ko), host(vo)
    wk, wv = oracle.lsd_sort(keys, vals, 16)
    assert np.array_equal(ko, wk) and np.array_equal(vo, wv)
    # the same array as PR4 (the stable sort is unique)
    k8, v8 = oracle.sr4(keys, vals)
    assert np.array_equal(ko, k8) and np.array_equal(vo, v8)
    check_kv_invariants(keys, ko, vo)


@pytest.mark.parametrize("n", [5, 4096, 4097, 300007])
def test_u64_keys(rs, n):
    announce("pr2 u64", n)
    keys = keygen.uniform_u64(n, 17 + n)
    keys[::7] = keys[2]
    vals = np.arange(n, dtype=np.uint32)
    ko, vo = rs.sort(dev(keys), dev(vals), algo="lsd16")
    wk, wv = oracle.lsd_sort(keys, vals, 16)
    assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)
    ko, _ = rs.sort(dev(keys), algo="lsd16")
    assert np.array_equal(host(ko), wk)


def test_state_after_first_round(rs):
    """Sorting on [0, 16) is the array after PR2's first round."""
    n = 250001
    announce("pr2 round 0")
    keys = keygen.uniform_u32(n, 56)
    vals = np.arange(n, dtype=np.uint32)
    ko, vo = rs.sort(dev(keys), dev(vals), algo="lsd16", end_bit=16)
    wk, wv = oracle.lsd_sort(keys, vals, 16, 0, 16)
    assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)


@pytest.mark.parametrize("lo,hi", [(0, 24), (4, 28), (3, 10), (16, 32), (0, 0), (31, 32),
                                   (0, 40)])
def test_bit_ranges_in_and_out_of_place(rs, lo, hi):
    import torch
    n = 70001
    announce("pr2 bits", lo, hi)
    keys = keygen.zipf_keys(n, 6) if hi <= 32 else keygen.uniform_u64(n, 6)
    vals = np.arange(n, dtype=np.uint32)
    wk, wv = oracle.lsd_sort(keys, vals, 16, lo, hi)
    ko, vo = rs.sort(dev(keys), dev(vals), algo="lsd16", begin_bit=lo, end_bit=hi)
    assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)
    k, v = dev(keys), dev(vals)
    rs.rsort_sort(k, k, v, v, lo, hi, algo="lsd16")
    torch.cuda.synchronize()
    assert np.array_equal(host(k), wk) and np.array_equal(host(v), wv)



@pytest.mark.parametrize("lo,hi", [(0, 16), (8, 24), (0, 48)])
@pytest.mark.parametrize("alias", ["vals", "keys"])
def test_one_array_in_place_odd_rounds(rs, lo, hi, alias):
    """An odd number of 16-bit rounds with only the payloads (or only the
    keys) sorted in place: round 0 must not read and write the same array."""
    import torch
    n = 70001
    announce("pr2 one array in place", lo, hi, alias)
    keys = keygen.zipf_keys(n, 8) if hi <= 32 else keygen.uniform_u64(n, 8)
    vals = np.arange(n, dtype=np.uint32)
    wk, wv = oracle.lsd_sort(keys, vals, 16, lo, hi)
    k, v = dev(keys), dev(vals)
    if alias == "vals":
        ko = torch.empty_like(k)
        rs.rsort_sort(k, ko, v, v, lo, hi, algo="lsd16")
        vo = v
    else:
        vo = torch.empty_like(v)
        rs.rsort_sort(k, k, v, vo, lo, hi, algo="lsd16")
        ko = k
    rs.rsort_synchronize()
    assert np.array_equal(host(ko), wk) and np.array_equal(host(vo), wv)

def test_caller_workspace_and_repeat(rs):
    import torch
    n = 523459
    keys = keygen.zipf_keys(n, 10)
    need = rs.rsort_workspace_bytes(torch.uint32, False, n, algo="lsd16")
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    announce("pr2 workspace", need)
    dk = dev(keys)
    ko = torch.empty_like(dk)
    want = oracle.lsd_sort(keys, None, 16)[0]
    for _ in range(3):
        rs.rsort_sort(dk, ko, algo="lsd16", workspace=ws)
        assert np.array_equal(host(ko), want)
    with pytest.raises(rs.RsortError):
        rs.rsort_sort(dk, ko, algo="lsd16", workspace=ws[: need // 2])


@pytest.mark.slow
def test_full_size_2p27_keys_only(rs):
    """The benchmark's single-array workload with radix 2^16, bit-exact."""
    n = 1 << 27
    announce("pr2 2^27 keys")
    keys = keygen.uniform_u32(n, keygen.SEED_LARGE)
    ko, _ = rs.sort(dev(keys), algo="lsd16")
    got = host(ko)
    want, _ = oracle.sr4(keys)
    assert np.array_equal(got, want)
    rs.rsort_synchronize()
