"""GPU parity of the regular-oversampling sample sort (GSD, Algorithm 1)
against the oracle's GSD, and of the random-oversampling variants (GER,
Algorithm 2; GVR, Algorithm 3) against the oracle's GER and GVR fed the same
random draws.

Compared bit-exactly: the sorted keys and payloads, the p x p split matrix
cnt[k][j] = |X_{k,j}|, the bucket sizes and the p - 1 splitter composites
(key, input index).  Also checked: the bucket bound of Lemma 1 on every
distribution (duplicates included), the clamp p = n for tiny inputs, small
blocks (whole-block LDS sorts) and large ones (tiled rounds), in-place sorting,
keys only, rsort_sort's default p = 256, r = 32, and argument errors.
"""
import numpy as np
import pytest

import keygen
import oracle
from tests.lemma2 import default_omega_and_s, gvr_n_max, lemma2_bucket_bound
from tests.gpu_util import announce, check_kv_invariants, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1808_10292_amd import rsort
    rsort.load_library()
    return rsort


def lemma1_bound(n, p, r):
    return (1.0 + 1.0 / r) * n / p + r * p


def run_case(rs, keys, p, r, with_vals=True, in_place=False):
    import torch
    n = keys.size
    vals = np.arange(n, dtype=np.uint32)
    want = oracle.gsd(keys, vals if with_vals else None, p, r)
    dk = dev(keys)
    dv = dev(vals) if with_vals else None
    if in_place:
        ko, vo = dk, dv
    else:
        ko = torch.empty_like(dk)
        vo = torch.empty_like(dv) if with_vals else None
    rs.rsort_sample_sort(dk, ko, dv, vo, p=p, r=r)
    rs.rsort_synchronize()
    got_k = host(ko)
    assert np.array_equal(got_k, want["keys"])
    if with_vals:
        assert np.array_equal(host(vo), want["vals"])
    st = rs.rsort_sample_sort_stats()
    pu = want["p"]
    assert st["p"] == pu
    assert np.array_equal(st["cnt"].astype(np.uint64), want["cnt"])
    assert np.array_equal(st["bucket"].astype(np.uint64), want["bucket"])
    assert np.array_equal(st["split_key"], want["split_key"])
    assert np.array_equal(st["split_index"].astype(np.uint64), want["split_g"])
    assert int(st["bucket"].max()) <= lemma1_bound(n, pu, r)
    return st


@pytest.mark.parametrize("dist", keygen.KV_DISTRIBUTIONS)
def test_distributions_small_blocks(rs, dist):
    """n = 300007, p = 256: blocks of ~1172 keys (in-LDS local sorts)."""
    n = 300007
    announce("gsd small blocks", dist, n)
    run_case(rs, keygen.kv_keys(dist, n), 256, 32)


@pytest.mark.parametrize("dist", keygen.KV_DISTRIBUTIONS)
def test_distributions_large_blocks(rs, dist):
    """n = 3000017, p = 256: blocks of ~11719 keys (tiled rounds, ragged tiles)."""
    n = 3000017
    announce("gsd large blocks", dist, n)
    run_case(rs, keygen.kv_keys(dist, n), 256, 32)


@pytest.mark.parametrize("n,p,r", [(1, 256, 32), (2, 256, 32), (299, 300, 2), (1000, 1, 1),
                                   (50000, 7, 3), (65536, 1024, 4), (123457, 100, 1),
                                   (200000, 64, 64)])
def test_shapes(rs, n, p, r):
    announce("gsd shape", n, p, r)
    keys = keygen.zipf_keys(n, 40 + p)
    run_case(rs, keys, p, r)


@pytest.mark.parametrize("dist", ["uniform", "zipf", "equal"])
def test_route_path_p512(rs, dist):
    """p = 512 > 256 takes the route + bucket re-sort finish instead of the
    merge: blocks of ~8192 keys, two route tiles each (the last ragged)."""
    n = (1 << 22) + 5
    announce("gsd route p512", dist, n)
    run_case(rs, keygen.kv_keys(dist, n), 512, 8)
    run_case(rs, keygen.kv_keys(dist, n), 512, 8, with_vals=False)


@pytest.mark.parametrize("dist", ["uniform", "zipf", "equal", "presorted"])
@pytest.mark.parametrize("n,p,r", [((1 << 22) + 5, 64, 4), (1 << 21, 16, 2)])
def test_merge_pieces_beyond_lds(rs, dist, n, p, r):
    """Shapes whose merge pieces often exceed one LDS tile (4096 keys): the
    edge pieces at n = 2^22 + 5, p = 64 (about 8 K keys each), and pieces of
    about 4096 keys on average at n = 2^21, p = 16, r = 2."""
    announce("gsd merge large pieces", dist, n, p, r)
    run_case(rs, keygen.kv_keys(dist, n), p, r)


def test_keys_only_and_in_place(rs):
    n = 1000003
    announce("gsd keys only / in place", n)
    keys = keygen.uniform_u32(n, 17)
    run_case(rs, keys, 256, 32, with_vals=False)
    run_case(rs, keys, 256, 32, with_vals=True, in_place=True)
    run_case(rs, keys, 128, 8, with_vals=False, in_place=True)


def test_rsort_sort_default_parameters(rs):
    """rsort_sort with the sample-sort algorithm: p = 256, r = 32."""
    n = 1 << 22
    announce("gsd via rsort_sort", n)
    keys = keygen.uniform_u32(n, 21)
    vals = np.arange(n, dtype=np.uint32)
    ko, vo = rs.sort(dev(keys), dev(vals), algo="sample")
    rs.rsort_synchronize()
    want = oracle.gsd(keys, vals, 256, 32)
    assert np.array_equal(host(ko), want["keys"])
    assert np.array_equal(host(vo), want["vals"])
    st = rs.rsort_sample_sort_stats()
    assert st["p"] == 256
    assert np.array_equal(st["bucket"].astype(np.uint64), want["bucket"])


def test_errors(rs):
    import torch
    k32 = dev(keygen.uniform_u32(1000, 3))
    o32 = torch.empty_like(k32)
    for p, r in ((0, 4), (1025, 1), (256, 0)):
        with pytest.raises(rs.RsortError) as e:
            rs.rsort_sample_sort(k32, o32, p=p, r=r)
        assert e.value.status == rs.RSORT_EINVAL
    with pytest.raises(rs.RsortError) as e:
        rs.rsort_sample_sort(k32, o32, p=1024, r=128)      # sample 2^27 > 2^26
    assert e.value.status == rs.RSORT_EUNSUPPORTED
    k64 = dev(keygen.uniform_u64(1000, 3))
    with pytest.raises(rs.RsortError) as e:
        rs.rsort_sample_sort(k64, torch.empty_like(k64))
    assert e.value.status == rs.RSORT_EUNSUPPORTED
    with pytest.raises(rs.RsortError):
        rs.sort(k32, algo="sample", begin_bit=0, end_bit=16)
    e0 = torch.empty(0, dtype=torch.uint32, device="cuda")
    rs.rsort_sample_sort(e0, e0)


def test_graph_capture_replays(rs):
    """The sample sort needs no host traffic: captured once, every replay
    (with eager work between) equals the eager result and follows new data."""
    import torch
    n = 500009
    announce("gsd graph", n)
    keys = keygen.zipf_keys(n, 91)
    vals = np.arange(n, dtype=np.uint32)
    dk, dv = dev(keys), dev(vals)
    ko, vo = torch.empty_like(dk), torch.empty_like(dv)
    need = rs.rsort_sample_sort_workspace_bytes(torch.uint32, True, n, 256, 32)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rs.rsort_sample_sort(dk, ko, dv, vo, workspace=ws)
    torch.cuda.synchronize()
    want = oracle.gsd(keys, vals, 256, 32)
    assert np.array_equal(host(ko), want["keys"]) and np.array_equal(host(vo), want["vals"])
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rs.rsort_sample_sort(dk, ko, dv, vo, workspace=ws)
    for rep in range(3):
        ko.view(torch.int32).fill_(rep)
        vo.view(torch.int32).fill_(rep)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(ko), want["keys"]), rep
        assert np.array_equal(host(vo), want["vals"]), rep
    keys2 = keygen.uniform_u32(n, 92)
    dk.copy_(dev(keys2))
    g.replay()
    torch.cuda.synchronize()
    assert np.array_equal(host(ko), oracle.gsd(keys2, vals, 256, 32)["keys"])


# ---------------------------------------------------------------------------
# GER (Algorithm 2): the random sample is drawn on the GPU from SplitMix64
# stream `seed`; the oracle gets the same draws from the input generator.

def run_ger(rs, keys, p, s, seed, with_vals=True):
    import torch
    n = keys.size
    pu = min(p, n)
    vals = np.arange(n, dtype=np.uint32)
    pos = keygen.sample_positions(seed, s * pu - 1, n)
    want = oracle.ger(keys, vals if with_vals else None, p, s, pos)
    dk = dev(keys)
    dv = dev(vals) if with_vals else None
    ko = torch.empty_like(dk)
    vo = torch.empty_like(dv) if with_vals else None
    rs.rsort_sample_sort_random(dk, ko, dv, vo, p=p, s=s, seed=seed)
    rs.rsort_synchronize()
    assert np.array_equal(host(ko), want["keys"])
    if with_vals:
        assert np.array_equal(host(vo), want["vals"])
    st = rs.rsort_sample_sort_stats()
    assert st["p"] == want["p"]
    assert np.array_equal(st["cnt"].astype(np.uint64), want["cnt"])
    assert np.array_equal(st["split_key"], want["split_key"])
    assert np.array_equal(st["split_index"].astype(np.uint64), want["split_g"])
    return st


@pytest.mark.parametrize("dist", keygen.KV_DISTRIBUTIONS)
def test_ger_distributions(rs, dist):
    n = 1000003
    announce("ger", dist, n)
    run_ger(rs, keygen.kv_keys(dist, n), 256, 40, 0x5EED + len(dist))


@pytest.mark.parametrize("n,p,s", [(1, 256, 3), (2, 4, 1), (999, 9, 1), (1000, 1, 5),
                                   (50000, 7, 300), (65536, 1024, 4), (300007, 256, 140)])
def test_ger_shapes(rs, n, p, s):
    announce("ger shape", n, p, s)
    run_ger(rs, keygen.zipf_keys(n, 60 + p), p, s, 1000 + n)


def test_ger_default_oversampling_and_keys_only(rs):
    """s = 0 takes s = 2 w^2 lg n, w = ceil(lg lg n): 2 * 25 * 22 = 1100 at n = 2^22."""
    import torch
    n = 1 << 22
    announce("ger default", n)
    keys = keygen.uniform_u32(n, 61)
    run_ger(rs, keys, 256, 1100, 7, with_vals=False)
    ko = torch.empty_like(dev(keys))
    rs.rsort_sample_sort_random(dev(keys), ko, p=256, s=0, seed=7)
    rs.rsort_synchronize()
    assert np.array_equal(host(ko), oracle.sr4(keys)[0])
    need0 = rs.rsort_sample_sort_random_workspace_bytes(torch.uint32, False, n, 256, 0)
    need1 = rs.rsort_sample_sort_random_workspace_bytes(torch.uint32, False, n, 256, 1100)
    assert need0 == need1
    with pytest.raises(rs.RsortError) as e:
        rs.rsort_sample_sort_random(dev(keys), ko, p=1024, s=1 << 17)
    assert e.value.status == rs.RSORT_EUNSUPPORTED


@pytest.mark.slow
@pytest.mark.parametrize("dist", ["uniform", "zipf", "equal"])
def test_ger_full_size_kv(rs, dist):
    """2^28 pairs, p = 256, default s = 1400: the stable sort (four invariants)
    and every bucket within the sampling lemma's ceil((1 + eps)(n - p + 1)/p)
    for rho = 1 (eps about 0.24; exceeded with probability at most 2^-28)."""
    import torch
    n = 1 << 28
    announce("ger full", dist, n)
    keys = keygen.kv_keys(dist, n)
    dk = dev(keys)
    dv = torch.arange(n, dtype=torch.int32, device="cuda")
    ko, vo = torch.empty_like(dk), torch.empty_like(dv)
    rs.rsort_sample_sort_random(dk, ko, dv, vo, p=256, s=0, seed=11)
    rs.rsort_synchronize()
    del dk
    st = rs.rsort_sample_sort_stats()
    assert int(st["bucket"].astype(np.uint64).sum()) == n
    _, s = default_omega_and_s(n)
    assert int(st["bucket"].max()) <= lemma2_bucket_bound(n, 256, s)
    check_kv_invariants(keys, host(ko), host(vo).view(np.uint32))


# ---------------------------------------------------------------------------
# GVR (Algorithm 3): the sample is drawn from the input with the same
# generator; no local sort; the input is routed by bucket, then each bucket is
# sorted.  cnt[k][j] counts input block k's keys in bucket j.

def run_gvr(rs, keys, p, s, seed, with_vals=True, in_place=False, offset=0):
    """offset > 0 sorts a view starting `offset` elements into a larger device
    array (an input pointer not 16-byte aligned)."""
    import torch
    n = keys.size
    pu = min(p, n)
    vals = np.arange(n, dtype=np.uint32)
    pos = keygen.sample_positions(seed, s * pu - 1, n)
    want = oracle.gvr(keys, vals if with_vals else None, p, s, pos)
    big = dev(np.concatenate([np.zeros(offset, np.uint32), keys]))
    dk = big[offset:]
    dv = dev(vals) if with_vals else None
    if in_place:
        ko, vo = dk, dv
    else:
        ko = torch.empty_like(dk)
        vo = torch.empty_like(dv) if with_vals else None
    rs.rsort_sample_sort_gvr(dk, ko, dv, vo, p=p, s=s, seed=seed)
    rs.rsort_synchronize()
    assert np.array_equal(host(ko), want["keys"])
    if with_vals:
        assert np.array_equal(host(vo), want["vals"])
    st = rs.rsort_sample_sort_stats()
    assert st["p"] == want["p"]
    assert np.array_equal(st["cnt"].astype(np.uint64), want["cnt"])
    assert np.array_equal(st["bucket"].astype(np.uint64), want["bucket"])
    assert np.array_equal(st["split_key"], want["split_key"])
    assert np.array_equal(st["split_index"].astype(np.uint64), want["split_g"])
    return st


@pytest.mark.parametrize("dist", keygen.KV_DISTRIBUTIONS)
def test_gvr_distributions(rs, dist):
    """p = 64 blocks of about 47 K keys: several route tiles per block, the
    last one ragged."""
    n = 3000017
    announce("gvr", dist, n)
    run_gvr(rs, keygen.kv_keys(dist, n), 64, 60, 0x6E5 + len(dist))


@pytest.mark.parametrize("n,p,s", [(1, 256, 3), (2, 4, 1), (999, 9, 1), (1000, 1, 5),
                                   (50000, 7, 300), (65536, 256, 4), (300007, 256, 140),
                                   (8192 * 16, 16, 50), ((1 << 21) + 77, 16, 50)])
def test_gvr_shapes(rs, n, p, s):
    announce("gvr shape", n, p, s)
    run_gvr(rs, keygen.zipf_keys(n, 70 + p), p, s, 2000 + n)


def test_gvr_in_place_unaligned_and_keys_only(rs):
    n = 1000003
    announce("gvr in place / unaligned / keys only", n)
    keys = keygen.uniform_u32(n, 63)
    run_gvr(rs, keys, 256, 40, 9, in_place=True)
    run_gvr(rs, keys, 256, 40, 10, offset=1)
    run_gvr(rs, keys, 128, 40, 11, with_vals=False, offset=3)


def _span_keys(case, n, seed):
    rng = np.random.default_rng(seed)
    if case == "one_value":
        return np.full(n, 0x9E3779B9, np.uint32)
    if case == "one_value_max":
        return np.full(n, 0xFFFFFFFF, np.uint32)
    if case == "top_byte_span":      # keys in [2^32 - 256, 2^32): spans below 2^8
        return (0xFFFFFF00 + rng.integers(0, 256, n)).astype(np.uint32)
    if case == "low16":
        return rng.integers(0, 1 << 16, n, dtype=np.uint32)
    if case == "low24":
        return rng.integers(0, 1 << 24, n, dtype=np.uint32)
    if case == "two_values":
        return np.where(rng.random(n) < 0.5, 5, 0xFFFFFFF0).astype(np.uint32)
    k = rng.integers(0, 1 << 32, n, dtype=np.uint32)   # "uniform_extremes"
    k[0], k[-1] = 0xFFFFFFFF, 0
    return k


@pytest.mark.parametrize("case,p,with_vals,in_place,offset", [
    ("one_value", 16, True, False, 0),
    ("one_value", 16, False, True, 0),
    ("one_value", 256, True, False, 0),
    ("one_value", 256, True, True, 0),
    ("one_value", 256, False, False, 2),
    ("one_value_max", 7, True, False, 1),
    ("top_byte_span", 4, True, False, 0),
    ("top_byte_span", 1, False, False, 3),
    ("low16", 1, True, False, 0),
    ("low16", 64, True, True, 0),
    ("low24", 4, True, False, 0),
    ("low24", 4, False, False, 2),
    ("two_values", 2, True, False, 0),
    ("uniform_extremes", 64, True, False, 0),
    ("uniform_extremes", 1, True, False, 1),
    ("uniform_extremes", 2, False, False, 0),
])
def test_gvr_bucket_spans(rs, case, p, with_vals, in_place, offset):
    """The route stores key - lo_j and the bucket sort runs only the digits of
    the widest bucket span: no round (one key value: the route writes the
    output itself, or in place the routed keys are copied; with p = 256 the
    buckets are below the small-segment limit), one, two, three (keys below 2^24 in 4 buckets) or four (spread
    keys: the keys are routed unchanged), including the extreme keys 0 and 2^32 - 1, unaligned
    outputs (scalar path) and a ragged tail; buckets above the small-segment
    limit take the tiled rounds."""
    n = (1 << 20) + 3
    announce("gvr spans", case, p, with_vals, in_place, offset)
    run_gvr(rs, _span_keys(case, n, 31 + p), p, 20, 77 + p, with_vals=with_vals,
            in_place=in_place, offset=offset)


def test_gvr_default_oversampling_and_errors(rs):
    """s = 0 takes s = 2 w^2 lg n as for GER; p above 256 is refused."""
    import torch
    n = 1 << 22
    announce("gvr default", n)
    keys = keygen.uniform_u32(n, 64)
    run_gvr(rs, keys, 256, 1100, 8, with_vals=False)
    ko = torch.empty_like(dev(keys))
    rs.rsort_sample_sort_gvr(dev(keys), ko, p=256, s=0, seed=8)
    rs.rsort_synchronize()
    assert np.array_equal(host(ko), oracle.sr4(keys)[0])
    need0 = rs.rsort_sample_sort_gvr_workspace_bytes(torch.uint32, False, n, 256, 0)
    need1 = rs.rsort_sample_sort_gvr_workspace_bytes(torch.uint32, False, n, 256, 1100)
    assert need0 == need1
    with pytest.raises(rs.RsortError) as e:
        rs.rsort_sample_sort_gvr(dev(keys), ko, p=257, s=4)
    assert e.value.status == rs.RSORT_EINVAL
    with pytest.raises(rs.RsortError) as e:
        rs.rsort_sample_sort_gvr(dev(keys), ko, p=256, s=(1 << 18) + 1)
    assert e.value.status == rs.RSORT_EUNSUPPORTED


@pytest.mark.slow
@pytest.mark.parametrize("dist", ["uniform", "zipf", "equal"])
def test_gvr_full_size_kv(rs, dist):
    """2^28 pairs, p = 256, default s: the stable sort (four invariants), the
    bucket sizes summing to n, the column sums of cnt equal to them, and every
    bucket within GVR's n_max = (1 + 1/omega)(n/p) = 1.2 n/p and within the
    sampling lemma's bound for rho = 1."""
    import torch
    n = 1 << 28
    announce("gvr full", dist, n)
    keys = keygen.kv_keys(dist, n)
    dk = dev(keys)
    dv = torch.arange(n, dtype=torch.int32, device="cuda")
    ko, vo = torch.empty_like(dk), torch.empty_like(dv)
    rs.rsort_sample_sort_gvr(dk, ko, dv, vo, p=256, s=0, seed=12)
    rs.rsort_synchronize()
    del dk
    st = rs.rsort_sample_sort_stats()
    assert int(st["bucket"].astype(np.uint64).sum()) == n
    assert np.array_equal(st["cnt"].astype(np.uint64).sum(axis=0), st["bucket"].astype(np.uint64))
    w, s = default_omega_and_s(n)
    assert int(st["bucket"].max()) <= gvr_n_max(n, 256, w)
    assert int(st["bucket"].max()) <= lemma2_bucket_bound(n, 256, s)
    check_kv_invariants(keys, host(ko), host(vo).view(np.uint32))


@pytest.mark.slow
@pytest.mark.parametrize("dist", keygen.KV_DISTRIBUTIONS)
def test_full_size_kv(rs, dist):
    """The key-value workload at full size: 2^28 pairs, payload = input index,
    p = 256, r = 32.  The four invariants of check_kv_invariants determine the
    stable sort uniquely; the bucket sizes obey Lemma 1 and sum to n."""
    import torch
    n = 1 << 28
    announce("gsd full", dist, n)
    keys = keygen.kv_keys(dist, n)
    dk = dev(keys)
    dv = torch.arange(n, dtype=torch.int32, device="cuda")
    ko, vo = torch.empty_like(dk), torch.empty_like(dv)
    rs.rsort_sample_sort(dk, ko, dv, vo, p=256, r=32)
    rs.rsort_synchronize()
    del dk
    st = rs.rsort_sample_sort_stats()
    assert int(st["bucket"].astype(np.uint64).sum()) == n
    assert int(st["bucket"].max()) <= lemma1_bound(n, 256, 32)
    assert np.all(st["cnt"].astype(np.uint64).sum(axis=1) == n // 256)   # block sizes
    check_kv_invariants(keys, host(ko), host(vo).view(np.uint32))
