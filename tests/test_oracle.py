"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test checks the oracle (``oracle/``) against one of: a brute-force stable
insertion sort on tiny inputs, the Python/numpy stable sorts (textbook library
routines), invariants that together characterise the unique stable sort, closed
forms for special inputs, and the paper's own bound on GSD bucket sizes
(Section 3.3, Lemma 1).  ``test_oracle_mutants.py`` shows that plausible
mistakes planted in the oracle's source fail these pins.
"""
import itertools

import numpy as np
import pytest

import keygen
import oracle

ALPHABET = [0, 1, 0xFF, 0x100, 0xFFFF, 0x10000, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF]


def insertion_sort_pairs(keys):
    """Brute force: stable insertion sort of (key, original index)."""
    out = []
    for i, k in enumerate(keys):
        j = len(out)
        while j > 0 and out[j - 1][0] > k:
            j -= 1
        out.insert(j, (k, i))
    return out


def stable_reference(keys):
    """Python's sorted() is stable: indices ordered by key, ties by position."""
    idx = sorted(range(len(keys)), key=lambda i: int(keys[i]))
    return np.asarray(idx, dtype=np.int64)


def check_kv_invariants(keys_in, keys_out, vals_out):
    """P3: with vals = original index, these four facts prove keys_out/vals_out is
    the unique stable sort of keys_in."""
    n = keys_in.size
    assert keys_out.size == n and vals_out.size == n
    if n == 0:
        return
    assert np.all(keys_out[1:] >= keys_out[:-1]), "not nondecreasing"
    seen = np.zeros(n, dtype=bool)
    assert vals_out.max() < n
    seen[vals_out] = True
    assert seen.all(), "payload is not a permutation"
    assert np.array_equal(keys_out, keys_in[vals_out]), "payload does not travel with its key"
    tie = keys_out[1:] == keys_out[:-1]
    assert np.all(vals_out[1:][tie] > vals_out[:-1][tie]), "ties not in input order"


# ---------------------------------------------------------------------------
# SR4 / LSD rounds (Section 3.2)

def test_exhaustive_small_alphabet_vs_insertion_sort():
    """Every sequence of length <= 4 over a 9-symbol alphabet that exercises each
    byte position, plus length 5 sampled, against brute-force insertion sort."""
    seqs = []
    for n in range(0, 5):
        seqs.extend(itertools.product(ALPHABET, repeat=n))
    rng = np.random.default_rng(1)
    for _ in range(3000):
        seqs.append(tuple(int(x) for x in rng.choice(ALPHABET, size=5)))
    sizes = np.array([len(s) for s in seqs], dtype=np.int64)
    keys = np.array([k for s in seqs for k in s], dtype=np.uint32)
    off = keygen.offsets_from_sizes(sizes)
    local_idx = np.concatenate([np.arange(len(s), dtype=np.uint32) for s in seqs])
    ko, vo = oracle.segmented(keys, local_idx, off)
    for si, s in enumerate(seqs):
        lo, hi = int(off[si]), int(off[si + 1])
        want = insertion_sort_pairs(list(s))
        got = list(zip(ko[lo:hi].tolist(), vo[lo:hi].tolist()))
        assert got == want, (s, got, want)


@pytest.mark.parametrize("digit_bits", [8, 16, 5, 11])
def test_random_vs_python_sorted(digit_bits):
    rng = np.random.default_rng(digit_bits)
    for trial in range(40):
        n = int(rng.integers(0, 2000))
        hi = [2, 300, 1 << 16, 1 << 32][trial % 4]
        keys = rng.integers(0, hi, size=n, dtype=np.uint64).astype(np.uint32)
        idx = np.arange(n, dtype=np.uint32)
        ko, vo = oracle.lsd_sort(keys, idx, digit_bits)
        ref = stable_reference(keys)
        assert np.array_equal(vo, ref.astype(np.uint32))
        assert np.array_equal(ko, keys[ref])


def test_large_vs_numpy_stable_argsort():
    for dist in keygen.KV_DISTRIBUTIONS:
        keys = keygen.kv_keys(dist, 1 << 18)
        idx = np.arange(keys.size, dtype=np.uint32)
        ko, vo = oracle.sr4(keys, idx)
        ref = np.argsort(keys, kind="stable")
        assert np.array_equal(vo, ref.astype(np.uint32)), dist
        assert np.array_equal(ko, keys[ref]), dist
        check_kv_invariants(keys, ko, vo)


def test_keys_only_matches_kv_keys():
    keys = keygen.uniform_u32(100003, 7)
    ko, vo = oracle.sr4(keys)
    assert vo is None
    ko2, _ = oracle.sr4(keys, np.zeros(keys.size, dtype=np.uint32))
    assert np.array_equal(ko, ko2)
    # multiset equality by a full count of values
    u1, c1 = np.unique(keys, return_counts=True)
    u2, c2 = np.unique(ko, return_counts=True)
    assert np.array_equal(u1, u2) and np.array_equal(c1, c2)


def test_round_invariant_after_each_round():
    """P6: after round d of SR4 the array is the stable sort by the low 8(d+1) bits."""
    keys = keygen.uniform_u32(50000, 11)
    idx = np.arange(keys.size, dtype=np.uint32)
    for d in range(4):
        ko, vo = oracle.lsd_sort(keys, idx, 8, 0, 8 * (d + 1))
        masked = keys.astype(np.uint64) & np.uint64((1 << (8 * (d + 1))) - 1)
        ref = np.argsort(masked, kind="stable")
        assert np.array_equal(vo, ref.astype(np.uint32)), d
        assert np.array_equal(ko, keys[ref]), d


def test_bit_ranges():
    keys = keygen.uniform_u32(30000, 12)
    idx = np.arange(keys.size, dtype=np.uint32)
    for lo, hi in [(0, 0), (3, 17), (8, 24), (16, 32), (31, 32)]:
        ko, vo = oracle.lsd_sort(keys, idx, 8, lo, hi)
        field = (keys.astype(np.uint64) >> np.uint64(lo)) & np.uint64((1 << (hi - lo)) - 1)
        ref = np.argsort(field, kind="stable")
        assert np.array_equal(vo, ref.astype(np.uint32)), (lo, hi)


def test_radix_16_equals_radix_8():
    """PR2's rounds (r = 2^16) and SR4's (r = 2^8) reach the same unique result."""
    for dist in keygen.KV_DISTRIBUTIONS:
        keys = keygen.kv_keys(dist, 70001)
        idx = np.arange(keys.size, dtype=np.uint32)
        a = oracle.lsd_sort(keys, idx, 8)
        b = oracle.lsd_sort(keys, idx, 16)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_special_cases_closed_form():
    """P5: closed forms for degenerate inputs."""
    n = 4097
    idx = np.arange(n, dtype=np.uint32)
    # all equal -> identity permutation
    ko, vo = oracle.sr4(keygen.all_equal(n), idx)
    assert np.array_equal(vo, idx)
    # strictly increasing -> identity
    inc = (np.arange(n, dtype=np.uint64) * np.uint64(1048573)).astype(np.uint32)
    ko, vo = oracle.sr4(inc, idx)
    assert np.array_equal(vo, idx) and np.array_equal(ko, inc)
    # strictly decreasing -> reversal
    dec = inc[::-1].copy()
    ko, vo = oracle.sr4(dec, idx)
    assert np.array_equal(vo, idx[::-1]) and np.array_equal(ko, inc)
    # decreasing with duplicates -> blocks reversed, indices increasing within blocks
    blk = np.repeat(np.arange(100, 0, -1, dtype=np.uint32) * np.uint32(0x01010101 // 3), 7)
    bi = np.arange(blk.size, dtype=np.uint32)
    ko, vo = oracle.sr4(blk, bi)
    want = np.concatenate([np.arange(7 * b, 7 * b + 7) for b in range(99, -1, -1)])
    assert np.array_equal(vo, want.astype(np.uint32))
    # empty and single
    ko, vo = oracle.sr4(np.zeros(0, dtype=np.uint32), np.zeros(0, dtype=np.uint32))
    assert ko.size == 0
    ko, vo = oracle.sr4(np.array([7], dtype=np.uint32), np.array([0], dtype=np.uint32))
    assert ko.tolist() == [7] and vo.tolist() == [0]


def test_low16_keys_upper_rounds_identity():
    keys = keygen.low16(20000, 3)
    idx = np.arange(keys.size, dtype=np.uint32)
    a = oracle.lsd_sort(keys, idx, 8, 0, 16)
    b = oracle.lsd_sort(keys, idx, 8, 0, 32)
    assert np.array_equal(a[1], b[1])


def test_digit_counts_vs_bincount():
    keys = keygen.zipf_keys(100000, 5)
    for shift, width in [(0, 8), (8, 8), (16, 8), (24, 8), (0, 16), (16, 16), (5, 3)]:
        c = oracle.digit_counts(keys, shift, width)
        field = (keys >> np.uint32(shift)) & np.uint32((1 << width) - 1)
        ref = np.bincount(field, minlength=1 << width)
        assert np.array_equal(c, ref.astype(np.uint64))
        assert int(c.sum()) == keys.size


def test_u64_vs_numpy():
    keys = keygen.uniform_u64(60000, 9)
    keys[::7] = keys[3]  # duplicates
    idx = np.arange(keys.size, dtype=np.uint32)
    for bits in (8, 16):
        ko, vo = oracle.lsd_sort(keys, idx, bits)
        ref = np.argsort(keys, kind="stable")
        assert np.array_equal(vo, ref.astype(np.uint32))
        assert np.array_equal(ko, keys[ref])
    c = oracle.digit_counts(keys, 56, 8)
    assert np.array_equal(c, np.bincount((keys >> np.uint64(56)).astype(np.int64),
                                         minlength=256).astype(np.uint64))


def test_segmented_vs_per_segment_argsort():
    sizes = np.array([0, 1, 2, 17, 0, 300, 5000, 3], dtype=np.int64)
    off = keygen.offsets_from_sizes(sizes)
    keys = keygen.uniform_u31(int(off[-1]), 21)
    vals = np.arange(keys.size, dtype=np.uint32)
    ko, vo = oracle.segmented(keys, vals, off)
    for s in range(sizes.size):
        lo, hi = int(off[s]), int(off[s + 1])
        ref = np.argsort(keys[lo:hi], kind="stable") + lo
        assert np.array_equal(vo[lo:hi], ref.astype(np.uint32))


# ---------------------------------------------------------------------------
# GSD (Section 3.3, Algorithm 1)

def lemma1_bounds(n, p, r):
    """Lemma 1: each Y_j holds at most (1 + 1/r) n/p + r p keys; when p | n and
    s = r p divides n/p, the proof's tighter (s + p - 1) x with x = n/(p s)."""
    general = (1.0 + 1.0 / r) * n / p + r * p
    s = r * p
    tight = None
    if n % p == 0 and (n // p) % s == 0:
        x = n // p // s
        tight = (s + p - 1) * x
    return general, tight


def gsd_composite_check(keys, res):
    """Every key lands in the bucket its composite (key, g) selects: bucket(e) =
    #{i : S_i < e}, g being the position of e in the locally sorted blocks."""
    n = keys.size
    p = res["p"]
    bounds = [(k * n) // p for k in range(p + 1)]
    X = np.concatenate([np.sort(keys[bounds[k]:bounds[k + 1]], kind="stable")
                        for k in range(p)])
    g = np.arange(n, dtype=np.uint64)
    comp = (X.astype(np.uint64) << np.uint64(32)) | g
    sp = (res["split_key"].astype(np.uint64) << np.uint64(32)) | res["split_g"]
    assert np.all(sp[1:] >= sp[:-1]), "splitters not nondecreasing"
    bucket = np.searchsorted(sp, comp, side="left")  # number of splitters < e
    cnt = np.zeros((p, p), dtype=np.uint64)
    blk = np.searchsorted(np.asarray(bounds[1:]), np.arange(n), side="right")
    np.add.at(cnt, (blk, bucket), 1)
    assert np.array_equal(cnt, res["cnt"])


@pytest.mark.parametrize("dist", keygen.KV_DISTRIBUTIONS)
def test_gsd_output_bounds_and_split(dist):
    n, p, r = 1 << 16, 16, 4
    keys = keygen.kv_keys(dist, n)
    idx = np.arange(n, dtype=np.uint32)
    res = oracle.gsd(keys, idx, p, r)
    check_kv_invariants(keys, res["keys"], res["vals"])
    ref = np.argsort(keys, kind="stable")
    assert np.array_equal(res["vals"], ref.astype(np.uint32))
    cnt = res["cnt"]
    assert int(cnt.sum()) == n
    bounds = [(k * n) // p for k in range(p + 1)]
    assert np.array_equal(cnt.sum(axis=1), np.diff(bounds).astype(np.uint64))
    general, tight = lemma1_bounds(n, p, r)
    assert res["bucket"].max() <= general
    if tight is not None:
        assert res["bucket"].max() <= tight
    gsd_composite_check(keys, res)


def test_gsd_ragged_and_small():
    rng = np.random.default_rng(3)
    for n, p, r in [(1, 4, 2), (5, 8, 1), (1000, 7, 3), (4097, 16, 5), (65537, 32, 2)]:
        keys = rng.integers(0, 50, size=n, dtype=np.uint64).astype(np.uint32)
        idx = np.arange(n, dtype=np.uint32)
        res = oracle.gsd(keys, idx, p, r)
        assert res["p"] == min(p, n)
        assert np.array_equal(res["vals"], np.argsort(keys, kind="stable").astype(np.uint32))
        general, _ = lemma1_bounds(n, res["p"], r)
        assert res["bucket"].max() <= general + 1  # +1: the proof pads blocks to ceil(n/p)
        gsd_composite_check(keys, res)


def test_gsd_closed_form_identity_input():
    """Increasing keys 0..n-1 with p | n and s | n/p: the sorted sample is
    x-1, 2x-1, ..., so splitter i is i N - 1 (N = n/p) and block k goes whole
    to bucket k."""
    p, r = 8, 4
    N = 512
    n = p * N
    keys = np.arange(n, dtype=np.uint32)
    res = oracle.gsd(keys, None, p, r)
    assert np.array_equal(res["split_key"], (np.arange(1, p) * N - 1).astype(np.uint32))
    assert np.array_equal(res["cnt"], np.eye(p, dtype=np.uint64) * N)
    assert np.array_equal(res["keys"], keys)
    # all-equal keys order by position alone: the same split
    res = oracle.gsd(np.full(n, 9, dtype=np.uint32), None, p, r)
    assert np.array_equal(res["split_g"], (np.arange(1, p) * N - 1).astype(np.uint64))
    assert np.array_equal(res["cnt"], np.eye(p, dtype=np.uint64) * N)


def test_gsd_splitters_brute_force():
    """Splitters from the definition of Algorithm 1 steps 2-3, recomputed by brute
    force in Python for sizes where every segment has exactly x keys."""
    rng = np.random.default_rng(8)
    for p, r, x in [(4, 2, 3), (6, 3, 2), (5, 1, 7)]:
        s = r * p
        N = s * x
        n = N * p
        keys = rng.integers(0, 40, size=n, dtype=np.uint64).astype(np.uint32)
        res = oracle.gsd(keys, None, p, r)
        sample = []
        for k in range(p):
            blk = sorted(((int(keys[k * N + q]), k * N + q) for q in range(N)))
            X = [(key, k * N + pos) for pos, (key, _) in enumerate(blk)]
            sample.extend(X[x * j - 1] for j in range(1, s + 1))
        sample.sort()
        want = [sample[i * s - 1] for i in range(1, p)]
        got = list(zip(res["split_key"].tolist(), res["split_g"].tolist()))
        assert got == want


# ---------------------------------------------------------------------------
# GER (Algorithm 2): the GSD skeleton with a random sample whose draws (positions
# into the locally sorted blocks) are an input.

def _local_blocks(keys, p):
    """X and its composites by brute force: block k stable-sorted by Python."""
    n = keys.size
    X = []
    for k in range(p):
        a, b = (k * n) // p, ((k + 1) * n) // p
        X.extend(sorted(int(x) for x in keys[a:b]))   # equal keys: any order, same values
    return X


@pytest.mark.parametrize("dist", ["uniform", "zipf", "equal", "low16"])
def test_ger_output_split_and_splitters(dist):
    """Sorted output = the stable sort; splitters = the (i s)-th smallest
    (key, position) sample composites; cnt = the composite split of each block;
    all recomputed by brute force from the definition of Algorithm 2."""
    n, p, s = 20011, 12, 9
    keys = keygen.kv_keys(dist, n)
    idx = np.arange(n, dtype=np.uint32)
    pos = keygen.sample_positions(1234 + len(dist), s * p - 1, n)
    res = oracle.ger(keys, idx, p, s, pos)
    assert np.array_equal(res["vals"], np.argsort(keys, kind="stable").astype(np.uint32))
    X = _local_blocks(keys, p)
    sample = sorted((X[q], int(q)) for q in pos)
    want = [sample[i * s - 1] for i in range(1, p)]
    got = list(zip(res["split_key"].tolist(), res["split_g"].tolist()))
    assert got == want
    bounds = [(k * n) // p for k in range(p + 1)]
    comp = [(X[q], q) for q in range(n)]
    for k in range(p):
        for j in range(p):
            lo_s = want[j - 1] if j > 0 else None
            hi_s = want[j] if j < p - 1 else None
            c = sum(1 for q in range(bounds[k], bounds[k + 1])
                    if (lo_s is None or comp[q] > lo_s) and (hi_s is None or comp[q] <= hi_s))
            assert res["cnt"][k, j] == c, (k, j)
    assert int(res["cnt"].sum()) == n


def test_ger_small_and_degenerate():
    """p = 1 (no splitters), p clamped to n, s = 1, and repeated draws."""
    rng = np.random.default_rng(4)
    for n, p, s in [(1, 4, 3), (7, 16, 2), (1000, 1, 5), (999, 9, 1), (4096, 8, 40)]:
        keys = rng.integers(0, 30, size=n, dtype=np.uint64).astype(np.uint32)
        idx = np.arange(n, dtype=np.uint32)
        pu = min(p, n)
        pos = keygen.sample_positions(77 + n, max(s * pu - 1, 0), n)
        res = oracle.ger(keys, idx, p, s, pos)
        assert res["p"] == pu
        assert np.array_equal(res["vals"], np.argsort(keys, kind="stable").astype(np.uint32))
        assert int(res["cnt"].sum()) == n
        gsd_composite_check(keys, res)
    with pytest.raises(ValueError):
        oracle.ger(np.arange(10, dtype=np.uint32), None, 2, 3, np.array([0, 1], dtype=np.uint32))
    with pytest.raises(ValueError):
        oracle.ger(np.arange(10, dtype=np.uint32), None, 2, 1, np.array([10], dtype=np.uint32))


# ---------------------------------------------------------------------------
# GVR (Algorithm 3): random sample of the INPUT (draws = input positions), the
# unsorted blocks split by binary search + a count sort on the bucket index,
# then SR4 on every bucket.

@pytest.mark.parametrize("dist", ["uniform", "zipf", "equal", "low16"])
def test_gvr_output_split_and_splitters(dist):
    """Sorted output = the stable sort; splitters = the (i s)-th smallest
    (key, input position) sample composites; cnt[k, j] = elements of input
    block k whose composite lies in (S_{j-1}, S_j]; all by brute force from
    the definition of Algorithm 3."""
    n, p, s = 20011, 12, 9
    keys = keygen.kv_keys(dist, n)
    idx = np.arange(n, dtype=np.uint32)
    pos = keygen.sample_positions(4321 + len(dist), s * p - 1, n)
    res = oracle.gvr(keys, idx, p, s, pos)
    assert np.array_equal(res["vals"], np.argsort(keys, kind="stable").astype(np.uint32))
    assert np.array_equal(res["keys"], np.sort(keys, kind="stable"))
    sample = sorted((int(keys[q]), int(q)) for q in pos)
    want = [sample[i * s - 1] for i in range(1, p)]
    got = list(zip(res["split_key"].tolist(), res["split_g"].tolist()))
    assert got == want
    bounds = [(k * n) // p for k in range(p + 1)]
    for k in range(p):
        for j in range(p):
            lo_s = want[j - 1] if j > 0 else None
            hi_s = want[j] if j < p - 1 else None
            c = sum(1 for q in range(bounds[k], bounds[k + 1])
                    if (lo_s is None or (int(keys[q]), q) > lo_s) and
                    (hi_s is None or (int(keys[q]), q) <= hi_s))
            assert res["cnt"][k, j] == c, (k, j)
    assert int(res["cnt"].sum()) == n


def test_gvr_small_and_degenerate():
    """p = 1 (no splitters), p clamped to n, s = 1, repeated draws, and a
    sample drawn from one position only (every splitter equal)."""
    rng = np.random.default_rng(5)
    for n, p, s in [(1, 4, 3), (7, 16, 2), (1000, 1, 5), (999, 9, 1), (4096, 8, 40)]:
        keys = rng.integers(0, 30, size=n, dtype=np.uint64).astype(np.uint32)
        idx = np.arange(n, dtype=np.uint32)
        pu = min(p, n)
        pos = keygen.sample_positions(91 + n, max(s * pu - 1, 0), n)
        res = oracle.gvr(keys, idx, p, s, pos)
        assert res["p"] == pu
        assert np.array_equal(res["vals"], np.argsort(keys, kind="stable").astype(np.uint32))
        assert int(res["cnt"].sum()) == n
        bounds = [(k * n) // pu for k in range(pu + 1)]
        assert np.array_equal(res["cnt"].sum(axis=1), np.diff(bounds).astype(np.uint64))
    # one repeated draw: all splitters are (x_q, q); everything at or below goes
    # to bucket 0, the rest to bucket p - 1
    n, p, s, q = 500, 5, 3, 123
    keys = rng.integers(0, 10, size=n, dtype=np.uint64).astype(np.uint32)
    res = oracle.gvr(keys, None, p, s, np.full(s * p - 1, q, dtype=np.uint32))
    below = sum(1 for i in range(n) if (int(keys[i]), i) <= (int(keys[q]), q))
    assert res["bucket"].tolist() == [below, 0, 0, 0, n - below]
    assert np.array_equal(res["keys"], np.sort(keys))
    with pytest.raises(ValueError):
        oracle.gvr(np.arange(10, dtype=np.uint32), None, 2, 3, np.array([0, 1], dtype=np.uint32))
    with pytest.raises(ValueError):
        oracle.gvr(np.arange(10, dtype=np.uint32), None, 2, 1, np.array([10], dtype=np.uint32))


def test_sample_positions_closed_form():
    """Position i is floor((splitmix64 value i >> 32) * n / 2^32)."""
    z = keygen.splitmix64(5, 8)
    got = keygen.sample_positions(5, 8, 1000)
    want = [((int(v) >> 32) * 1000) >> 32 for v in z]
    assert got.tolist() == want
    assert keygen.sample_positions(5, 100000, 7).max() == 6


# ---------------------------------------------------------------------------
# Signed and floating-point keys (an extension: the paper sorts unsigned
# integers): pinned to numpy's stable argsort and to totalOrder's special
# values written out.

@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_signed_vs_numpy(dtype):
    rng = np.random.default_rng(11)
    info = np.iinfo(dtype)
    k = rng.integers(info.min, info.max, 20000, dtype=dtype, endpoint=True)
    k[:4] = [info.min, info.max, 0, -1]
    k[100:2000] = k[2000:3900]                      # duplicates
    ko, vo = oracle.sort_signed_or_float(k, np.arange(k.size, dtype=np.uint32), "signed")
    ref = np.argsort(k, kind="stable")
    assert np.array_equal(vo, ref.astype(np.uint32))
    assert np.array_equal(ko, k[ref])


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_float_vs_numpy(dtype):
    """Without NaNs and negative zeros numpy's order is totalOrder."""
    rng = np.random.default_rng(12)
    k = (rng.standard_normal(20000) * 1e3).astype(dtype)
    k[::5] = np.round(k[::5])                        # duplicates
    k[:6] = [np.inf, -np.inf, 0.0, np.finfo(dtype).tiny, -np.finfo(dtype).max, 1e-45]
    k[k == 0] = 0.0                                  # rounding made -0.0s: numpy ties them with +0.0
    ko, vo = oracle.sort_signed_or_float(k, np.arange(k.size, dtype=np.uint32), "float")
    ref = np.argsort(k, kind="stable")
    assert np.array_equal(vo, ref.astype(np.uint32))


def test_float_total_order_special_values():
    """-NaN < -inf < -1 < -0 < +0 < 1 < +inf < +NaN, ties in input order."""
    for dtype in (np.float32, np.float64):
        k = np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -1.0, np.nan, -np.nan, -0.0, 0.0],
                     dtype=dtype)
        ko, vo = oracle.sort_signed_or_float(k, np.arange(k.size, dtype=np.uint32), "float")
        assert vo.tolist() == [7, 3, 5, 1, 8, 0, 9, 4, 2, 6]
