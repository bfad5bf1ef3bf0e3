"""The seeded input generators reproduce and have the stated distributions."""
import numpy as np

import keygen


def test_splitmix64_reference_values():
    # First outputs of SplitMix64 seeded with 1234567 (published reference
    # sequence of the algorithm, as used e.g. to seed xoshiro generators).
    got = keygen.splitmix64(1234567, 5).tolist()
    assert got == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]


def test_counter_based_streams_reproduce_and_split():
    a = keygen.splitmix64(42, 1000)
    b = keygen.splitmix64(42, 600, start=400)
    assert np.array_equal(a[400:], b)
    assert not np.array_equal(keygen.uniform_u32(100, 1), keygen.uniform_u32(100, 2))


def test_uniform_ranges():
    u = keygen.uniform_u31(1 << 16, 5)
    assert u.max() < (1 << 31)
    v = keygen.uniform_u32(1 << 16, 5)
    assert v.max() >= (1 << 31)
    m = keygen.low16(1000, 3)
    assert np.all((m >> np.uint32(16)) == 0xA5A5)


def test_zipf_top_rank_frequency():
    n = 1 << 20
    r = keygen.zipf_ranks(n, 9)
    h = np.sum(np.arange(1, (1 << 20) + 1, dtype=np.float64) ** -1.1)
    p1 = 1.0 / h
    f1 = np.mean(r == 1)
    assert abs(f1 - p1) < 5 * np.sqrt(p1 * (1 - p1) / n)
    f2 = np.mean(r == 2)
    p2 = 2.0 ** -1.1 / h
    assert abs(f2 - p2) < 5 * np.sqrt(p2 * (1 - p2) / n)
    k = keygen.zipf_keys(1000, 9)
    assert k.dtype == np.uint32


def test_monotone_generators():
    a = keygen.nondecreasing_u32(100000, 4)
    assert np.all(a[1:] >= a[:-1])
    assert a[0] < (1 << 20) and a[-1] > 0xFFF00000
    b = keygen.nonincreasing_u32(1000, 4)
    assert np.all(b[1:] <= b[:-1])


def test_lognormal_sizes():
    s = keygen.lognormal_sizes(4096)
    assert s.min() >= 16 and s.max() <= (1 << 20)
    assert 3000 < np.median(s) < 5500
    total = int(s.sum())
    assert 2e7 < total < 1.2e8  # expected about 5e7 keys


def test_poisson_and_log_uniform():
    t = keygen.poisson_arrivals(20000, 100.0, 3)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 0.01) < 0.0005
    s = keygen.log_uniform_sizes(20000, 3)
    assert s.min() >= 1024 and s.max() <= (1 << 26)
    assert abs(np.median(np.log2(s)) - 18.0) < 0.3
