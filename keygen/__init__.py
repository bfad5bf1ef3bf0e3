"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random inputs; it contains no sorting arithmetic (no
counting, prefix, ranking or ordering of keys), so both the CPU reference under
``oracle/`` and the GPU library can be fed from it without sharing any of the
method.

The paper (arXiv 1808.10292, Section 4) states problem sizes but never a key
distribution or generator.  The inputs below stand in for its workloads:

* every random number comes from SplitMix64 (Steele, Lea and Flood, "Fast
  splittable pseudorandom number generators", OOPSLA 2014), used as a
  counter-based generator: value i of stream ``seed`` is
  ``mix(seed + (i + 1) * 0x9E3779B97F4A7C15)``;
* key distributions: uniform 31-bit and 32-bit, low-16-bit-only, Zipf(s) over a
  finite rank set drawn with Vose's alias method, all-equal, nondecreasing and
  nonincreasing;
* segment sizes for batched sorting: lognormal, clipped;
* request streams for serving: log-uniform sizes and Poisson arrivals.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 24

# Seeds of the standard workloads (one per workload, distributions offset by index).
SEED_SMALL = 0x18081029201
SEED_LARGE = 0x18081029202
SEED_KV = 0x18081029203
SEED_SEGMENTS = 0x18081029204
SEED_SERVE = 0x18081029205


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Values start..start+count-1 of the SplitMix64 stream ``seed`` (uint64)."""
    out = np.empty(count, dtype=np.uint64)
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        for lo in range(0, count, _CHUNK):
            hi = min(count, lo + _CHUNK)
            z = np.arange(start + lo + 1, start + hi + 1, dtype=np.uint64)
            z *= GOLDEN
            z += s
            z ^= z >> np.uint64(30)
            z *= _M1
            z ^= z >> np.uint64(27)
            z *= _M2
            z ^= z >> np.uint64(31)
            out[lo:hi] = z
    return out


def unit_doubles(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in the open interval (0, 1): 53 high bits, centred."""
    x = splitmix64(seed, count, start) >> np.uint64(11)
    return (x.astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def uniform_u32(n: int, seed: int) -> np.ndarray:
    """Keys uniform over the full 32-bit range."""
    return (splitmix64(seed, n) >> np.uint64(32)).astype(np.uint32)


def uniform_u31(n: int, seed: int) -> np.ndarray:
    """Keys uniform in [0, 2^31)."""
    return (splitmix64(seed, n) >> np.uint64(33)).astype(np.uint32)


def uniform_u64(n: int, seed: int) -> np.ndarray:
    """Keys uniform over the full 64-bit range."""
    return splitmix64(seed, n)


def low16(n: int, seed: int, high: int = 0xA5A5) -> np.ndarray:
    """Only the low 16 bits vary; the high half is the constant ``high``."""
    u = (splitmix64(seed, n) >> np.uint64(32)).astype(np.uint32)
    return (np.uint32(high << 16) | (u & np.uint32(0xFFFF))).astype(np.uint32)


def all_equal(n: int, value: int = 0x5A5A5A5A) -> np.ndarray:
    return np.full(n, value, dtype=np.uint32)


def _alias_table(weights: np.ndarray):
    """Vose's alias method (Vose, IEEE TSE 1991): probability and alias columns."""
    m = weights.size
    prob = weights * (m / weights.sum())
    alias = np.zeros(m, dtype=np.int64)
    small = [i for i in range(m) if prob[i] < 1.0]
    large = [i for i in range(m) if prob[i] >= 1.0]
    while small and large:
        s = small.pop()
        l = large.pop()
        alias[s] = l
        prob[l] = prob[l] + prob[s] - 1.0
        (small if prob[l] < 1.0 else large).append(l)
    for i in large + small:
        prob[i] = 1.0
    return prob, alias


_ZIPF_CACHE: dict = {}


def zipf_ranks(n: int, seed: int, s: float = 1.1, num_ranks: int = 1 << 20) -> np.ndarray:
    """Ranks 1..num_ranks with P(k) proportional to k^-s (alias method)."""
    key = (s, num_ranks)
    if key not in _ZIPF_CACHE:
        w = np.arange(1, num_ranks + 1, dtype=np.float64) ** (-s)
        _ZIPF_CACHE[key] = _alias_table(w)
    prob, alias = _ZIPF_CACHE[key]
    u = unit_doubles(seed, 2 * n)
    col = np.minimum((u[0::2] * num_ranks).astype(np.int64), num_ranks - 1)
    take_alias = u[1::2] >= prob[col]
    ranks = np.where(take_alias, alias[col], col) + 1
    return ranks.astype(np.uint64)


def zipf_keys(n: int, seed: int, s: float = 1.1, num_ranks: int = 1 << 20) -> np.ndarray:
    """Zipf ranks mapped by Knuth's multiplicative hash k -> k * 2654435761 mod 2^32,
    a bijection on 32-bit words that spreads the distinct values over every digit."""
    r = zipf_ranks(n, seed, s, num_ranks)
    with np.errstate(over="ignore"):
        return ((r * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def nondecreasing_u32(n: int, seed: int) -> np.ndarray:
    """n nondecreasing keys distributed as the order statistics of n uniform
    32-bit draws, built from normalised partial sums of exponential spacings
    (so no sorting is involved)."""
    if n == 0:
        return np.zeros(0, dtype=np.uint32)
    e = -np.log(unit_doubles(seed, n + 1))
    c = np.cumsum(e)
    x = np.floor(c[:n] / c[n] * 4294967296.0)
    return np.minimum(x, 4294967295.0).astype(np.uint32)


def nonincreasing_u32(n: int, seed: int) -> np.ndarray:
    return nondecreasing_u32(n, seed)[::-1].copy()


KV_DISTRIBUTIONS = ("uniform", "low16", "zipf", "equal", "presorted", "reverse")


def kv_keys(dist: str, n: int, seed: int = SEED_KV) -> np.ndarray:
    """Keys of the key-value workload; distribution d uses seed + index(d)."""
    i = KV_DISTRIBUTIONS.index(dist)
    sd = seed + i
    if dist == "uniform":
        return uniform_u32(n, sd)
    if dist == "low16":
        return low16(n, sd)
    if dist == "zipf":
        return zipf_keys(n, sd)
    if dist == "equal":
        return all_equal(n)
    if dist == "presorted":
        return nondecreasing_u32(n, sd)
    return nonincreasing_u32(n, sd)


def lognormal_sizes(num: int, seed: int = SEED_SEGMENTS, median: float = 4096.0,
                    sigma: float = 1.5, lo: int = 16, hi: int = 1 << 20) -> np.ndarray:
    """Segment sizes clip(round(exp(ln(median) + sigma Z)), lo, hi); Z ~ N(0,1) by
    the Box-Muller transform."""
    u = unit_doubles(seed, 2 * num)
    z = np.sqrt(-2.0 * np.log(u[0::2])) * np.cos(2.0 * np.pi * u[1::2])
    sz = np.rint(np.exp(np.log(median) + sigma * z))
    return np.clip(sz, lo, hi).astype(np.int64)


def log_uniform_sizes(num: int, seed: int, lo_log2: float = 10.0,
                      hi_log2: float = 26.0) -> np.ndarray:
    """Sizes round(2^U) with U uniform on [lo_log2, hi_log2]."""
    u = unit_doubles(seed, num)
    return np.rint(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def poisson_arrivals(num: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process: cumulative exponential gaps."""
    gaps = -np.log(unit_doubles(seed, num)) / rate_per_s
    return np.cumsum(gaps)


def offsets_from_sizes(sizes: np.ndarray) -> np.ndarray:
    """CSR offsets (num+1, uint64) of consecutive segments with the given sizes."""
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(np.asarray(sizes, dtype=np.uint64))
    return off


def sample_positions(seed: int, count: int, n: int) -> np.ndarray:
    """Uniform draws with replacement from [0, n): position i is
    ((splitmix64 value i) >> 32) * n >> 32 (the high 32 bits scaled to n)."""
    hi = splitmix64(seed, count) >> np.uint64(32)
    with np.errstate(over="ignore"):
        return ((hi * np.uint64(n)) >> np.uint64(32)).astype(np.uint32)
