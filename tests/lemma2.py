"""Bucket-size bounds of the random-oversampling sample sorts (GER, GVR), from
Section 3.3 of arXiv 1808.10292: its sampling lemma (after Gerbessiotis and
Valiant) and the n_max of GVR stated after it.

Lemma: for p >= 2, s >= 1, ps < n/2, 0 < eps < 1, rho > 0 with
    s >= (1 + eps) / eps^2 * (2 rho log n + log(2 pi p^2 (ps - 1) e^(1 / (3 (ps - 1))))),
the probability that some bucket holds more than ceil((1 + eps)(n - p + 1) / p)
keys is at most n^-rho.  The logarithms are read as natural ones (the 2 pi
and the e^(1/(3m)) factor are those of Stirling's formula).
"""
import math


def lemma2_rhs_factor(n, p, s, rho=1.0):
    """The bracket 2 rho log n + log(2 pi p^2 (ps - 1) e^(1 / (3 (ps - 1))))."""
    m = p * s - 1
    return 2.0 * rho * math.log(n) + math.log(2.0 * math.pi * p * p * m) + 1.0 / (3.0 * m)


def lemma2_epsilon(n, p, s, rho=1.0):
    """Smallest eps in (0, 1) for which s satisfies the lemma's condition, by
    bisection on the condition as stated ((1 + eps) / eps^2 decreases in eps);
    None when no eps below 1 does."""
    if not (p >= 2 and s >= 1 and p * s < n / 2):
        return None
    L = lemma2_rhs_factor(n, p, s, rho)

    def ok(eps):
        return s >= (1.0 + eps) / (eps * eps) * L

    if not ok(1.0 - 1e-12):
        return None
    lo, hi = 1e-12, 1.0 - 1e-12   # ok(lo) is false, ok(hi) true
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if ok(mid):
            hi = mid
        else:
            lo = mid
    return hi


def lemma2_bucket_bound(n, p, s, rho=1.0):
    """ceil((1 + eps)(n - p + 1) / p) with the lemma's eps, or None."""
    eps = lemma2_epsilon(n, p, s, rho)
    if eps is None:
        return None
    return math.ceil((1.0 + eps) * (n - p + 1) / p)


def gvr_n_max(n, p, omega):
    """n_max = (1 + 1 / omega_n)(n / p), the bucket size GVR's choice of s
    keeps every bucket below with high probability."""
    return (1.0 + 1.0 / omega) * n / p


def default_omega_and_s(n):
    """The library's default oversampling: omega = ceil(lg lg n), s = 2
    omega^2 lg n (lg n rounded up), as in Algorithm 2's choice of s."""
    lg = max(1, math.ceil(math.log2(n)))
    w = max(1, math.ceil(math.log2(lg)))
    return w, 2 * w * w * lg
