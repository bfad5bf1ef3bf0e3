"""Host checks of the sampling-lemma bound used by the GER / GVR tests: the
bisection's eps against the closed form of the quadratic the condition
reduces to, its monotonicity in s and rho, and the full-size numbers."""
import math

import pytest

from tests.lemma2 import (default_omega_and_s, gvr_n_max, lemma2_bucket_bound,
                          lemma2_epsilon, lemma2_rhs_factor)


def closed_form_eps(n, p, s, rho):
    # s >= (1 + e) L / e^2  <=>  (s / L) e^2 - e - 1 >= 0: the positive root
    a = s / lemma2_rhs_factor(n, p, s, rho)
    return (1.0 + math.sqrt(1.0 + 4.0 * a)) / (2.0 * a)


@pytest.mark.parametrize("n,p,s,rho", [(1 << 28, 256, 1400, 1.0), (1 << 20, 64, 500, 1.0),
                                       (1 << 24, 128, 2000, 2.0), (10 ** 7, 16, 3000, 0.5)])
def test_bisection_matches_closed_form(n, p, s, rho):
    e = lemma2_epsilon(n, p, s, rho)
    assert e is not None and 0 < e < 1
    assert abs(e - closed_form_eps(n, p, s, rho)) < 1e-9
    # the condition holds at eps and fails just below it
    L = lemma2_rhs_factor(n, p, s, rho)
    assert s >= (1 + e) / e ** 2 * L * (1 - 1e-12)
    assert s < (1 + e * 0.999) / (e * 0.999) ** 2 * L


def test_monotone_in_s_and_rho():
    n, p = 1 << 28, 256
    es = [lemma2_epsilon(n, p, s) for s in (700, 1400, 2800, 5600)]
    assert all(a > b for a, b in zip(es, es[1:]))
    er = [lemma2_epsilon(n, p, 1400, r) for r in (0.5, 1.0, 2.0)]
    assert all(a < b for a, b in zip(er, er[1:]))


def test_out_of_range_requests():
    assert lemma2_epsilon(1 << 20, 1, 100) is None            # p < 2
    assert lemma2_epsilon(1000, 64, 100) is None               # ps >= n / 2
    assert lemma2_epsilon(1 << 28, 256, 5) is None             # s too small for eps < 1


def test_full_size_numbers():
    """n = 2^28, p = 256 and the default s: omega = 5, s = 1400; eps about
    0.24, so every bucket stays within 1.24 n / p with probability at least
    1 - 2^-28; GVR's n_max = 1.2 n / p."""
    n, p = 1 << 28, 256
    w, s = default_omega_and_s(n)
    assert (w, s) == (5, 1400)
    e = lemma2_epsilon(n, p, s)
    assert 0.23 < e < 0.25
    b = lemma2_bucket_bound(n, p, s)
    assert b == math.ceil((1 + e) * (n - p + 1) / p)
    assert 1.23 * n / p < b < 1.25 * n / p
    assert gvr_n_max(n, p, w) == 1.2 * n / p
