"""Host tests of the look-back protocol on a step-by-step CPU model
(tests/lookback_model.py) that uses the device's constants: the flag encoding,
the window widths of the counted and single-read rounds, and the largest
supported key count, read from the library's sources."""
import itertools
import os
import random
import re

import numpy as np
import pytest

from tests import lookback_model as lm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1808_10292_amd", "csrc")


def _const(fname, pattern):
    with open(os.path.join(CSRC, fname)) as f:
        m = re.search(pattern, f.read())
    assert m, (fname, pattern)
    return int(m.group(1))


FLAG_SHIFT = _const("device_common.h", r"kFlagShift\s*=\s*(\d+)")
LB_WINDOW = _const("lsd_kernels.h", r"#define LB_WINDOW (\d+)")
OS_WINDOW = _const("onesweep_kernels.h", r"kOsWindow\s*=\s*(\d+)")
MAX_N_LOG2 = _const("api.hip", r"kMaxN\s*=\s*\(size_t\)1 << (\d+)")
ENC = lm.Encoding(FLAG_SHIFT)


def exclusive(totals):
    return [int(x) for x in np.concatenate([[0], np.cumsum(totals)[:-1]])]


@pytest.mark.parametrize("window,first_single", [(1, False), (2, False), (LB_WINDOW, False),
                                                 (OS_WINDOW, True)])
def test_prefixes_under_random_schedules(window, first_single):
    rng = random.Random(window * 7 + first_single)
    for trial in range(60):
        n = rng.choice([1, 2, 3, 5, 8, 13, 31, 64])
        totals = [rng.choice([0, 0, 1, rng.randrange(1 << 20)]) for _ in range(n)]
        order = list(range(n))
        if trial % 3 == 1:
            rng.shuffle(order)
        resident = rng.choice([1, 2, 4, n])
        out, err, _ = lm.run(totals, window=window, resident=resident, launch_order=order,
                             seed=trial, first_single=first_single, enc=ENC)
        assert err == 0
        assert [out[i] for i in range(n)] == exclusive(totals), (n, resident, trial)


def test_tickets_make_any_dispatch_order_safe():
    """One resident workgroup, dispatched last-first: positions follow the
    order in which workgroups start, so no workgroup waits on one that cannot
    run."""
    totals = list(range(1, 41))
    for resident in (1, 2, 3):
        out, err, _ = lm.run(totals, resident=resident, launch_order=list(range(39, -1, -1)),
                             seed=resident, enc=ENC)
        assert err == 0 and [out[i] for i in range(40)] == exclusive(totals)


def test_launch_index_positions_would_time_out_and_drain():
    """The same dispatch with the launch index as position: the first
    workgroup to run waits on ones that cannot start, gives up after the spin
    limit, and every later one gives up at once; the error word is set and
    every workgroup still finishes."""
    totals = [3] * 12
    out, err, steps = lm.run(totals, resident=1, launch_order=list(range(11, -1, -1)),
                             use_tickets=False, spin_limit=50, enc=ENC)
    assert err == 1 and len(out) == 12 and steps < 10 ** 5


@pytest.mark.parametrize("stalled", [0, 5, 18])
def test_a_stalled_workgroup_sets_the_error_and_the_grid_drains(stalled):
    totals = [7] * 20
    out, err, _ = lm.run(totals, resident=20, seed=stalled, stalled=stalled, spin_limit=40,
                         enc=ENC)
    # everyone but the stalled workgroup finishes; those before its position
    # are exact, and the error word is set unless the stalled one was last
    assert len(out) == 19
    pos_stalled = next(i for i in range(20) if i not in out)
    for i in range(pos_stalled):
        assert out[i] == 7 * i
    assert err == (1 if pos_stalled < 19 else 0)


def test_flag_encoding_holds_every_supported_count():
    """A digit count is at most the number of keys, below 2^MAX_N_LOG2; the
    count field must hold it (and a whole round's prefix) without touching
    the flag bits."""
    assert (1 << MAX_N_LOG2) - 1 <= ENC.count_mask
    assert ENC.aggregate >> FLAG_SHIFT == 1 and ENC.prefix >> FLAG_SHIFT == 2
    big = ENC.count_mask // 4
    totals = [big, big, big, ENC.count_mask - 3 * big]
    out, err, _ = lm.run(totals, resident=4, seed=3, enc=ENC)
    assert err == 0 and [out[i] for i in range(4)] == exclusive(totals)
    # one more key than the field holds changes the last prefix: the limit
    # on the key count is what keeps the encoding exact
    totals2 = totals + [1, 0]
    out2, _, _ = lm.run(totals2, resident=1, seed=3, enc=ENC)
    assert out2[5] != sum(totals2[:5])


def test_reads_per_workgroup_when_predecessors_are_done():
    """Run one at a time in order: every workgroup finds its nearest
    predecessor's prefix in the first word it reads (one window, or the
    single first read of the single-read rounds)."""
    for window, first in itertools.product((LB_WINDOW,), (False, True)):
        out, err, _ = lm.run([1] * 16, window=window, resident=1, first_single=first, enc=ENC)
        assert err == 0 and [out[i] for i in range(16)] == list(range(16))
