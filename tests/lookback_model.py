"""Step-by-step CPU model of the decoupled look-back that turns per-block digit
totals into exclusive prefixes (the tile scan of a counted radix round, and
the chains of the single-read rounds).

Each workgroup is a generator that yields before every access to shared
memory, so a scheduler can interleave the accesses of all workgroups in any
order.  The protocol modelled, for one digit column:

* a workgroup first takes a ticket (an atomic counter): its position in the
  scan is the order in which workgroups start, not their launch index;
* it publishes its own total with the aggregate flag (position 0 publishes it
  as a prefix at once);
* it reads the words of its predecessors, nearest first, a window at a time
  (optionally the nearest alone first), adding every flagged count until it
  meets a prefix flag; a window that starts with an unflagged word is a spin;
* after ``spin_limit`` spins, or at its next check once the shared error
  word is set (the device checks every 256 spins, the model every spin), it sets the error word and stops looking back, so the grid
  always drains;
* it publishes its inclusive prefix with the prefix flag.

The words pack the flag into the top two bits and the count into the rest,
as the device does; the model keeps that encoding so that a count that would
reach the flag bits shows up.
"""
from __future__ import annotations

import random
from dataclasses import dataclass


@dataclass
class Encoding:
    flag_shift: int = 30

    @property
    def aggregate(self):
        return 1 << self.flag_shift

    @property
    def prefix(self):
        return 2 << self.flag_shift

    @property
    def count_mask(self):
        return (1 << self.flag_shift) - 1


@dataclass
class Shared:
    words: list
    ticket: int = 0
    err: int = 0
    reads: int = 0


def workgroup(sh: Shared, totals, enc: Encoding, window: int, spin_limit: int,
              use_tickets: bool, launch_index: int, first_single: bool, out: dict):
    """One workgroup of the scan; yields before each shared access."""
    yield
    if use_tickets:
        pos = sh.ticket
        sh.ticket += 1
    else:
        pos = launch_index
    total = totals[pos]
    yield
    sh.words[pos] = (enc.prefix if pos == 0 else enc.aggregate) | total
    excl = 0
    if pos > 0:
        j = pos            # words j-1, j-2, ... still to be folded
        spins = 0
        first = first_single
        while True:
            width = 1 if first else window
            first = False
            got = []
            for q in range(width):
                yield
                sh.reads += 1
                got.append(sh.words[j - 1 - q] if q < j else enc.prefix)
            used = 0
            done = False
            for q, w in enumerate(got):
                f = w >> enc.flag_shift
                if f == 0:
                    break
                excl += w & enc.count_mask
                used = q + 1
                if f == enc.prefix >> enc.flag_shift:
                    done = True
                    break
            if done:
                break
            j -= used
            if used == 0:
                spins += 1
                yield
                if spins > spin_limit or sh.err:
                    sh.err = 1
                    break
        yield
        sh.words[pos] = enc.prefix | ((excl + total) & enc.count_mask)
    out[pos] = excl


def run(totals, *, window=4, resident=4, launch_order=None, seed=0, spin_limit=64,
        use_tickets=True, first_single=False, stalled=None, enc=None, max_steps=10 ** 7):
    """Run the scan of ``totals`` under a random schedule.

    ``resident`` workgroups run at a time (the rest wait for a free slot, as
    workgroups wait for a compute unit); ``launch_order`` is the order in
    which they are dispatched; ``stalled`` names a launch index that, once it
    has taken its ticket, is never scheduled again.  Returns (exclusive prefixes by
    position, error word, steps taken)."""
    enc = enc or Encoding()
    n = len(totals)
    order = list(range(n)) if launch_order is None else list(launch_order)
    rng = random.Random(seed)
    sh = Shared(words=[0] * n)
    out = {}
    pending = list(order)
    live = []
    calls = {}
    steps = 0
    while pending or live:
        while pending and len(live) < resident:
            b = pending.pop(0)
            live.append((b, workgroup(sh, totals, enc, window, spin_limit, use_tickets, b,
                                      first_single, out)))
        # the stalled workgroup runs up to taking its ticket, then never again
        runnable = [x for x in live if x[0] != stalled or calls.get(x[0], 0) < 2]
        if not runnable:
            break          # only the stalled workgroup remains
        b, g = rng.choice(runnable)
        calls[b] = calls.get(b, 0) + 1
        steps += 1
        if steps > max_steps:
            raise RuntimeError("model did not drain")
        try:
            next(g)
        except StopIteration:
            live.remove((b, g))
    return out, sh.err, steps
