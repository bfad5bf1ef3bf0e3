"""GPU tests of the sort server (continuous batching under an HBM cap).

Each served result is compared bit-exactly with the oracle's SR4 and with the
same request sorted alone by rsort_sort, for a mix of 32- and 64-bit keys
whose sizes cover the in-LDS batch classes (<= 1024, 4096, 8192 keys) and the
radix path (> 8192), submitted concurrently from several threads, in place
and out of place.  Also: refusal of a request larger than the cap, a cap small
enough that requests must wait for memory, poll / wait / statistics, and
destruction with requests still queued.
"""
import threading

import numpy as np
import pytest

import keygen
import oracle
from tests.gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 7, 100, 1000, 1024, 1025, 4096, 4097, 8191, 8192, 8193, 50000, 300001, 1 << 20]


@pytest.fixture(scope="module")
def rs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1808_10292_amd import rsort
    rsort.load_library()
    return rsort


def make_requests(seed, sizes):
    reqs = []
    for i, n in enumerate(sizes):
        if (seed + i) % 2:
            keys = keygen.uniform_u64(n, seed * 1000 + i)
            keys[::3] = keys[0]
        else:
            keys = keygen.zipf_keys(n, seed * 1000 + i)
        reqs.append(keys)
    return reqs


def alone(rs, keys):
    import torch
    d = dev(keys)
    o = torch.empty_like(d)
    rs.rsort_sort(d, o)
    rs.rsort_synchronize()
    return host(o)


def test_mix_equals_alone_and_oracle(rs):
    import torch
    sizes = SIZES * 3
    reqs = make_requests(3, sizes)
    announce("server mix", len(reqs))
    srv = rs.Server(64 << 30, num_streams=4)
    ins = [dev(k) for k in reqs]
    outs = [torch.empty_like(d) for d in ins]
    tickets = [None] * len(reqs)
    in_place = [i % 5 == 4 for i in range(len(reqs))]

    def worker(part):
        for i in range(part, len(reqs), 4):
            tickets[i] = srv.submit(ins[i], ins[i] if in_place[i] else outs[i])

    threads = [threading.Thread(target=worker, args=(p,)) for p in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for t in tickets:
        srv.wait(t)
    p50, p99, kps, done = srv.latency()
    assert done == len(reqs) and p99 >= p50 > 0 and kps > 0
    for i, keys in enumerate(reqs):
        got = host(ins[i] if in_place[i] else outs[i])
        want = oracle.sr4(keys)[0]
        assert np.array_equal(got, want), (i, keys.size)
        assert np.array_equal(got, alone(rs, keys)), (i, keys.size)
    srv.destroy()


def test_cap_refusal_and_waiting_for_memory(rs):
    import torch
    n = 1 << 20
    announce("server cap")
    # footprint of a 2^20-key u32 request: in + out (8 MiB) + workspace (> 4 MiB)
    srv = rs.Server(20 << 20, num_streams=4)
    big = dev(keygen.uniform_u32(4 << 20, 1))
    with pytest.raises(rs.RsortError) as e:
        srv.submit(big, torch.empty_like(big))
    assert e.value.status == rs.RSORT_ENOMEM
    reqs = [keygen.uniform_u32(n, 10 + i) for i in range(6)]   # at most one fits at a time
    ins = [dev(k) for k in reqs]
    outs = [torch.empty_like(d) for d in ins]
    ts = [srv.submit(a, b) for a, b in zip(ins, outs)]
    for t in ts:
        srv.wait(t)
    for k, o in zip(reqs, outs):
        assert np.array_equal(host(o), oracle.sr4(k)[0])
    srv.destroy()


def test_poll_stats_reset_and_empty(rs):
    import torch
    announce("server poll")
    srv = rs.Server(1 << 30, num_streams=2)
    keys = keygen.uniform_u32(100000, 5)
    d = dev(keys)
    o = torch.empty_like(d)
    t = srv.submit(d, o)
    while not srv.poll(t):
        pass
    assert np.array_equal(host(o), oracle.sr4(keys)[0])
    assert srv.latency()[3] == 1
    srv.reset_stats()
    assert srv.latency()[3] == 0
    e = torch.empty(0, dtype=torch.uint32, device="cuda")
    t0 = srv.submit(e, e)
    assert srv.poll(t0)
    with pytest.raises(rs.RsortError):
        srv.poll(123456789)
    srv.destroy()


def test_destroy_drains_queued_requests(rs):
    import torch
    announce("server drain")
    srv = rs.Server(64 << 30, num_streams=2)
    reqs = make_requests(9, [5000, 70000, 300, 1 << 19, 8192, 12345] * 4)
    ins = [dev(k) for k in reqs]
    outs = [torch.empty_like(d) for d in ins]
    for a, b in zip(ins, outs):
        srv.submit(a, b)
    srv.destroy()   # returns after every request has completed
    torch.cuda.synchronize()
    for k, o in zip(reqs, outs):
        assert np.array_equal(host(o), oracle.sr4(k)[0])


def test_device_failure_completes_with_edevice(rs):
    """A sort whose slot error word is set (as a look-back that gave up would
    set it) completes with RSORT_EDEVICE; the next request is unaffected."""
    import torch
    announce("server failure path")
    srv = rs.Server(1 << 30, num_streams=2)
    keys = keygen.uniform_u32(100000, 31)
    d = dev(keys)
    o = torch.empty_like(d)
    srv.fail_next()
    t = srv.submit(d, o)
    with pytest.raises(rs.RsortError) as e:
        srv.wait(t)
    assert e.value.status == rs.RSORT_EDEVICE
    o2 = torch.empty_like(d)
    srv.wait(srv.submit(d, o2))
    assert np.array_equal(host(o2), oracle.sr4(keys)[0])
    srv.destroy()


def test_submit_waits_for_the_producing_stream(rs):
    """keys_in is written on a side stream behind slow work; the request is
    submitted at once, without a host synchronisation, and must see the keys."""
    import torch
    announce("server stream order")
    srv = rs.Server(1 << 30, num_streams=2)
    n = 1 << 20
    keys = keygen.uniform_u32(n, 32)
    src = dev(keys)
    side = torch.cuda.Stream()
    junk = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
    results = []
    for rep in range(3):
        kin = torch.zeros(n, dtype=torch.uint32, device="cuda")
        out = torch.empty_like(kin)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            for _ in range(20):        # about a millisecond of work ahead of the copy
                junk.mul_(1.0000001)
            kin.copy_(src)
            t = srv.submit(kin, out)  # ordered after the copy on `side`
        srv.wait(t)
        results.append(host(out))
    want = oracle.sr4(keys)[0]
    for got in results:
        assert np.array_equal(got, want)
    srv.destroy()


def test_reserve_and_memory_accounting(rs):
    import torch
    announce("server reserve")
    srv = rs.Server(1 << 32, num_streams=3)
    srv.reserve("u64", 1 << 20)
    inflight, peak, held = srv.memory()
    assert inflight == 0 and peak == 0
    assert held >= 3 * 8 * (1 << 20)   # each slot: at least the temporary keys of 2^20 u64
    reqs = make_requests(12, [1 << 20, 300001, 5000, 1 << 19])
    ins = [dev(k) for k in reqs]
    outs = [torch.empty_like(d) for d in ins]
    ts = [srv.submit(a, b) for a, b in zip(ins, outs)]
    for t in ts:
        srv.wait(t)
    for k, o in zip(reqs, outs):
        assert np.array_equal(host(o), oracle.sr4(k)[0])
    inflight, peak, held2 = srv.memory()
    assert inflight == 0 and peak > 0 and held2 == held   # nothing grew past the reservation
    srv.reset_stats()
    assert srv.memory()[1] == 0
    srv.destroy()
