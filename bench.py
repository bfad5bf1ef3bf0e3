#!/usr/bin/env python3
"""Throughput of the integer-sort hot path on one MI355X.

Workload: one stable sort of n = 2^27 uint32 keys drawn uniformly over the full
32-bit range (SplitMix64, seed 0x18081029202), keys only, with the radix-2^8
LSD sort (PR4 of arXiv 1808.10292, Section 3.2): one all-digit count kernel,
then per count-sort round a tile-count kernel, a tile-offset scan and a
rank-and-scatter kernel.  A step is one whole sort; inputs are resident in HBM
before timing starts and the output buffer is reused.

Printed as one JSON line:
  value        whole-sort Gkeys/s (n / seconds per step)
  roofline     the dominant kernel (the rank-and-scatter kernel of a round):
               algorithmic bytes per launch (read + write of every key,
               2 n 4 B) over its average
               duration from HIP events recorded on its stream during the timed
               steps, against MI355X's 8 TB/s; traffic = HBM bytes per launch
               from rocprofv3 FETCH_SIZE/WRITE_SIZE when the committed counter
               summary matches the current kernel source, else null
  cpu_baseline the CPU oracle (serial SR4 in C, one thread) on the same keys
  variants     other algorithms on the same keys (reported, not in value)
  batched      4096 lognormal arrays: batched segmented sort vs one plain
               sort per array, latency p50/p99, graph replay, the one-launch
               persistent mode
  kv           2^28 key-value pairs per key distribution: PR4 vs the
               regular-oversampling sample sort (GSD, p = 256, r = 32)
  small        2^20 keys uniform in [0, 2^31): per-call latency p50/p99
  serve        Poisson streams (rho = 0.5, 0.8 of the plain-launch capacity) and
               a saturated stream (every request at once) of mixed-size
               uint32/uint64 requests through the continuous-batching server:
               p50/p99 latency, keys/s against one plain launch per request,
               peak HBM in flight, alone == in the mix
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
METRIC = "Gkeys/s + % HBM roofline, 2^27 uint32; batched vs plain; p50/p99 latency"
ROUND_SAMPLE_PERIOD = 5   # time launches 0, 5, 10, ... of the scatter in the timed region
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_scatter_u32_keys_2p27_counters.md")
ROUND_SOURCE = os.path.join(ROOT, "paper_1808_10292_amd", "csrc", "lsd_r8.hip")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def source_sha():
    h = hashlib.sha256()
    for p in (ROUND_SOURCE, os.path.join(ROOT, "paper_1808_10292_amd", "csrc", "lsd_kernels.h"),
              os.path.join(ROOT, "paper_1808_10292_amd", "csrc", "device_common.h")):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic():
    """HBM bytes per round launch measured with rocprofv3 counters, if the
    summary was taken on the current kernel source."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    fields = {}
    for line in open(COUNTERS_FILE):
        if "=" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split("=", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("source_sha256_16") != source_sha():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


WARM_MS = 40.0   # the GPU's clocks take about 30 ms of work to recover from an idle gap


def time_steps(fn, steps, warmup, torch):
    """Seconds per call of fn over `steps` calls, after at least `warmup`
    calls and at least WARM_MS of device work."""
    t0 = time.perf_counter()
    done = 0
    while done < warmup or (time.perf_counter() - t0) * 1e3 < WARM_MS:
        fn()
        torch.cuda.synchronize()
        done += 1
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def bench_sample_only(rsort, torch, np, keygen, args):
    """GSD (p = 256, r = 32), GER and GVR (p = 256, s = 2 w^2 lg n) on
    2^kv-log2n uniform (uint32 key, uint32 payload = input index) pairs, one
    JSON line per sort; for profiling the sample sorts' kernels alone."""
    n = 1 << args.kv_log2n
    keys = keygen.kv_keys("uniform", n)
    dk = torch.from_numpy(keys).cuda()
    dv = torch.arange(n, dtype=torch.int32, device="cuda")
    ko = torch.empty_like(dk)
    vo = torch.empty_like(dv)
    fns = {"gsd": lambda: rsort.rsort_sample_sort(dk, ko, dv, vo, p=256, r=32),
           "ger": lambda: rsort.rsort_sample_sort_random(dk, ko, dv, vo, p=256, s=0, seed=11),
           "gvr": lambda: rsort.rsort_sample_sort_gvr(dk, ko, dv, vo, p=256, s=0, seed=12)}
    for name, fn in fns.items():
        sec = time_steps(fn, args.steps, args.warmup, torch)
        got = ko.cpu().numpy()
        print(json.dumps({"mode": "sample", "algo": name, "pairs": n, "ms": round(sec * 1e3, 4),
                          "sorted": bool(np.all(got[1:] >= got[:-1]))}), flush=True)


def bench_segmented_only(rsort, torch, np, keygen, args):
    """The batched segmented sort of the 4096 lognormal arrays (median 2^12,
    sigma 1.5, clipped to [16, 2^20]), uniform 32-bit keys, keys only, with the
    default configuration; for profiling its kernels alone."""
    sizes = keygen.lognormal_sizes(4096)
    off = keygen.offsets_from_sizes(sizes)
    keys = keygen.uniform_u32(int(off[-1]), keygen.SEED_SEGMENTS)
    dk = torch.from_numpy(keys).cuda()
    out = torch.empty_like(dk)
    sec = time_steps(lambda: rsort.rsort_segmented_sort(dk, out, off), args.steps, args.warmup,
                     torch)
    print(json.dumps({"mode": "segmented", "arrays": int(sizes.size), "keys": int(off[-1]),
                      "ms": round(sec * 1e3, 4)}), flush=True)


def bench_batched(rsort, torch, np, keygen, args):
    """Batched segmented sort vs one plain sort per array: 4096 arrays with
    lognormal sizes (median 2^12, sigma 1.5, clipped to [16, 2^20]), uniform
    32-bit keys, keys only."""
    sizes = keygen.lognormal_sizes(4096)
    off = keygen.offsets_from_sizes(sizes)
    total = int(off[-1])
    log("batched: %d arrays, %d keys" % (sizes.size, total))
    keys = keygen.uniform_u32(total, keygen.SEED_SEGMENTS)
    dk = torch.from_numpy(keys).cuda()
    out = torch.empty_like(dk)
    reps = max(5, args.steps // 2)
    # the small-segment sorters (radix rounds, BTN, OET) at the 4096-key split
    rsort.rsort_segmented_set_split(4096)
    sorter_ms = {}
    for name in ("radix", "btn", "oet"):
        rsort.rsort_segmented_set_small_sort(name)
        sorter_ms[name] = round(time_steps(lambda: rsort.rsort_segmented_sort(dk, out, off),
                                           reps, 1, torch) * 1e3, 3)
    split, tune_ms = rsort.rsort_segmented_tune(dk, out, off, reps=3)
    sorter = {v: k for k, v in rsort.SMALL_SORTS.items()}[rsort.rsort_segmented_get_small_sort()]
    tuned = rsort.rsort_segmented_get_config()
    # the one-launch persistent mode on the same batch (the tuner's other launch mode)
    rsort.rsort_segmented_set_launch("persistent")
    persist_s = time_steps(lambda: rsort.rsort_segmented_sort(dk, out, off), reps, 1, torch)
    rsort.rsort_synchronize()
    gotp = out.cpu().numpy()
    okp = all(np.array_equal(gotp[a:b], np.sort(keys[a:b])) for a, b in zip(off[:-1:97], off[1::97]))
    rsort.rsort_segmented_set_launch(tuned["launch"])
    # per-call latency: submit -> completion, one call at a time
    lat = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rsort.rsort_segmented_sort(dk, out, off)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    got = out.cpu().numpy()
    ok = all(bool(np.all(got[a:b][1:] >= got[a:b][:-1])) for a, b in zip(off[:-1:97], off[1::97]))
    batched = time_steps(lambda: rsort.rsort_segmented_sort(dk, out, off), reps, 2, torch)
    # the same call replayed from a HIP graph (a cooperative launch is not
    # captured: the rounds then stand in for a persistent pick)
    if tuned["launch"] == "persistent":
        rsort.rsort_segmented_set_launch("rounds")
    need = rsort.rsort_segmented_workspace_bytes(torch.uint32, False, off)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rsort.rsort_segmented_sort(dk, out, off, workspace=ws)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rsort.rsort_segmented_sort(dk, out, off, workspace=ws)
    graph = time_steps(g.replay, reps, 2, torch)
    rsort.rsort_segmented_set_launch(tuned["launch"])
    # one plain sort call per array, same stream
    bounds = [(int(a), int(b)) for a, b in zip(off[:-1], off[1:])]
    views = [(dk[a:b], out[a:b]) for a, b in bounds]

    def plain():
        for ki, ko in views:
            rsort.rsort_sort(ki, ko)
    plain_s = time_steps(plain, 2, 1, torch)
    lat_us = np.array(lat) * 1e6
    return {"workload": "4096 arrays, lognormal sizes (median 4096, sigma 1.5, clip [16, 2^20]), "
                        "uniform u32 keys, keys only",
            "keys": total, "split_small_max": split, "small_sorter": sorter,
            "tuned": {"split": tuned["split"], "small_sorter": sorter,
                      "tile_threads": tuned["tile_threads"], "radix_bits": tuned["radix_bits"],
                      "launch": tuned["launch"], "tune_ms": round(tune_ms, 3)},
            "persistent_launch_ms": round(persist_s * 1e3, 3),
            "persistent_launch_check": "segments equal np.sort (sampled)" if okp else "FAILED",
            "small_sorter_ms_at_split_4096": sorter_ms,
            "batched_ms": round(batched * 1e3, 3), "batched_gkeys_per_s": round(total / batched / 1e9, 3),
            "graph_replay_ms": round(graph * 1e3, 3),
            "graph_gkeys_per_s": round(total / graph / 1e9, 3),
            "plain_per_array_ms": round(plain_s * 1e3, 3),
            "plain_gkeys_per_s": round(total / plain_s / 1e9, 3),
            "speedup_batched_vs_plain": round(plain_s / batched, 2),
            "latency_us_p50": round(float(np.percentile(lat_us, 50)), 1),
            "latency_us_p99": round(float(np.percentile(lat_us, 99)), 1),
            "check": "segments sorted (sampled)" if ok else "FAILED"}


def identity_rounds(np, keys, digit_bits=8):
    """Rounds whose digit is the same for every key (skipped by the sort)."""
    diff = np.bitwise_or.reduce(keys ^ keys[0]) if keys.size else 0
    width = keys.dtype.itemsize * 8
    return [d for d in range(width // digit_bits)
            if (int(diff) >> (digit_bits * d)) & ((1 << digit_bits) - 1) == 0]


def bench_kv(rsort, torch, np, keygen, args):
    """Key-value sort, radix (PR4) against the sample sorts: regular
    oversampling (GSD, p = 256 buckets, oversampling factor r = 32) and the two
    random-oversampling ones (GER, GVR; p = 256, s = 2 w^2 lg n): 2^28 pairs by
    default (uint32 key, uint32 payload = input index) per key distribution."""
    n = 1 << args.kv_log2n
    res = {"workload": "2^%d (uint32 key, uint32 payload = input index) pairs; PR4 vs GSD "
                       "p=256 r=32 vs GER and GVR p=256 s=2w^2 lg n" % args.kv_log2n, "n": n,
           "algorithmic_bytes_per_pass": 2 * n * 8}
    dv = torch.arange(n, dtype=torch.int32, device="cuda")
    ko = torch.empty(n, dtype=torch.uint32, device="cuda")
    vo = torch.empty_like(dv)
    steps = max(3, args.steps // 4)
    for dist in args.kv_dists.split(","):
        log("kv %s: generating %d keys" % (dist, n))
        keys = keygen.kv_keys(dist, n)
        dk = torch.from_numpy(keys).cuda()
        skipped = identity_rounds(np, keys)
        row = {}
        fns = {"lsd8": lambda: rsort.rsort_sort(dk, ko, dv, vo, algo="lsd8"),
               "sample": lambda: rsort.rsort_sample_sort(dk, ko, dv, vo, p=256, r=32),
               "sample_random": lambda: rsort.rsort_sample_sort_random(dk, ko, dv, vo, p=256,
                                                                       s=0, seed=11),
               "sample_gvr": lambda: rsort.rsort_sample_sort_gvr(dk, ko, dv, vo, p=256, s=0,
                                                                 seed=12)}
        buckets = {}
        for algo, fn in fns.items():
            sec = time_steps(fn, steps, 1, torch)
            # spot check: sorted keys and payloads that point at their keys
            idx = np.random.default_rng(5).integers(0, n, 4096)
            ti = torch.from_numpy(idx).cuda()
            k_h = ko.view(torch.int32)[ti].cpu().numpy().view(np.uint32)
            v_h = vo[ti].cpu().numpy().view(np.uint32)
            ok = bool(np.array_equal(keys[v_h], k_h))
            head = ko[:1 << 20].cpu().numpy()
            ok = ok and bool(np.all(head[1:] >= head[:-1]))
            row[algo] = {"ms": round(sec * 1e3, 3), "gkeys_per_s": round(n / sec / 1e9, 3),
                         "check": "sampled ok" if ok else "FAILED"}
            if algo != "lsd8":
                buckets[algo] = int(rsort.rsort_sample_sort_stats()["bucket"].max())
        executed = 4 - len(skipped)
        row["lsd8"]["rounds_executed"] = executed
        if executed:
            row["lsd8"]["gbps_per_executed_pass"] = round(
                2 * n * 8 * executed / (row["lsd8"]["ms"] * 1e-3) / 1e9, 1)
        row["sample"]["max_bucket"] = buckets["sample"]
        row["sample"]["lemma1_bound"] = round((1 + 1 / 32) * n / 256 + 32 * 256, 1)
        row["sample_random"]["max_bucket"] = buckets["sample_random"]
        row["sample_gvr"]["max_bucket"] = buckets["sample_gvr"]
        res[dist] = row
        del dk
    return res


def bench_small(rsort, torch, np, keygen, args):
    """The small single-array sort: 2^20 keys uniform in [0, 2^31), keys only,
    PR4; per-call latency (launch to completion, one call at a time)."""
    n = 1 << 20
    keys = keygen.uniform_u31(n, keygen.SEED_SMALL)
    dk = torch.from_numpy(keys).cuda()
    out = torch.empty_like(dk)
    for _ in range(5):
        rsort.rsort_sort(dk, out)
    torch.cuda.synchronize()
    lat = []
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for _ in range(max(50, args.steps)):
        ev[0].record()
        rsort.rsort_sort(dk, out)
        ev[1].record()
        ev[1].synchronize()
        lat.append(ev[0].elapsed_time(ev[1]) * 1e3)
    lat = np.array(lat)
    ok = bool(np.all(np.diff(out.cpu().numpy().astype(np.int64)) >= 0))
    # the same sort captured once in a HIP graph and replayed (no per-kernel host launches)
    need = rsort.rsort_workspace_bytes(torch.uint32, False, n)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rsort.rsort_sort(dk, out, workspace=ws)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rsort.rsort_sort(dk, out, workspace=ws)
    glat = []
    for _ in range(max(50, args.steps)):
        ev[0].record()
        g.replay()
        ev[1].record()
        ev[1].synchronize()
        glat.append(ev[0].elapsed_time(ev[1]) * 1e3)
    glat = np.array(glat)
    ok = ok and bool(np.all(np.diff(out.cpu().numpy().astype(np.int64)) >= 0))
    res = {"workload": "2^20 keys uniform in [0, 2^31), keys only, PR4", "runs": int(lat.size),
           "us_p50": round(float(np.percentile(lat, 50)), 1),
           "us_p99": round(float(np.percentile(lat, 99)), 1),
           "gkeys_per_s_p50": round(n / (np.percentile(lat, 50) * 1e-6) / 1e9, 3),
           "graph_us_p50": round(float(np.percentile(glat, 50)), 1),
           "graph_us_p99": round(float(np.percentile(glat, 99)), 1),
           "check": "sorted" if ok else "FAILED"}
    if args.cpu_seconds > 0:
        import oracle
        t0 = time.perf_counter()
        oracle.sr4(keys)
        res["oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    return res


def bench_serve(rsort, torch, np, keygen, args):
    """Served sorting: Poisson streams of requests, sizes log-uniform in
    [2^10, 2^26] keys, key type 50% uint32 / 50% uint64 (uniform full range),
    admitted under a 64 GB HBM cap onto 4 streams and batched on arrival.  The
    rate is set to rho times what one plain launch per request sustains on the
    same mix.  Latency = submit to completion seen by the server."""
    num, warm = args.serve_requests, args.serve_warmup
    total_req = num + warm
    sizes = keygen.log_uniform_sizes(total_req, keygen.SEED_SERVE)
    u32 = keygen.unit_doubles(keygen.SEED_SERVE + 1, total_req) < 0.5
    # input arena of random 64-bit words; every request reads a window of it
    g = torch.Generator(device="cuda")
    g.manual_seed(keygen.SEED_SERVE + 3)
    arena = torch.randint(-2 ** 63, 2 ** 63 - 1, (1 << 27,), dtype=torch.int64, device="cuda",
                          generator=g)
    a64, a32 = arena.view(torch.uint64), arena.view(torch.uint32)
    offs = keygen.unit_doubles(keygen.SEED_SERVE + 4, total_req)

    def request_input(i):
        n = int(sizes[i])
        src = a32 if u32[i] else a64
        start = int(offs[i] * (src.numel() - n))
        return src[start:start + n]

    # output ring: a request's output region is reused only after its last user completed
    ring = torch.empty(8 << 30, dtype=torch.uint8, device="cuda")
    ring_users = []   # (start, end, ticket)
    ring_at = [0]

    def request_output(i, srv):
        nbytes = int(sizes[i]) * (4 if u32[i] else 8)
        start = (ring_at[0] + 255) // 256 * 256
        if start + nbytes > ring.numel():
            start = 0
        end = start + nbytes
        for (a, b, t) in list(ring_users):
            if a < end and start < b:
                srv.wait(t)
                ring_users.remove((a, b, t))
        ring_at[0] = end
        view = ring[start:end].view(torch.uint32 if u32[i] else torch.uint64)
        return view, (start, end)

    # capacity: one plain launch per request, back to back on one stream
    outs_plain = torch.empty(1 << 27, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(warm, total_req):
        x = request_input(i)
        o = outs_plain[:x.numel()].view(torch.uint64) if not u32[i] else \
            outs_plain.view(torch.uint32)[:x.numel()]
        rsort.rsort_sort(x, o)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    keys_meas = int(sizes[warm:].sum())
    cap_kps = keys_meas / plain_s
    mean_n = float(sizes[warm:].mean())
    res = {"workload": "Poisson stream, sizes log-uniform [2^10, 2^26], 50%% uint32 / 50%% "
                       "uint64, cap 64 GB, 4 streams; %d requests after %d warm-up" % (num, warm),
           "plain_launch_gkeys_per_s": round(cap_kps / 1e9, 3)}
    for rho in (0.5, 0.8, None):
        # rho None: every request submitted at once (closed loop, the server saturated)
        if rho is None:
            rate = float("inf")
            arrivals = np.zeros(total_req)
        else:
            rate = rho * cap_kps / mean_n
            arrivals = keygen.poisson_arrivals(total_req, rate, keygen.SEED_SERVE + 2)
        srv = rsort.Server(64 * 10 ** 9, num_streams=4)
        srv.reserve("u64", int(sizes.max()))   # slot workspaces allocated before traffic
        ring_users.clear()
        ring_at[0] = 0
        pick = set(int(j) for j in np.random.default_rng(1).choice(np.arange(warm, total_req), 16,
                                                                    replace=False))
        pick |= {warm + int(np.argmin(sizes[warm:])), warm + int(np.argmax(sizes[warm:]))}
        kept = {}
        t0 = time.perf_counter()
        tickets = []
        for i in range(total_req):
            if i == warm:
                for t in tickets:
                    srv.wait(t)
                ring_users.clear()   # all complete; their tickets are forgotten below
                srv.reset_stats()
                tickets = []
                t0 = time.perf_counter() - arrivals[warm]
            while time.perf_counter() - t0 < arrivals[i]:
                pass
            x = request_input(i)
            if i in pick:
                o = torch.empty_like(x)
                kept[i] = o
                tickets.append(srv.submit(x, o))
            else:
                o, (a, b) = request_output(i, srv)
                t = srv.submit(x, o)
                ring_users.append((a, b, t))
                tickets.append(t)
        for t in tickets:
            srv.wait(t)
        p50, p99, kps, done = srv.latency()
        _, max_in_flight, held = srv.memory()
        srv.destroy()
        same = True
        for i, o in kept.items():
            x = request_input(i)
            ref = torch.empty_like(x)
            rsort.rsort_sort(x, ref)
            torch.cuda.synchronize()
            same = same and bool(torch.equal(ref.view(torch.uint8), o.view(torch.uint8)))
        leg = {"rate_req_per_s": round(rate, 1) if rho is not None else "all at once",
               "completed": int(done),
               "latency_us_p50": round(p50, 1), "latency_us_p99": round(p99, 1),
               "gkeys_per_s": round(kps / 1e9, 3),
               "max_in_flight_gb": round(max_in_flight / 1e9, 3),
               "server_held_gb": round(held / 1e9, 3),
               "alone_equals_mix": "%d sampled requests %s" % (len(kept), "identical" if same
                                                                else "DIFFER")}
        if rho is not None:
            leg["offered_gkeys_per_s"] = round(keys_meas / (arrivals[-1] - arrivals[warm]) / 1e9, 3)
        else:
            res["served_gkeys_per_s"] = leg["gkeys_per_s"]
            res["served_vs_plain"] = round(kps / cap_kps, 3)
        res["saturated" if rho is None else "rho_%.1f" % rho] = leg
        log("serve %s: p50 %.0f us p99 %.0f us, %.2f Gkeys/s" %
            ("saturated" if rho is None else "rho %.1f" % rho, p50, p99, kps / 1e9))
    res["small_requests_frac"] = round(float((sizes <= 8192).mean()), 3)
    del ring, arena, outs_plain
    return res


def host_info():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu": model, "nproc": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # the GPU lowers its clocks whenever it idles; about 20 sorts of 2^27
    # keys (30 ms) pass before they are back at their steady rate
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--log2n", type=int, default=27)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum CPU time spent timing the oracle (0 disables)")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--kv-log2n", type=int, default=28)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--kv-dists", default="uniform,low16,zipf,equal,presorted,reverse",
                    help="comma list of key distributions for the key-value leg "
                         "(uniform, low16, zipf, equal, presorted, reverse)")
    ap.add_argument("--mode", choices=("sort", "copy", "pr2", "sample", "segmented", "small"),
                    default="sort",
                    help="copy: time the library's plain device copy of the same bytes "
                         "(calibrates rocprofv3 byte counters against a known transfer); "
                         "pr2: time only the radix-65536 sort of the same keys; "
                         "sample: only GSD, GER and GVR on 2^kv-log2n uniform key-value pairs; "
                         "segmented: only the batched segmented sort of the 4096 lognormal "
                         "arrays; small: only the 2^20-key latency leg (these four for "
                         "profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import keygen
    from paper_1808_10292_amd import rsort

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    rsort.load_library()
    if args.mode == "sample":
        bench_sample_only(rsort, torch, np, keygen, args)
        return
    if args.mode == "segmented":
        bench_segmented_only(rsort, torch, np, keygen, args)
        return
    if args.mode == "small":
        res = bench_small(rsort, torch, np, keygen, args)
        print(json.dumps(dict(mode="small", **res)), flush=True)
        return
    n = 1 << args.log2n
    log("generating %d keys" % n)
    keys = keygen.uniform_u32(n, keygen.SEED_LARGE)
    dk = torch.from_numpy(keys).cuda()
    out = torch.empty_like(dk)
    torch.cuda.synchronize()

    if args.mode == "copy":
        # begin_bit == end_bit: nothing to compare, the sort is a plain copy
        sec = time_steps(lambda: rsort.rsort_sort(dk, out, begin_bit=0, end_bit=0),
                         args.steps, args.warmup, torch)
        print(json.dumps({"mode": "copy", "bytes_moved": 2 * n * 4, "ms": round(sec * 1e3, 4),
                          "gbps": round(2 * n * 4 / sec / 1e9, 1)}), flush=True)
        return

    if args.mode == "pr2":
        sec = time_steps(lambda: rsort.rsort_sort(dk, out, algo="lsd16"), args.steps, args.warmup,
                         torch)
        got = out.cpu().numpy()
        print(json.dumps({"mode": "pr2", "keys": n, "ms": round(sec * 1e3, 4),
                          "gkeys_per_s": round(n / sec / 1e9, 3),
                          "sorted": bool(np.all(got[1:] >= got[:-1]))}), flush=True)
        return

    def step():
        rsort.rsort_sort(dk, out, algo="lsd8")

    log("timing %d steps after %d warm-up" % (args.steps, args.warmup))
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: HIP events on the launch stream around the dominant kernel
    # only, and around every fifth launch of it (every event pair delays the
    # stream; 5 against 4 rounds per sort samples each round equally often)
    rsort.rsort_profile_enable(True, kinds=[rsort.RSORT_KERNEL_ROUND])
    rsort.rsort_profile_set_period(ROUND_SAMPLE_PERIOD)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    launches, round_ms = rsort.rsort_profile_read(rsort.RSORT_KERNEL_ROUND)
    rsort.rsort_profile_enable(False)
    # the other kernels' durations, from a separate profiled pass
    rsort.rsort_profile_enable(True, kinds=[rsort.RSORT_KERNEL_HIST, rsort.RSORT_KERNEL_COUNT,
                                            rsort.RSORT_KERNEL_TILESCAN])
    for _ in range(max(3, args.steps // 4)):
        step()
    hl, hist_ms = rsort.rsort_profile_read(rsort.RSORT_KERNEL_HIST)
    cl, count_ms = rsort.rsort_profile_read(rsort.RSORT_KERNEL_COUNT)
    sl, scan_ms = rsort.rsort_profile_read(rsort.RSORT_KERNEL_TILESCAN)
    rsort.rsort_profile_enable(False)
    rsort.rsort_synchronize()

    # sanity: sorted, same multiset fingerprint as the input
    got = out.cpu().numpy()
    ok = bool(np.all(got[1:] >= got[:-1])) and \
        int(got.astype(np.uint64).sum()) == int(keys.astype(np.uint64).sum()) and \
        int(np.bitwise_xor.reduce(got)) == int(np.bitwise_xor.reduce(keys))
    if not ok:
        log("OUTPUT CHECK FAILED")

    # the library's plain copy of the same bytes: the achievable streaming rate
    copy_s = time_steps(lambda: rsort.rsort_sort(dk, out, begin_bit=0, end_bit=0), 10, 2, torch)
    copy_gbps = 2 * n * 4 / copy_s / 1e9
    rsort.rsort_sort(dk, out, algo="lsd8")
    torch.cuda.synchronize()

    round_avg_ms = round_ms / max(launches, 1)
    bytes_per_round = 2 * n * 4
    achieved = bytes_per_round / (round_avg_ms * 1e-3) / 1e9
    # a whole count-sort round: tile counts + scan of the counts + rank and scatter
    pass_ms = count_ms / max(cl, 1) + scan_ms / max(sl, 1) + round_avg_ms
    pass_gbps = bytes_per_round / (pass_ms * 1e-3) / 1e9
    gkeys = n / sec / 1e9
    traffic = committed_traffic()
    result = {
        "metric": METRIC,
        "value": round(gkeys, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic: uniform 32-bit keys from SplitMix64 (no dataset in the paper)",
        "config": {"workload": "lsd-r8 (PR4) stable sort of 2^%d uniform uint32 keys, keys only"
                               % args.log2n, "n": n, "key": "uint32", "payload": None,
                   "algo": "lsd_r8", "rounds": 4},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBPS, 4),
                     "pass_frac": round(pass_gbps / PEAK_HBM_GBPS, 4),
                     "traffic": traffic,
                     "kernel": "k_scatter<uint32, keys-only> (rank and route of one count-sort round)",
                     "algorithmic_bytes_per_launch": bytes_per_round,
                     "avg_launch_ms": round(round_avg_ms, 5), "timed_launches": launches,
                     "launches_in_timed_region": 4 * args.steps,
                     "copy_gbps": round(copy_gbps, 1),
                     "frac_of_copy": round(achieved / copy_gbps, 4)},
        "per_round_ms": {"count": round(count_ms / max(cl, 1), 5),
                         "tilescan": round(scan_ms / max(sl, 1), 5),
                         "scatter": round(round_avg_ms, 5),
                         "pass": round(pass_ms, 5), "pass_gbps": round(pass_gbps, 1),
                         "pass_frac": round(pass_gbps / PEAK_HBM_GBPS, 4)},
        "whole_sort": {"algorithmic_bytes": n * 4 + 4 * bytes_per_round,
                       "gbps": round((n * 4 + 4 * bytes_per_round) / sec / 1e9, 1),
                       "hist_kernel_ms": round(hist_ms / max(hl, 1), 5)},
        "output_check": "sorted+fingerprint " + ("ok" if ok else "FAILED"),
    }

    if not args.no_variants:
        # PR2 (radix 2^16, two rounds) on the same keys, with per-pass timings
        reps = max(3, args.steps // 4)
        s16 = time_steps(lambda: rsort.rsort_sort(dk, out, algo="lsd16"), reps, 1, torch)
        rsort.rsort_profile_enable(True)
        for _ in range(reps):
            rsort.rsort_sort(dk, out, algo="lsd16")
        parts = {}
        for name, kind in (("group_high_byte", rsort.RSORT_KERNEL_GROUP),
                           ("count_rows", rsort.RSORT_KERNEL_COUNT),
                           ("column_scan", rsort.RSORT_KERNEL_TILESCAN),
                           ("place", rsort.RSORT_KERNEL_ROUND)):
            cnt_l, ms = rsort.rsort_profile_read(kind)
            parts[name] = round(ms / max(cnt_l, 1), 5)
        rsort.rsort_profile_enable(False)
        got16 = out.cpu().numpy()
        pass_ms = sum(parts.values())
        result["variants"] = {"lsd16": {
            "algo": "PR2, radix 2^16, 2 rounds", "ms": round(s16 * 1e3, 3),
            "gkeys_per_s": round(n / s16 / 1e9, 3),
            "per_pass_ms": parts,
            "per_pass_gbps": round(2 * n * 4 / (pass_ms * 1e-3) / 1e9, 1),
            "place_kernel_gbps": round(2 * n * 4 / (parts["place"] * 1e-3) / 1e9, 1),
            "same_as_pr4": bool(np.array_equal(got16, got))}}
        # PR4 with single-read rounds (one counting pass, then one kernel per
        # round that counts, looks back inside its chain of tiles and routes)
        rsort.rsort_set_pr4_rounds("single_read")
        s1 = time_steps(step, reps, 30, torch)
        rsort.rsort_profile_enable(True)
        for _ in range(reps):
            step()
        parts1 = {}
        for name, kind in (("counting_pass", rsort.RSORT_KERNEL_HIST),
                           ("chain_plan", rsort.RSORT_KERNEL_TILESCAN),
                           ("round", rsort.RSORT_KERNEL_ROUND)):
            cnt_l, ms = rsort.rsort_profile_read(kind)
            parts1[name] = round(ms / max(cnt_l, 1), 5)
        rsort.rsort_profile_enable(False)
        got1 = out.cpu().numpy()
        rsort.rsort_set_pr4_rounds("counted")
        result["variants"]["lsd8_single_read"] = {
            "algo": "PR4, single-read rounds (look-back inside chains of tiles)",
            "ms": round(s1 * 1e3, 3), "gkeys_per_s": round(n / s1 / 1e9, 3),
            "per_sort_or_round_ms": parts1,
            "round_gbps": round(2 * n * 4 / (parts1["round"] * 1e-3) / 1e9, 1),
            "same_as_pr4": bool(np.array_equal(got1, got))}

    if not args.no_variants:
        result["small"] = bench_small(rsort, torch, np, keygen, args)
        result["batched"] = bench_batched(rsort, torch, np, keygen, args)
        del dk, out
        result["kv"] = bench_kv(rsort, torch, np, keygen, args)
        result["serve"] = bench_serve(rsort, torch, np, keygen, args)

    if args.cpu_seconds > 0:
        import oracle
        log("timing the CPU oracle for >= %.0f s" % args.cpu_seconds)
        runs, t = 0, 0.0
        while t < args.cpu_seconds or runs == 0:
            t0 = time.perf_counter()
            oracle.sr4(keys)
            t += time.perf_counter() - t0
            runs += 1
        result["cpu_baseline"] = {"value": round(n * runs / t / 1e9, 4), "unit": "Gkeys/s",
                                  "cores": 1, "kind": "oracle", "host": host_info(),
                                  "sample": "%d full runs of serial SR4 (C, one thread) on the "
                                            "same 2^%d keys, %.1f s" % (runs, args.log2n, t)}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
