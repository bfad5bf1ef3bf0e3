// Host-only checks of the sort server's admission and batching policy
// (paper_1808_10292_amd/csrc/serve_sched.h), driven by a simulated executor.
// Exit status 0 and a final "OK" line mean every check passed.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <queue>
#include <random>
#include <set>
#include <vector>

#include "../paper_1808_10292_amd/csrc/serve_sched.h"

using rsort::ServeBatch;
using rsort::ServeRequest;
using rsort::ServeScheduler;

#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            exit(1);                                                      \
        }                                                                 \
    } while (0)

static ServeRequest req(uint64_t t, int kt, uint64_t n, uint64_t fp)
{
    ServeRequest r;
    r.ticket = t;
    r.key_type = kt;
    r.n = n;
    r.footprint = fp;
    return r;
}

static void batching_and_fifo()
{
    ServeScheduler s(1000, 2, 8192, 100);
    CHECK(!s.admissible(1001));
    CHECK(s.admissible(1000));
    s.push(req(1, 0, 100, 10));     // small u32: opens a batch
    s.push(req(2, 0, 100000, 500)); // large
    s.push(req(3, 0, 50, 10));      // small u32: joins batch 1
    s.push(req(4, 1, 50, 10));      // small u64: different key type
    s.push(req(5, 0, 8192, 10));    // small u32 at the limit: joins batch 1
    s.push(req(6, 0, 8193, 10));    // large by one key
    std::vector<ServeBatch> b = s.admit();
    CHECK(b.size() == 2);
    CHECK(b[0].small && b[0].key_type == 0 && b[0].reqs.size() == 3);
    CHECK(b[0].reqs[0].ticket == 1 && b[0].reqs[1].ticket == 3 && b[0].reqs[2].ticket == 5);
    CHECK(b[0].footprint == 30);
    CHECK(!b[1].small && b[1].reqs.size() == 1 && b[1].reqs[0].ticket == 2);
    CHECK(s.used() == 530 && s.busy_slots() == 2 && s.queued() == 2);
    CHECK(s.admit().empty());       // no free slot
    s.release(b[1].slot);
    b = s.admit();                  // ticket 4 (u64 small) is now the head
    CHECK(b.size() == 1 && b[0].small && b[0].key_type == 1 && b[0].reqs.size() == 1 &&
          b[0].reqs[0].ticket == 4);
    s.release(b[0].slot);
    b = s.admit();
    CHECK(b.size() == 1 && !b[0].small && b[0].reqs[0].ticket == 6);
    s.release(0);
    s.release(1);
    s.release(1);                   // releasing a free slot is ignored
    CHECK(s.used() == 0 && s.busy_slots() == 0 && s.queued() == 0);
}

static void memory_cap_blocks_in_order()
{
    ServeScheduler s(100, 4, 8192, 100);
    s.push(req(1, 0, 100000, 60));
    s.push(req(2, 0, 100000, 60));  // does not fit next to 1: waits
    s.push(req(3, 0, 10, 5));       // small, fits, but must not overtake 2
    std::vector<ServeBatch> b = s.admit();
    CHECK(b.size() == 1 && b[0].reqs[0].ticket == 1 && s.used() == 60);
    CHECK(s.admit().empty());
    s.release(b[0].slot);
    b = s.admit();
    CHECK(b.size() == 2);
    CHECK(b[0].reqs[0].ticket == 2 && b[1].reqs[0].ticket == 3);
    CHECK(s.used() == 65);
}

static void batch_limit_and_cap_inside_batch()
{
    ServeScheduler s(50, 1, 8192, 3);
    for (uint64_t t = 1; t <= 6; ++t) s.push(req(t, 0, 100, 10));
    std::vector<ServeBatch> b = s.admit();
    CHECK(b.size() == 1 && b[0].reqs.size() == 3);   // the batch size limit
    s.release(b[0].slot);
    ServeScheduler c(25, 1, 8192, 100);
    for (uint64_t t = 1; t <= 4; ++t) c.push(req(t, 0, 100, 10));
    b = c.admit();
    CHECK(b.size() == 1 && b[0].reqs.size() == 2 && c.used() == 20);   // the cap inside a batch
}

// A Poisson stream through a simulated device: each batch takes a fixed
// overhead plus time proportional to its bytes.  Checks the invariants at
// every event and that every request completes exactly once.
static void simulated_stream(uint64_t seed, int slots, uint64_t cap, int nreq, double rate)
{
    std::mt19937_64 rng(seed);
    std::exponential_distribution<double> gap(rate);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    struct Arrival {
        double t;
        ServeRequest r;
    };
    std::vector<Arrival> arr;
    double t = 0.0;
    for (int i = 0; i < nreq; ++i) {
        t += gap(rng);
        const int kt = u(rng) < 0.5 ? 0 : 1;
        const uint64_t n = (uint64_t)std::exp2(10.0 + 16.0 * u(rng));
        const uint64_t fp = n * (kt ? 8 : 4) * 3;
        ServeRequest r = req((uint64_t)i + 1, kt, n, fp);
        r.t_submit = t;
        arr.push_back({t, r});
    }
    ServeScheduler s(cap, slots, 8192, 1024);
    using Ev = std::pair<double, int>;   // completion time, slot
    std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> running;
    std::set<uint64_t> waiting, done;
    std::map<int, ServeBatch> in_slot;
    uint64_t last_head = 0;
    size_t next = 0;
    double now = 0.0;
    std::vector<double> lat;
    while (next < arr.size() || !running.empty() || s.queued()) {
        const double ta = next < arr.size() ? arr[next].t : 1e300;
        const double tc = running.empty() ? 1e300 : running.top().first;
        if (ta <= tc) {
            now = ta;
            if (s.admissible(arr[next].r.footprint)) {
                s.push(arr[next].r);
                waiting.insert(arr[next].r.ticket);
            } else {
                done.insert(arr[next].r.ticket);   // refused at submission
            }
            ++next;
        } else {
            now = tc;
            const int sl = running.top().second;
            running.pop();
            for (const ServeRequest& r : in_slot[sl].reqs) {
                CHECK(!done.count(r.ticket));
                done.insert(r.ticket);
                lat.push_back(now - r.t_submit);
            }
            in_slot.erase(sl);
            s.release(sl);
        }
        for (ServeBatch& b : s.admit()) {
            CHECK(!in_slot.count(b.slot));
            // the head is the oldest waiting request; members are not older
            CHECK(b.reqs[0].ticket == *waiting.begin());
            CHECK(b.reqs[0].ticket > last_head);
            last_head = b.reqs[0].ticket;
            uint64_t bytes = 0, fp = 0;
            for (const ServeRequest& r : b.reqs) {
                CHECK(waiting.erase(r.ticket) == 1);
                CHECK(r.ticket >= b.reqs[0].ticket);
                CHECK(r.key_type == b.key_type);
                CHECK(b.small == (r.n <= 8192));
                bytes += r.n * (r.key_type ? 8 : 4);
                fp += r.footprint;
            }
            CHECK(fp == b.footprint);
            CHECK(b.small || b.reqs.size() == 1);
            running.push({now + 20e-6 + (double)bytes * 8.0 / 4e12, b.slot});
            in_slot[b.slot] = b;
        }
        CHECK(s.used() <= s.cap());
        CHECK((int)s.busy_slots() <= slots);
        CHECK(s.busy_slots() == in_slot.size());
    }
    CHECK(done.size() == (size_t)nreq && waiting.empty() && s.used() == 0);
    std::sort(lat.begin(), lat.end());
    printf("stream seed=%llu slots=%d requests=%d p50_us=%.1f p99_us=%.1f\n",
           (unsigned long long)seed, slots, nreq, lat[lat.size() / 2] * 1e6,
           lat[(size_t)(0.99 * (double)(lat.size() - 1))] * 1e6);
}

int main()
{
    batching_and_fifo();
    memory_cap_blocks_in_order();
    batch_limit_and_cap_inside_batch();
    simulated_stream(1, 4, 64ull << 30, 2000, 2000.0);
    simulated_stream(2, 1, 64ull << 30, 500, 500.0);
    simulated_stream(3, 8, 1ull << 30, 2000, 20000.0);   // tight cap: requests above 1 GiB refused
    printf("OK\n");
    return 0;
}
