// Sort server: a request loop over the library's sorts with continuous
// batching.  Clients submit device-resident key arrays from any thread; one
// scheduling thread admits them under an HBM footprint cap onto a fixed set
// of streams (serve_sched.h holds the policy), launches them, and watches
// their completion events.  Requests that arrive while others run are
// admitted as soon as a stream slot and memory free up, so their work
// overlaps on the device.
//
//   small requests (<= 8192 keys) of one key type are packed into one launch
//   of k_serve_small: one workgroup per request sorts it whole in LDS, one
//   8-bit count-sort round per digit (SR4, arXiv 1808.10292 Section 3.2);
//   larger requests run alone through the PR4 sort on their slot's stream.
//
// Every request's result is the stable sort of its keys, whatever else runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <iterator>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/rsort.h"
#include "rsort_internal.h"
#include "serve_sched.h"
#include "tile_sort.h"

namespace rsort {
namespace {

constexpr uint64_t kServeSmallMax = 8192;   // in-LDS capacity of the largest class
constexpr size_t kServeMaxBatch = 65536;

struct ServeDesc {
    const void* in;
    void* out;
    uint32_t len;
    uint32_t pad[3];
};

struct ServeClass {
    int wg, items;
};
constexpr ServeClass kServeClasses[3] = {{256, 4}, {512, 8}, {512, 16}};

int serve_class(uint64_t n)
{
    for (int c = 0; c < 3; ++c)
        if (n <= (uint64_t)kServeClasses[c].wg * kServeClasses[c].items) return c;
    return 2;
}

template <typename K, int WG, int ITEMS>
__global__ __launch_bounds__(WG) void k_serve_small(const ServeDesc* descs)
{
    __shared__ TileSmem<K, false, WG, ITEMS, true> sm;
    const ServeDesc d = descs[blockIdx.x];
    const K* in = (const K*)d.in;
    K* out = (K*)d.out;
    const uint32_t len = d.len;
    const uint32_t hofs = (threadIdx.x >> 5) * ITEMS * 32 + (threadIdx.x & 31);
    K k[ITEMS];
    uint32_t v[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t o = hofs + i * 32;
        k[i] = o < len ? in[o] : K(0);
        v[i] = 0;
    }
    for (uint32_t r = 0; r < sizeof(K); ++r) tile_round<K, false, WG, ITEMS>(sm, k, v, len, 8u * r, 0xFFu);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t o = hofs + i * 32;
        if (o < len) out[o] = k[i];
    }
}

template <typename K>
void launch_serve_small(int cls, const ServeDesc* d, uint32_t count, hipStream_t s)
{
    if (!count) return;
    switch (cls) {
    case 0: hipLaunchKernelGGL((k_serve_small<K, 256, 4>), dim3(count), dim3(256), 0, s, d); break;
    case 1: hipLaunchKernelGGL((k_serve_small<K, 512, 8>), dim3(count), dim3(512), 0, s, d); break;
    default: hipLaunchKernelGGL((k_serve_small<K, 512, 16>), dim3(count), dim3(512), 0, s, d); break;
    }
}

// Clears a slot's error word in stream order (a kernel, not a memset, so the
// sequence can sit in a captured graph).
__global__ void k_serve_clear(uint32_t* w)
{
    w[threadIdx.x] = 0;
}

// Sets a failure bit in a slot's error word (rsort_server_fail_next).
__global__ void k_serve_flag(uint32_t* w, uint32_t bits)
{
    w[0] |= bits;
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    uint32_t* err_dev = nullptr;    // device error word of this slot's sorts
    uint32_t* err_host = nullptr;   // pinned copy, written before `done` completes
    ServeDesc* desc_host = nullptr;   // pinned
    ServeDesc* desc_dev = nullptr;
    size_t desc_cap = 0;
    bool busy = false;
    ServeBatch batch;
    int status = RSORT_OK;
};

struct TicketState {
    bool done = false;
    int status = RSORT_OK;
};

}  // namespace
}  // namespace rsort

struct rsort_server {
    int device = 0;
    rsort::ServeScheduler sched;
    std::vector<rsort::Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work;   // submissions, stop
    std::condition_variable cv_done;   // completions
    std::thread worker;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::unordered_map<uint64_t, rsort::TicketState> tickets;
    std::vector<hipEvent_t> free_events;   // input-ready events of finished requests
    std::atomic<int> fail_next{0};         // rsort_server_fail_next
    std::vector<double> latency_s;
    uint64_t keys_done = 0;
    double t_first = 0.0, t_last = 0.0;

    rsort_server(int dev, uint64_t cap, int nslots)
        : device(dev), sched(cap, nslots, rsort::kServeSmallMax, rsort::kServeMaxBatch),
          slots((size_t)nslots)
    {
    }
};

namespace rsort {
namespace {

uint64_t request_footprint(int kb, uint64_t n, bool in_place)
{
    const uint64_t bufs = (in_place ? 1u : 2u) * n * (uint64_t)kb;
    if (n <= kServeSmallMax) return bufs + sizeof(ServeDesc);
    return bufs + lsd_r8_layout(kb, false, (size_t)n, 0, 8 * kb).bytes;
}

hipError_t grow(void** p, size_t* have, size_t need)
{
    if (need <= *have) return hipSuccess;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *have = 0;
    hipError_t e = dev_malloc(p, need);
    if (e == hipSuccess) *have = need;
    return e;
}

// Enqueue one admitted batch on its slot's stream (scheduling thread only).
int launch_batch(rsort_server* sv, Slot& sl)
{
    const ServeBatch& b = sl.batch;
    const int kb = b.key_type == RSORT_U64 ? 8 : 4;
    hipError_t e = hipSuccess;
    // nothing of the batch starts before its inputs are written
    for (const ServeRequest& r : b.reqs)
        if (r.ready && hipStreamWaitEvent(sl.stream, (hipEvent_t)r.ready, 0) != hipSuccess)
            return RSORT_EDEVICE;
    *sl.err_host = 0;
    if (b.small) {
        const size_t cnt = b.reqs.size();
        if (cnt > sl.desc_cap) {
            if (sl.desc_host) (void)hipHostFree(sl.desc_host);
            if (sl.desc_dev) (void)hipFree(sl.desc_dev);
            sl.desc_host = nullptr;
            sl.desc_dev = nullptr;
            sl.desc_cap = 0;
            const size_t cap = std::max<size_t>(cnt, 1024);
            e = hipHostMalloc((void**)&sl.desc_host, cap * sizeof(ServeDesc), hipHostMallocDefault);
            if (e == hipSuccess) e = dev_malloc((void**)&sl.desc_dev, cap * sizeof(ServeDesc));
            if (e != hipSuccess) return RSORT_ENOMEM;
            sl.desc_cap = cap;
        }
        // descriptors grouped by capacity class
        uint32_t count[3] = {0, 0, 0};
        for (const ServeRequest& r : b.reqs) ++count[serve_class(r.n)];
        uint32_t at[3] = {0, count[0], count[0] + count[1]};
        const uint32_t first[3] = {at[0], at[1], at[2]};
        for (const ServeRequest& r : b.reqs) {
            ServeDesc& d = sl.desc_host[at[serve_class(r.n)]++];
            d.in = r.keys_in;
            d.out = r.keys_out;
            d.len = (uint32_t)r.n;
        }
        // the pinned descriptors are rewritten only after this slot's previous
        // batch completed, so the copy below never races with a reuse
        e = hipMemcpyAsync(sl.desc_dev, sl.desc_host, cnt * sizeof(ServeDesc), hipMemcpyHostToDevice,
                           sl.stream);
        if (e != hipSuccess) return RSORT_EDEVICE;
        for (int c = 0; c < 3; ++c) {
            if (kb == 4)
                launch_serve_small<uint32_t>(c, sl.desc_dev + first[c], count[c], sl.stream);
            else
                launch_serve_small<uint64_t>(c, sl.desc_dev + first[c], count[c], sl.stream);
        }
        e = hipGetLastError();
    } else {
        const ServeRequest& r = b.reqs[0];
        const LsdR8Layout L = lsd_r8_layout(kb, false, (size_t)r.n, 0, 8 * kb);
        e = grow(&sl.ws, &sl.ws_bytes, L.bytes);   // no-op for requests within the reservation
        if (e != hipSuccess) return RSORT_ENOMEM;
        hipLaunchKernelGGL(k_serve_clear, dim3(1), dim3(64), 0, sl.stream, sl.err_dev);
        e = lsd_r8_sort(kb, r.keys_in, r.keys_out, nullptr, nullptr, (size_t)r.n, 0, 8 * kb, sl.ws, L,
                        sl.err_dev, sl.stream, nullptr);
        if (e == hipSuccess && sv->fail_next.exchange(0))
            hipLaunchKernelGGL(k_serve_flag, dim3(1), dim3(1), 0, sl.stream, sl.err_dev,
                               (uint32_t)kErrLookbackTimeout);
        // the slot's error word comes back with the batch (read once `done` completes)
        if (e == hipSuccess)
            e = hipMemcpyAsync(sl.err_host, sl.err_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, sl.stream);
    }
    if (e != hipSuccess) return RSORT_EDEVICE;
    e = hipEventRecord(sl.done, sl.stream);
    return e == hipSuccess ? RSORT_OK : RSORT_EDEVICE;
}

void worker_main(rsort_server* sv)
{
    (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        // admit and launch
        std::vector<ServeBatch> admitted = sv->sched.admit();
        lk.unlock();
        for (ServeBatch& b : admitted) {
            Slot& sl = sv->slots[(size_t)b.slot];
            sl.batch = std::move(b);
            sl.busy = true;
            sl.status = launch_batch(sv, sl);
        }
        // completions
        std::vector<int> finished;
        bool running = false;
        for (size_t i = 0; i < sv->slots.size(); ++i) {
            Slot& sl = sv->slots[i];
            if (!sl.busy) continue;
            if (sl.status != RSORT_OK) {
                (void)hipStreamSynchronize(sl.stream);   // nothing may still read the slot
                finished.push_back((int)i);
                continue;
            }
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                // a look-back wait of the sort gave up: its output is not the stable sort
                if (*sl.err_host) sl.status = RSORT_EDEVICE;
                finished.push_back((int)i);
            } else if (q == hipErrorNotReady) {
                running = true;
            } else {
                sl.status = RSORT_EDEVICE;
                finished.push_back((int)i);
            }
        }
        const double t = now_s();
        lk.lock();
        for (int i : finished) {
            Slot& sl = sv->slots[(size_t)i];
            for (const ServeRequest& r : sl.batch.reqs) {
                if (r.ready) sv->free_events.push_back((hipEvent_t)r.ready);
                TicketState& ts = sv->tickets[r.ticket];
                ts.done = true;
                ts.status = sl.status;
                if (sl.status == RSORT_OK) {
                    sv->latency_s.push_back(t - r.t_submit);
                    sv->keys_done += r.n;
                }
            }
            sv->t_last = t;
            sl.busy = false;
            sl.batch.reqs.clear();
            sv->sched.release(i);
        }
        if (!finished.empty()) sv->cv_done.notify_all();
        if (sv->stop && !running && sv->sched.queued() == 0 && sv->sched.busy_slots() == 0) break;
        if (!finished.empty() || !admitted.empty()) continue;
        if (running) {
            // poll the running batches' events without a timed sleep (a timed
            // wait oversleeps by tens of microseconds on a loaded host)
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            sv->cv_work.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

bool device_ptr(const void* p, int device)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice && a.device == device;
}

}  // namespace
}  // namespace rsort

extern "C" {

int rsort_server_create(int hip_device, size_t hbm_cap_bytes, int num_streams, rsort_server** out)
{
    if (!out) return RSORT_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count)
        return RSORT_EINVAL;
    if (num_streams < 1 || num_streams > 64 || hbm_cap_bytes == 0) return RSORT_EINVAL;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(hip_device);
    rsort_server* sv = new (std::nothrow) rsort_server(hip_device, hbm_cap_bytes, num_streams);
    int rc = RSORT_OK;
    if (!sv) {
        rc = RSORT_ENOMEM;
    } else {
        for (rsort::Slot& sl : sv->slots) {
            if (rc) break;
            if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
                rc = RSORT_EDEVICE;
                break;
            }
            // error word and the descriptors of the largest small-request batch,
            // so that the scheduling thread never allocates for them
            const size_t dbytes = rsort::kServeMaxBatch * sizeof(rsort::ServeDesc);
            if (rsort::dev_malloc((void**)&sl.err_dev, 256) != hipSuccess ||
                hipHostMalloc((void**)&sl.err_host, 256, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc((void**)&sl.desc_host, dbytes, hipHostMallocDefault) != hipSuccess ||
                rsort::dev_malloc((void**)&sl.desc_dev, dbytes) != hipSuccess) {
                rc = RSORT_ENOMEM;
                break;
            }
            *sl.err_host = 0;
            sl.desc_cap = rsort::kServeMaxBatch;
        }
        if (!rc) {
            try {
                sv->worker = std::thread(rsort::worker_main, sv);
            } catch (...) {
                rc = RSORT_ENOMEM;
            }
        }
        if (rc) {
            for (rsort::Slot& sl : sv->slots) {
                if (sl.stream) (void)hipStreamDestroy(sl.stream);
                if (sl.done) (void)hipEventDestroy(sl.done);
                if (sl.err_dev) (void)hipFree(sl.err_dev);
                if (sl.err_host) (void)hipHostFree(sl.err_host);
                if (sl.desc_host) (void)hipHostFree(sl.desc_host);
                if (sl.desc_dev) (void)hipFree(sl.desc_dev);
            }
            delete sv;
            sv = nullptr;
        }
    }
    (void)hipSetDevice(prev);
    *out = sv;
    return rc;
}

int rsort_server_submit_async(rsort_server* sv, int key_type, const void* keys_in, void* keys_out,
                              size_t n, void* stream, uint64_t* ticket)
{
    if (!sv || !ticket) return RSORT_EINVAL;
    if (key_type != RSORT_U32 && key_type != RSORT_U64) return RSORT_EINVAL;
    if (n >= ((size_t)1 << 30)) return RSORT_EUNSUPPORTED;
    const int kb = key_type == RSORT_U64 ? 8 : 4;
    if (n) {
        if (!keys_in || !keys_out) return RSORT_EINVAL;
        if (!rsort::device_ptr(keys_in, sv->device) || !rsort::device_ptr(keys_out, sv->device))
            return RSORT_EINVAL;
        const char* a = (const char*)keys_in;
        const char* b = (const char*)keys_out;
        if (a != b && a < b + n * kb && b < a + n * kb) return RSORT_EINVAL;
    }
    rsort::ServeRequest r;
    r.key_type = key_type;
    r.n = n;
    r.keys_in = keys_in;
    r.keys_out = keys_out;
    r.footprint = rsort::request_footprint(kb, n, keys_in == keys_out);
    if (!sv->sched.admissible(r.footprint)) return RSORT_ENOMEM;
    if (n) {
        // mark the point of `stream` the sort must wait for: everything enqueued
        // there so far (the writes of keys_in, earlier uses of keys_out)
        hipEvent_t ev = nullptr;
        {
            std::lock_guard<std::mutex> g(sv->mu);
            if (!sv->free_events.empty()) {
                ev = sv->free_events.back();
                sv->free_events.pop_back();
            }
        }
        int prev = 0;
        (void)hipGetDevice(&prev);
        if (prev != sv->device) (void)hipSetDevice(sv->device);
        hipError_t e = ev ? hipSuccess : hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ev, (hipStream_t)stream);
        if (prev != sv->device) (void)hipSetDevice(prev);
        if (e != hipSuccess) {
            if (ev) {
                std::lock_guard<std::mutex> g(sv->mu);
                sv->free_events.push_back(ev);
            }
            return RSORT_EDEVICE;
        }
        r.ready = ev;
    }
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->stop) {
        if (r.ready) sv->free_events.push_back((hipEvent_t)r.ready);
        return RSORT_EBUSY;
    }
    r.ticket = sv->next_ticket++;
    r.t_submit = rsort::now_s();
    if (sv->t_first == 0.0) sv->t_first = r.t_submit;
    *ticket = r.ticket;
    if (n == 0) {
        sv->tickets[r.ticket].done = true;
        sv->cv_done.notify_all();
        return RSORT_OK;
    }
    sv->tickets[r.ticket] = rsort::TicketState{};
    sv->sched.push(r);
    sv->cv_work.notify_one();
    return RSORT_OK;
}

int rsort_server_submit(rsort_server* sv, int key_type, const void* keys_in, void* keys_out,
                        size_t n, uint64_t* ticket)
{
    return rsort_server_submit_async(sv, key_type, keys_in, keys_out, n, nullptr, ticket);
}

int rsort_server_reserve(rsort_server* sv, int key_type, size_t max_n)
{
    if (!sv) return RSORT_EINVAL;
    if (key_type != RSORT_U32 && key_type != RSORT_U64) return RSORT_EINVAL;
    if (max_n >= ((size_t)1 << 30)) return RSORT_EUNSUPPORTED;
    const int kb = key_type == RSORT_U64 ? 8 : 4;
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->sched.queued() || sv->sched.busy_slots()) return RSORT_EBUSY;
    if (max_n <= rsort::kServeSmallMax) return RSORT_OK;
    const size_t need = rsort::lsd_r8_layout(kb, false, max_n, 0, 8 * kb).bytes;
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (prev != sv->device) (void)hipSetDevice(sv->device);
    int rc = RSORT_OK;
    for (rsort::Slot& sl : sv->slots)
        if (rsort::grow(&sl.ws, &sl.ws_bytes, need) != hipSuccess) {
            rc = RSORT_ENOMEM;
            break;
        }
    if (prev != sv->device) (void)hipSetDevice(prev);
    return rc;
}

int rsort_server_fail_next(rsort_server* sv)
{
    if (!sv) return RSORT_EINVAL;
    sv->fail_next.store(1);
    return RSORT_OK;
}

int rsort_server_memory(rsort_server* sv, size_t* in_flight, size_t* max_in_flight,
                        size_t* reserved)
{
    if (!sv) return RSORT_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    if (in_flight) *in_flight = (size_t)sv->sched.used();
    if (max_in_flight) *max_in_flight = (size_t)sv->sched.max_used();
    if (reserved) {
        size_t r = 0;
        for (const rsort::Slot& sl : sv->slots)
            r += sl.ws_bytes + 2 * sl.desc_cap * sizeof(rsort::ServeDesc) + 2 * 256;
        *reserved = r;
    }
    return RSORT_OK;
}

int rsort_server_poll(rsort_server* sv, uint64_t ticket, int* done)
{
    if (!sv || !done) return RSORT_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return RSORT_EINVAL;
    *done = it->second.done ? 1 : 0;
    return it->second.done ? it->second.status : RSORT_OK;
}

int rsort_server_wait(rsort_server* sv, uint64_t ticket)
{
    if (!sv) return RSORT_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return RSORT_EINVAL;
    sv->cv_done.wait(lk, [&] {
        auto f = sv->tickets.find(ticket);
        return f == sv->tickets.end() || f->second.done;
    });
    auto f = sv->tickets.find(ticket);
    return f == sv->tickets.end() ? RSORT_OK : f->second.status;
}

int rsort_server_latency(rsort_server* sv, double* p50_us, double* p99_us, double* keys_per_s,
                         uint64_t* completed)
{
    if (!sv) return RSORT_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    std::vector<double> v = sv->latency_s;
    if (completed) *completed = v.size();
    double p50 = 0.0, p99 = 0.0;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&v](double q) {
            // nearest rank
            size_t k = (size_t)(q * (double)v.size() + 0.999999999);
            if (k < 1) k = 1;
            if (k > v.size()) k = v.size();
            return v[k - 1];
        };
        p50 = pct(0.50);
        p99 = pct(0.99);
    }
    if (p50_us) *p50_us = p50 * 1e6;
    if (p99_us) *p99_us = p99 * 1e6;
    if (keys_per_s) {
        const double span = sv->t_last - sv->t_first;
        *keys_per_s = span > 0 ? (double)sv->keys_done / span : 0.0;
    }
    return RSORT_OK;
}

int rsort_server_reset_stats(rsort_server* sv)
{
    if (!sv) return RSORT_EINVAL;
    std::lock_guard<std::mutex> g(sv->mu);
    sv->latency_s.clear();
    sv->sched.reset_max_used();
    sv->keys_done = 0;
    sv->t_first = sv->t_last = 0.0;
    for (auto it = sv->tickets.begin(); it != sv->tickets.end();)
        it = it->second.done ? sv->tickets.erase(it) : std::next(it);
    return RSORT_OK;
}

int rsort_server_destroy(rsort_server* sv)
{
    if (!sv) return RSORT_EINVAL;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->stop = true;
        sv->cv_work.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(sv->device);
    for (rsort::Slot& sl : sv->slots) {
        if (sl.stream) {
            (void)hipStreamSynchronize(sl.stream);
            (void)hipStreamDestroy(sl.stream);
        }
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.ws) (void)hipFree(sl.ws);
        if (sl.desc_host) (void)hipHostFree(sl.desc_host);
        if (sl.desc_dev) (void)hipFree(sl.desc_dev);
        if (sl.err_dev) (void)hipFree(sl.err_dev);
        if (sl.err_host) (void)hipHostFree(sl.err_host);
    }
    for (hipEvent_t ev : sv->free_events) (void)hipEventDestroy(ev);
    (void)hipSetDevice(prev);
    delete sv;
    return RSORT_OK;
}

}  // extern "C"
