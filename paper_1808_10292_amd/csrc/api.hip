// C ABI of the library (declarations and contracts in include/rsort.h):
// argument validation, workspace management and dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rsort.h"
#include "rsort_internal.h"
#include "tune_cache.h"

namespace rsort {

// Event pairs recorded around kernels of each kind; totals are folded in when
// read.  Events are pooled so steady-state recording creates none.
struct Profiler {
    struct Pair {
        int kind;
        hipEvent_t start, stop;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Pair> pending;
    uint32_t kinds = ~0u;   // bit k: kernels of kind k are timed
    uint32_t period = 1;    // time launches 0, period, 2 period, ... of each kind
    uint64_t seen[kNumKinds] = {};
    bool skipping[kNumKinds] = {};
    hipEvent_t open_start[kNumKinds] = {};
    uint64_t launches[kNumKinds] = {};
    double total_ms[kNumKinds] = {};

    hipEvent_t get()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void fold()
    {
        for (Pair& p : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(p.stop) == hipSuccess &&
                hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
                launches[p.kind] += 1;
                total_ms[p.kind] += ms;
            }
            pool.push_back(p.start);
            pool.push_back(p.stop);
        }
        pending.clear();
    }
    ~Profiler()
    {
        fold();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

void profiler_mark(Profiler* p, hipStream_t s, int kind, bool begin)
{
    if (!(p->kinds & (1u << kind))) return;
    if (begin) {
        p->skipping[kind] = p->seen[kind]++ % p->period != 0;
        if (p->skipping[kind]) return;
    } else if (p->skipping[kind]) {
        return;
    }
    hipEvent_t e = p->get();
    if (!e) return;
    (void)hipEventRecord(e, s);
    if (begin) {
        p->open_start[kind] = e;
    } else if (p->open_start[kind]) {
        p->pending.push_back({kind, p->open_start[kind], e});
        p->open_start[kind] = nullptr;
        if (p->pending.size() > 4096) p->fold();
    }
}

}  // namespace rsort

namespace {

// Workspace of rsort_sort_noalloc: a file-scope device array, so every GPU the
// library runs on holds its own copy (allocated when the code object is loaded
// there, kept until the process ends).  Host code never uses the array's name
// as an address: the address on each device comes from hipGetSymbolAddress,
// taken once per device when a context is created on it.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on `device` (the caller has made it current), or
// nullptr if the runtime cannot resolve it.
void* scratch_address(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_ptr[device] = ptr;
        else (void)hipGetLastError();
    }
    return g_scratch_ptr[device];
}

}  // namespace

struct rsort_ctx {
    int device = 0;
    void* scratch = nullptr;     // this device's address of `scratch` (rsort_sort_noalloc)
    void* ws = nullptr;          // cached workspace (grown on demand)
    size_t ws_bytes = 0;
    uint32_t* dev_err = nullptr; // device-side failure bits (DeviceError)
    rsort::Profiler* prof = nullptr;
    // pinned host staging of the segmented sort's plan, and the event that
    // marks the end of its last upload (the buffer is reused only after it)
    void* meta_host = nullptr;
    size_t meta_bytes = 0;
    hipEvent_t meta_done = nullptr;
    bool meta_pending = false;
    // second stream of the segmented sort (whole-segment sorts beside the
    // large segments' rounds) and its fork / join events; made on first use
    rsort::SegOverlap seg_ov;
    uint32_t small_max = rsort::kSmallMaxDefault;
    int small_sort = RSORT_SMALL_RADIX;   // sorter of the small segments
    int seg_tile_shape = rsort::kSegTileShapeDefault;   // tiles of the large segments
    int seg_launch = RSORT_SEG_ROUNDS;                   // launches of the segmented sort
    int pr4_rounds = RSORT_PR4_COUNTED;  // round kind of RSORT_LSD_R8
    rsort::SegPlan plan;
    uint64_t upload_sig = 0;         // plan last uploaded into upload_ws
    void* upload_ws = nullptr;
    // split statistics of the last sample sort (device), sized for p = kMaxP
    uint32_t* gsd_stats = nullptr;
    uint32_t gsd_p = 0;
    std::string tune_cache;   // the tuner's persisted choices (empty: none)
    std::string last_error;
};


namespace {

constexpr size_t kMaxN = (size_t)1 << 30;
constexpr int kMaxP = 1024;                       // sample sort buckets
constexpr uint64_t kMaxSample = (uint64_t)1 << 26; // r p^2
constexpr int kDefaultP = 256, kDefaultR = 32;

int fail(rsort_ctx* ctx, int status, const char* fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->last_error = buf;
    }
    return status;
}

int hip_fail(rsort_ctx* ctx, hipError_t e, const char* where)
{
    return fail(ctx, e == hipErrorOutOfMemory ? RSORT_ENOMEM : RSORT_EDEVICE, "%s: %s", where,
                hipGetErrorString(e));
}

// True if p is memory the GPU `device` can address as device memory.
bool is_device_pointer(const void* p, int device)
{
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice && attr.device == device;
}

// A caller's workspace must be device memory of the context's device; the
// scratch of rsort_sort_noalloc is (it is not a hipMalloc allocation, so the
// pointer query is not asked about it).
bool workspace_ok(const rsort_ctx* ctx, const void* ws)
{
    return (ctx->scratch && ws == ctx->scratch) || is_device_pointer(ws, ctx->device);
}

bool overlap_partial(const void* a, size_t abytes, const void* b, size_t bbytes)
{
    if (a == b) return false;
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + bbytes && y < x + abytes;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int ensure_workspace(rsort_ctx* ctx, size_t need, void** ws)
{
    if (need <= ctx->ws_bytes) {
        *ws = ctx->ws;
        return RSORT_OK;
    }
    if (ctx->ws) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
        (void)hipFree(ctx->ws);
        if (ctx->upload_ws == ctx->ws) ctx->upload_ws = nullptr;
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    size_t grow = std::max(need, (size_t)1 << 20);
    hipError_t e = rsort::dev_malloc(&ctx->ws, grow);
    if (e != hipSuccess) {
        ctx->ws = nullptr;
        return hip_fail(ctx, e, "hipMalloc(workspace)");
    }
    ctx->ws_bytes = grow;
    *ws = ctx->ws;
    return RSORT_OK;
}

int key_bytes_of(int key_type)
{
    return key_type == RSORT_U32 ? 4 : (key_type == RSORT_U64 ? 8 : 0);
}

// Signed and floating-point key types: the unsigned type of the same width
// and the order-preserving map between them.  False for the unsigned types.
bool mapped_key(int key_type, int* ukey, int* kind)
{
    switch (key_type) {
    case RSORT_I32: *ukey = RSORT_U32; *kind = rsort::kKeySigned; return true;
    case RSORT_F32: *ukey = RSORT_U32; *kind = rsort::kKeyFloat; return true;
    case RSORT_I64: *ukey = RSORT_U64; *kind = rsort::kKeySigned; return true;
    case RSORT_F64: *ukey = RSORT_U64; *kind = rsort::kKeyFloat; return true;
    default: return false;
    }
}

int validate_bits(rsort_ctx* ctx, int key_type, int begin_bit, int end_bit)
{
    const int width = key_bytes_of(key_type) * 8;
    if (begin_bit < 0 || end_bit > width || begin_bit > end_bit)
        return fail(ctx, RSORT_EINVAL, "bit range [%d, %d) outside [0, %d]", begin_bit, end_bit, width);
    return RSORT_OK;
}

size_t sort_ws_bytes(int key_type, bool has_vals, size_t n, int algo, int begin_bit, int end_bit,
                     int pr4_rounds)
{
    if (algo == RSORT_SAMPLE_REGULAR)
        return rsort::gsd_layout(has_vals, n, kDefaultP, kDefaultR).bytes;
    if (algo == RSORT_LSD_R16)
        return rsort::lsd_r16_layout(key_bytes_of(key_type), has_vals, n, begin_bit, end_bit).bytes;
    return rsort::lsd_r8_layout(key_bytes_of(key_type), has_vals, n, begin_bit, end_bit,
                                pr4_rounds == RSORT_PR4_SINGLE_READ).bytes;
}

// Device residency and aliasing of the key / payload arrays of a sort of n
// keys (the caller has checked n > 0 and the NULL rules).
int check_arrays(rsort_ctx* ctx, int kb, const void* keys_in, const void* keys_out,
                 const uint32_t* vals_in, const uint32_t* vals_out, size_t n)
{
    if (!is_device_pointer(keys_in, ctx->device) || !is_device_pointer(keys_out, ctx->device))
        return fail(ctx, RSORT_EINVAL, "key arrays must be device memory of device %d", ctx->device);
    if (vals_in && (!is_device_pointer(vals_in, ctx->device) || !is_device_pointer(vals_out, ctx->device)))
        return fail(ctx, RSORT_EINVAL, "payload arrays must be device memory of device %d", ctx->device);
    const size_t kbytes = n * kb, vbytes = n * 4;
    if (overlap_partial(keys_in, kbytes, keys_out, kbytes))
        return fail(ctx, RSORT_EINVAL, "keys_in and keys_out overlap without being equal");
    if (vals_in) {
        if (overlap_partial(vals_in, vbytes, vals_out, vbytes))
            return fail(ctx, RSORT_EINVAL, "vals_in and vals_out overlap without being equal");
        if (overlap_partial(keys_in, kbytes, vals_in, vbytes) || keys_in == (const void*)vals_in ||
            overlap_partial(keys_out, kbytes, vals_out, vbytes) || keys_out == (const void*)vals_out ||
            overlap_partial(keys_out, kbytes, vals_in, vbytes) || keys_out == (const void*)vals_in ||
            overlap_partial(keys_in, kbytes, vals_out, vbytes) || keys_in == (const void*)vals_out)
            return fail(ctx, RSORT_EINVAL, "key and payload arrays overlap");
    }
    return RSORT_OK;
}

// p and the oversampling parameter q: r for GSD (sample r p^2), s for GER and
// GVR (sample s p - 1).
int check_gsd_params(rsort_ctx* ctx, int key_type, int p, int q, int kind = rsort::kGSD)
{
    if (key_type != RSORT_U32)
        return fail(ctx, RSORT_EUNSUPPORTED, "the sample sort takes uint32 keys only");
    const int pmax = kind == rsort::kGVR ? (int)rsort::kGvrMaxP : kMaxP;
    if (p < 1 || p > pmax) return fail(ctx, RSORT_EINVAL, "p = %d outside [1, %d]", p, pmax);
    if (q < 1) return fail(ctx, RSORT_EINVAL, "oversampling %d < 1", q);
    const uint64_t sample = kind != rsort::kGSD ? (uint64_t)q * p : (uint64_t)q * p * p;
    if (sample > kMaxSample)
        return fail(ctx, RSORT_EUNSUPPORTED, "sample of %llu keys above 2^26",
                    (unsigned long long)sample);
    return RSORT_OK;
}

}  // namespace

namespace rsort {

namespace {
// Allocations left up to and including the one that fails; 0: none fails.
std::atomic<long> g_fail_alloc{0};
std::once_flag g_fail_alloc_env;

void fail_alloc_from_env()
{
    std::call_once(g_fail_alloc_env, [] {
        const char* s = getenv("RSORT_FAULT_ALLOC");
        const long k = s ? strtol(s, nullptr, 10) : 0;
        if (k > 0) g_fail_alloc.store(k);
    });
}
}  // namespace

hipError_t dev_malloc(void** p, size_t bytes)
{
    fail_alloc_from_env();
    long k = g_fail_alloc.load();
    while (k > 0 && !g_fail_alloc.compare_exchange_weak(k, k - 1)) {
    }
    if (k == 1) {   // this call is the k-th
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

}  // namespace rsort

extern "C" {

int rsort_debug_fail_alloc(int k)
{
    if (k < 0) return RSORT_EINVAL;
    rsort::fail_alloc_from_env();
    rsort::g_fail_alloc.store(k);
    return RSORT_OK;
}

int rsort_set_tune_cache(rsort_ctx* ctx, const char* path)
{
    if (!ctx) return RSORT_EINVAL;
    ctx->tune_cache = path ? path : "";
    return RSORT_OK;
}

int rsort_create(int hip_device, rsort_ctx** out)
{
    if (!out) return RSORT_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count)
        return RSORT_EINVAL;
    rsort_ctx* ctx = new (std::nothrow) rsort_ctx;
    if (!ctx) return RSORT_ENOMEM;
    ctx->device = hip_device;
    DeviceGuard g(hip_device);
    if (rsort::dev_malloc((void**)&ctx->dev_err, 256) != hipSuccess ||
        hipMemset(ctx->dev_err, 0, 256) != hipSuccess) {
        if (ctx->dev_err) (void)hipFree(ctx->dev_err);
        delete ctx;
        return RSORT_ENOMEM;
    }
    ctx->scratch = scratch_address(hip_device);
    if (const char* tc = getenv("RSORT_TUNE_CACHE")) ctx->tune_cache = tc;
    *out = ctx;
    return RSORT_OK;
}

int rsort_destroy(rsort_ctx* ctx)
{
    if (!ctx) return RSORT_EINVAL;
    {
        DeviceGuard g(ctx->device);
        (void)hipDeviceSynchronize();
        delete ctx->prof;
        if (ctx->meta_host) (void)hipHostFree(ctx->meta_host);
        if (ctx->meta_done) (void)hipEventDestroy(ctx->meta_done);
        if (ctx->seg_ov.fork) (void)hipEventDestroy(ctx->seg_ov.fork);
        if (ctx->seg_ov.join) (void)hipEventDestroy(ctx->seg_ov.join);
        if (ctx->seg_ov.aux) (void)hipStreamDestroy(ctx->seg_ov.aux);
        if (ctx->ws) (void)hipFree(ctx->ws);
        if (ctx->dev_err) (void)hipFree(ctx->dev_err);
        if (ctx->gsd_stats) (void)hipFree(ctx->gsd_stats);
    }
    delete ctx;
    return RSORT_OK;
}

const char* rsort_status_string(int status)
{
    switch (status) {
    case RSORT_OK: return "success";
    case RSORT_EINVAL: return "invalid argument";
    case RSORT_ENOMEM: return "out of device memory";
    case RSORT_EDEVICE: return "device error";
    case RSORT_EBUSY: return "resource busy";
    case RSORT_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status";
    }
}

const char* rsort_last_error(const rsort_ctx* ctx)
{
    return ctx ? ctx->last_error.c_str() : "";
}

int rsort_workspace_bytes(rsort_ctx* ctx, int key_type, int has_vals, size_t n, int algo,
                          size_t* bytes)
{
    if (!ctx || !bytes) return RSORT_EINVAL;
    int ukey = 0, kind = 0;
    if (mapped_key(key_type, &ukey, &kind)) {
        // the unsigned sort's workspace, then the mapped keys
        if (algo == RSORT_SAMPLE_REGULAR)
            return fail(ctx, RSORT_EUNSUPPORTED, "the sample sort takes uint32 keys only");
        size_t inner = 0;
        const int rc = rsort_workspace_bytes(ctx, ukey, has_vals, n, algo, &inner);
        if (rc) return rc;
        *bytes = rsort::align_up(inner) + n * key_bytes_of(ukey);
        return RSORT_OK;
    }
    if (!key_bytes_of(key_type)) return fail(ctx, RSORT_EINVAL, "unknown key type %d", key_type);
    if (n >= kMaxN) return fail(ctx, RSORT_EUNSUPPORTED, "n = %zu >= 2^30", n);
    if (algo == RSORT_SAMPLE_REGULAR)
        return rsort_sample_sort_workspace_bytes(ctx, key_type, has_vals, n, kDefaultP, kDefaultR,
                                                 bytes);
    *bytes = sort_ws_bytes(key_type, has_vals != 0, n, algo, 0, key_bytes_of(key_type) * 8,
                           ctx->pr4_rounds);
    return RSORT_OK;
}

int rsort_sample_sort_workspace_bytes(rsort_ctx* ctx, int key_type, int has_vals, size_t n,
                                      int p, int r, size_t* bytes)
{
    if (!ctx || !bytes) return RSORT_EINVAL;
    int rc = check_gsd_params(ctx, key_type, p, r);
    if (rc) return rc;
    if (n >= kMaxN) return fail(ctx, RSORT_EUNSUPPORTED, "n = %zu >= 2^30", n);
    *bytes = n ? rsort::gsd_layout(has_vals != 0, n, (uint32_t)p, (uint32_t)r).bytes : 0;
    return RSORT_OK;
}

}  // extern "C"

namespace {

rsort::GsdLayout skeleton_layout(int kind, bool has_vals, size_t n, int p, int q)
{
    if (kind == rsort::kGER) return rsort::ger_layout(has_vals, n, (uint32_t)p, (uint32_t)q);
    if (kind == rsort::kGVR) return rsort::gvr_layout(has_vals, n, (uint32_t)p, (uint32_t)q);
    return rsort::gsd_layout(has_vals, n, (uint32_t)p, (uint32_t)q);
}

// Signed / floating-point keys: map into a workspace temporary, sort that as
// unsigned keys into keys_out (never in place, whatever the caller's
// pointers), map keys_out back.
int sort_mapped(rsort_ctx* ctx, int ukey, int kind, const void* keys_in, void* keys_out,
                const uint32_t* vals_in, uint32_t* vals_out, size_t n, int begin_bit, int end_bit,
                int algo, void* workspace, size_t ws_bytes, void* stream)
{
    const int kb = key_bytes_of(ukey);
    if (begin_bit != 0 || end_bit != kb * 8)
        return fail(ctx, RSORT_EUNSUPPORTED, "signed and floating-point keys are sorted whole");
    if (algo != RSORT_AUTO && algo != RSORT_LSD_R8 && algo != RSORT_LSD_R16)
        return fail(ctx, RSORT_EUNSUPPORTED, "signed and floating-point keys take the radix sorts");
    if ((vals_in == nullptr) != (vals_out == nullptr))
        return fail(ctx, RSORT_EINVAL, "vals_in and vals_out must both be NULL or both be set");
    if ((workspace == nullptr) != (ws_bytes == 0))
        return fail(ctx, RSORT_EINVAL, "workspace and ws_bytes must both be 0 or both be set");
    if (n == 0) return RSORT_OK;
    if (n >= kMaxN) return fail(ctx, RSORT_EUNSUPPORTED, "n = %zu >= 2^30", n);
    if (!keys_in || !keys_out) return fail(ctx, RSORT_EINVAL, "NULL key pointer with n > 0");
    DeviceGuard g(ctx->device);
    int rc = check_arrays(ctx, kb, keys_in, keys_out, vals_in, vals_out, n);
    if (rc) return rc;
    const size_t inner =
        rsort::align_up(sort_ws_bytes(ukey, vals_in != nullptr, n, algo, 0, kb * 8, ctx->pr4_rounds));
    const size_t need = inner + n * kb;
    void* ws = workspace;
    if (ws) {
        if (ws_bytes < need)
            return fail(ctx, RSORT_EINVAL, "workspace of %zu bytes < %zu needed", ws_bytes, need);
        if (!workspace_ok(ctx, ws))
            return fail(ctx, RSORT_EINVAL, "workspace must be device memory");
    } else {
        rc = ensure_workspace(ctx, need, &ws);
        if (rc) return rc;
    }
    void* mapped = (uint8_t*)ws + inner;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = rsort::map_keys(kb, kind, false, keys_in, mapped, n, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
    rc = rsort_sort(ctx, ukey, mapped, keys_out, vals_in, vals_out, n, 0, kb * 8, algo, ws, inner,
                    stream);
    if (rc) return rc;
    e = rsort::map_keys(kb, kind, true, keys_out, keys_out, n, s);
    return e == hipSuccess ? RSORT_OK : hip_fail(ctx, e, "kernel launch");
}

// Shared part of the sample sorts once the layout is known.
int run_skeleton(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
                 const uint32_t* vals_in, uint32_t* vals_out, size_t n, int kind, int p, int s,
                 uint64_t seed, void* workspace, size_t ws_bytes, void* stream)
{
    ctx->last_error.clear();
    int rc = check_gsd_params(ctx, key_type, p, s, kind);
    if (rc) return rc;
    if ((vals_in == nullptr) != (vals_out == nullptr))
        return fail(ctx, RSORT_EINVAL, "vals_in and vals_out must both be NULL or both be set");
    if ((workspace == nullptr) != (ws_bytes == 0))
        return fail(ctx, RSORT_EINVAL, "workspace and ws_bytes must both be 0 or both be set");
    if (n == 0) return RSORT_OK;
    if (n >= kMaxN) return fail(ctx, RSORT_EUNSUPPORTED, "n = %zu >= 2^30", n);
    if (!keys_in || !keys_out) return fail(ctx, RSORT_EINVAL, "NULL key pointer with n > 0");
    DeviceGuard g(ctx->device);
    rc = check_arrays(ctx, 4, keys_in, keys_out, vals_in, vals_out, n);
    if (rc) return rc;
    const rsort::GsdLayout L = skeleton_layout(kind, vals_in != nullptr, n, p, s);
    hipStream_t st = (hipStream_t)stream;
    if (!ctx->gsd_stats) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone)
            return fail(ctx, RSORT_EINVAL,
                        "first sample sort on a context cannot be captured (it allocates)");
        hipError_t e = rsort::dev_malloc((void**)&ctx->gsd_stats, rsort::gsd_stats_words(kMaxP) * 4);
        if (e != hipSuccess) {
            ctx->gsd_stats = nullptr;
            return hip_fail(ctx, e, "hipMalloc(sample sort statistics)");
        }
    }
    void* ws = workspace;
    if (ws) {
        if (ws_bytes < L.bytes)
            return fail(ctx, RSORT_EINVAL, "workspace of %zu bytes < %zu needed", ws_bytes, L.bytes);
        if (!workspace_ok(ctx, ws))
            return fail(ctx, RSORT_EINVAL, "workspace must be device memory");
    } else {
        rc = ensure_workspace(ctx, L.bytes, &ws);
        if (rc) return rc;
    }
    hipError_t e = rsort::gsd_sort((const uint32_t*)keys_in, (uint32_t*)keys_out, vals_in, vals_out,
                                   n, L, seed, ws, ctx->gsd_stats, ctx->dev_err, st, ctx->prof);
    if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
    ctx->gsd_p = L.p;
    return RSORT_OK;
}

// Default GER oversampling s = 2 w^2 lg n with w = ceil(lg lg n) (at least 1).
int ger_default_s(size_t n)
{
    int lg = 0;
    while (((size_t)1 << lg) < n) ++lg;
    int w = 0;
    while ((1 << w) < lg) ++w;
    if (w < 1) w = 1;
    if (lg < 1) lg = 1;
    return 2 * w * w * lg;
}

}  // namespace

extern "C" {

int rsort_sample_sort(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
                      const uint32_t* vals_in, uint32_t* vals_out, size_t n, int p, int r,
                      void* workspace, size_t ws_bytes, void* stream)
{
    if (!ctx) return RSORT_EINVAL;
    return run_skeleton(ctx, key_type, keys_in, keys_out, vals_in, vals_out, n, rsort::kGSD, p, r, 0,
                        workspace, ws_bytes, stream);
}

int rsort_sample_sort_random(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
                             const uint32_t* vals_in, uint32_t* vals_out, size_t n, int p, int s,
                             uint64_t seed, void* workspace, size_t ws_bytes, void* stream)
{
    if (!ctx) return RSORT_EINVAL;
    if (s == 0) s = ger_default_s(n);
    return run_skeleton(ctx, key_type, keys_in, keys_out, vals_in, vals_out, n, rsort::kGER, p, s,
                        seed, workspace, ws_bytes, stream);
}

int rsort_sample_sort_random_workspace_bytes(rsort_ctx* ctx, int key_type, int has_vals, size_t n,
                                             int p, int s, size_t* bytes)
{
    if (!ctx || !bytes) return RSORT_EINVAL;
    if (s == 0) s = ger_default_s(n);
    int rc = check_gsd_params(ctx, key_type, p, s, rsort::kGER);
    if (rc) return rc;
    if (n >= kMaxN) return fail(ctx, RSORT_EUNSUPPORTED, "n = %zu >= 2^30", n);
    *bytes = n ? rsort::ger_layout(has_vals != 0, n, (uint32_t)p, (uint32_t)s).bytes : 0;
    return RSORT_OK;
}

int rsort_sample_sort_gvr(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
                          const uint32_t* vals_in, uint32_t* vals_out, size_t n, int p, int s,
                          uint64_t seed, void* workspace, size_t ws_bytes, void* stream)
{
    if (!ctx) return RSORT_EINVAL;
    if (s == 0) s = ger_default_s(n);
    return run_skeleton(ctx, key_type, keys_in, keys_out, vals_in, vals_out, n, rsort::kGVR, p, s,
                        seed, workspace, ws_bytes, stream);
}

int rsort_sample_sort_gvr_workspace_bytes(rsort_ctx* ctx, int key_type, int has_vals, size_t n,
                                          int p, int s, size_t* bytes)
{
    if (!ctx || !bytes) return RSORT_EINVAL;
    if (s == 0) s = ger_default_s(n);
    int rc = check_gsd_params(ctx, key_type, p, s, rsort::kGVR);
    if (rc) return rc;
    if (n >= kMaxN) return fail(ctx, RSORT_EUNSUPPORTED, "n = %zu >= 2^30", n);
    *bytes = n ? rsort::gvr_layout(has_vals != 0, n, (uint32_t)p, (uint32_t)s).bytes : 0;
    return RSORT_OK;
}

int rsort_sample_sort_stats(rsort_ctx* ctx, int p_cap, int* p_used, uint32_t* cnt,
                            uint32_t* bucket, uint32_t* split_key, uint32_t* split_index)
{
    if (!ctx || !p_used) return RSORT_EINVAL;
    if (!ctx->gsd_p) return fail(ctx, RSORT_EINVAL, "no sample sort has run on this context");
    const uint32_t p = ctx->gsd_p;
    *p_used = (int)p;
    if (p_cap < (int)p) return fail(ctx, RSORT_EINVAL, "p_cap %d < p %u", p_cap, p);
    DeviceGuard g(ctx->device);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
    std::vector<uint32_t> h(rsort::gsd_stats_words(p));
    e = hipMemcpy(h.data(), ctx->gsd_stats, h.size() * 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(statistics)");
    const uint32_t* bnd = h.data();
    for (uint32_t j = 0; j < p; ++j) {
        uint32_t tot = 0;
        for (uint32_t k = 0; k < p; ++k) {
            const uint32_t c = bnd[(size_t)k * (p + 1) + j + 1] - bnd[(size_t)k * (p + 1) + j];
            if (cnt) cnt[(size_t)k * p + j] = c;
            tot += c;
        }
        if (bucket) bucket[j] = tot;
    }
    for (uint32_t i = 0; i + 1 < p; ++i) {
        if (split_key) split_key[i] = h[(size_t)p * (p + 1) + i];
        if (split_index) split_index[i] = h[(size_t)p * (p + 1) + p + i];
    }
    return RSORT_OK;
}

int rsort_sort(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
               const uint32_t* vals_in, uint32_t* vals_out, size_t n, int begin_bit,
               int end_bit, int algo, void* workspace, size_t ws_bytes, void* stream)
{
    if (!ctx) return RSORT_EINVAL;
    ctx->last_error.clear();
    int ukey = 0, kind = 0;
    if (mapped_key(key_type, &ukey, &kind))
        return sort_mapped(ctx, ukey, kind, keys_in, keys_out, vals_in, vals_out, n, begin_bit,
                           end_bit, algo, workspace, ws_bytes, stream);
    const int kb = key_bytes_of(key_type);
    if (!kb) return fail(ctx, RSORT_EINVAL, "unknown key type %d", key_type);
    if (algo != RSORT_AUTO && algo != RSORT_LSD_R8 && algo != RSORT_LSD_R16 &&
        algo != RSORT_SAMPLE_REGULAR)
        return fail(ctx, RSORT_EUNSUPPORTED, "algorithm %d not available", algo);
    int rc = validate_bits(ctx, key_type, begin_bit, end_bit);
    if (rc) return rc;
    if (algo == RSORT_SAMPLE_REGULAR) {
        if (begin_bit != 0 || end_bit != kb * 8)
            return fail(ctx, RSORT_EUNSUPPORTED, "the sample sort compares whole keys");
        return rsort_sample_sort(ctx, key_type, keys_in, keys_out, vals_in, vals_out, n, kDefaultP,
                                 kDefaultR, workspace, ws_bytes, stream);
    }
    if ((vals_in == nullptr) != (vals_out == nullptr))
        return fail(ctx, RSORT_EINVAL, "vals_in and vals_out must both be NULL or both be set");
    if (n == 0) return RSORT_OK;
    if (n >= kMaxN) return fail(ctx, RSORT_EUNSUPPORTED, "n = %zu >= 2^30", n);
    if (!keys_in || !keys_out) return fail(ctx, RSORT_EINVAL, "NULL key pointer with n > 0");
    if ((workspace == nullptr) != (ws_bytes == 0))
        return fail(ctx, RSORT_EINVAL, "workspace and ws_bytes must both be 0 or both be set");

    DeviceGuard g(ctx->device);
    rc = check_arrays(ctx, kb, keys_in, keys_out, vals_in, vals_out, n);
    if (rc) return rc;
    const size_t kbytes = n * kb, vbytes = n * 4;
    hipStream_t s = (hipStream_t)stream;

    if (end_bit == begin_bit) {  // nothing to compare: the stable sort is the identity
        hipError_t e = rsort::copy_bytes(keys_out, keys_in, kbytes, s);
        if (e == hipSuccess && vals_in) e = rsort::copy_bytes(vals_out, vals_in, vbytes, s);
        return e == hipSuccess ? RSORT_OK : hip_fail(ctx, e, "copy");
    }

    if (algo == RSORT_LSD_R16) {
        const rsort::LsdR16Layout L16 =
            rsort::lsd_r16_layout(kb, vals_in != nullptr, n, begin_bit, end_bit);
        void* ws = workspace;
        if (ws) {
            if (ws_bytes < L16.bytes)
                return fail(ctx, RSORT_EINVAL, "workspace of %zu bytes < %zu needed", ws_bytes, L16.bytes);
            if (!workspace_ok(ctx, ws))
                return fail(ctx, RSORT_EINVAL, "workspace must be device memory");
        } else {
            rc = ensure_workspace(ctx, L16.bytes, &ws);
            if (rc) return rc;
        }
        hipError_t e = rsort::lsd_r16_sort(kb, keys_in, keys_out, vals_in, vals_out, n, begin_bit,
                                           end_bit, ws, L16, ctx->dev_err, s, ctx->prof);
        return e == hipSuccess ? RSORT_OK : hip_fail(ctx, e, "kernel launch");
    }
    const rsort::LsdR8Layout L = rsort::lsd_r8_layout(kb, vals_in != nullptr, n, begin_bit, end_bit,
                                                      ctx->pr4_rounds == RSORT_PR4_SINGLE_READ);
    void* ws = workspace;
    if (ws) {
        if (ws_bytes < L.bytes)
            return fail(ctx, RSORT_EINVAL, "workspace of %zu bytes < %zu needed", ws_bytes, L.bytes);
        if (!is_device_pointer(ws, ctx->device))
            return fail(ctx, RSORT_EINVAL, "workspace must be device memory");
    } else {
        rc = ensure_workspace(ctx, L.bytes, &ws);
        if (rc) return rc;
    }
    hipError_t e = rsort::lsd_r8_sort(kb, keys_in, keys_out, vals_in, vals_out, n, begin_bit,
                                      end_bit, ws, L, ctx->dev_err, s, ctx->prof);
    if (e != hipSuccess) return hip_fail(ctx, e, "kernel launch");
    return RSORT_OK;
}

int rsort_sort_noalloc(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
                       const uint32_t* vals_in, uint32_t* vals_out, size_t n, int begin_bit,
                       int end_bit, void* stream)
{
    if (!ctx) return RSORT_EINVAL;
    ctx->last_error.clear();
    if (!ctx->scratch)
        return fail(ctx, RSORT_EDEVICE, "no address of the scratch array on device %d", ctx->device);
    size_t need = 0;
    int rc = rsort_workspace_bytes(ctx, key_type, vals_in != nullptr, n, RSORT_LSD_R8, &need);
    if (rc) return rc;
    if (need > kScratchBytes)
        return fail(ctx, RSORT_EUNSUPPORTED,
                    "n = %zu needs %zu bytes of workspace, above the %zu-byte scratch of "
                    "rsort_sort_noalloc", n, need, kScratchBytes);
    // no event is created or recorded: the profiler stays off for this call
    rsort::Profiler* prof = ctx->prof;
    ctx->prof = nullptr;
    rc = rsort_sort(ctx, key_type, keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit,
                    RSORT_LSD_R8, ctx->scratch, kScratchBytes, stream);
    ctx->prof = prof;
    return rc;
}

int rsort_histogram(rsort_ctx* ctx, int key_type, const void* keys, size_t n, int digit_bits,
                    int begin_bit, int end_bit, uint32_t* hist_out, void* stream)
{
    if (!ctx) return RSORT_EINVAL;
    ctx->last_error.clear();
    const int kb = key_bytes_of(key_type);
    if (!kb) return fail(ctx, RSORT_EINVAL, "unknown key type %d", key_type);
    if (digit_bits != 8 && digit_bits != 16)
        return fail(ctx, RSORT_EINVAL, "digit_bits must be 8 or 16");
    int rc = validate_bits(ctx, key_type, begin_bit, end_bit);
    if (rc) return rc;
    if (n >= kMaxN) return fail(ctx, RSORT_EUNSUPPORTED, "n = %zu >= 2^30", n);
    if (end_bit == begin_bit) return RSORT_OK;
    DeviceGuard g(ctx->device);
    if (!hist_out || !is_device_pointer(hist_out, ctx->device))
        return fail(ctx, RSORT_EINVAL, "hist_out must be device memory");
    if (n && (!keys || !is_device_pointer(keys, ctx->device)))
        return fail(ctx, RSORT_EINVAL, "keys must be device memory");
    void* ws = nullptr;
    size_t need = rsort::histogram_ws_bytes(digit_bits, begin_bit, end_bit);
    if (need) {
        rc = ensure_workspace(ctx, need, &ws);
        if (rc) return rc;
    }
    hipError_t e = rsort::histogram(kb, keys, n, digit_bits, begin_bit, end_bit, hist_out, ws,
                                    (hipStream_t)stream);
    return e == hipSuccess ? RSORT_OK : hip_fail(ctx, e, "kernel launch");
}

int rsort_profile_enable(rsort_ctx* ctx, int enable)
{
    if (!ctx) return RSORT_EINVAL;
    DeviceGuard g(ctx->device);
    delete ctx->prof;
    ctx->prof = nullptr;
    if (enable) {
        ctx->prof = new (std::nothrow) rsort::Profiler;
        if (!ctx->prof) return fail(ctx, RSORT_ENOMEM, "profiler");
        ctx->prof->kinds = (uint32_t)enable;
    }
    return RSORT_OK;
}

int rsort_profile_set_period(rsort_ctx* ctx, uint32_t period)
{
    if (!ctx) return RSORT_EINVAL;
    if (!ctx->prof) return fail(ctx, RSORT_EINVAL, "profiling is not enabled");
    if (!period) return fail(ctx, RSORT_EINVAL, "period must be at least 1");
    ctx->prof->period = period;
    return RSORT_OK;
}

int rsort_profile_read(rsort_ctx* ctx, int kind, uint64_t* launches, double* total_ms)
{
    if (!ctx || !launches || !total_ms || kind < 0 || kind >= rsort::kNumKinds) return RSORT_EINVAL;
    if (!ctx->prof) return fail(ctx, RSORT_EINVAL, "profiling is not enabled");
    DeviceGuard g(ctx->device);
    ctx->prof->fold();
    *launches = ctx->prof->launches[kind];
    *total_ms = ctx->prof->total_ms[kind];
    return RSORT_OK;
}

}  // extern "C"

namespace {

// Validate host CSR offsets; total key count in *total.
int check_offsets(rsort_ctx* ctx, const uint64_t* off, size_t num_segs, size_t* total)
{
    if (num_segs && !off) return fail(ctx, RSORT_EINVAL, "seg_offsets is NULL");
    *total = num_segs ? (size_t)off[num_segs] : 0;
    for (size_t s = 0; s < num_segs; ++s)
        if (off[s + 1] < off[s])
            return fail(ctx, RSORT_EINVAL, "seg_offsets decreases at segment %zu", s);
    if (*total >= kMaxN) return fail(ctx, RSORT_EUNSUPPORTED, "total = %zu >= 2^30", *total);
    return RSORT_OK;
}

// The persistent segmented launch (seg_persist.hip: one cooperative launch,
// phases separated by grid-wide barriers) can be selected and tuned.
constexpr bool kPersistentLaunch = true;

// The host plan of a segmented sort on ctx and the workspace it needs, for
// the context's launch mode (the persistent launch sorts segments of at most
// one of its tiles in LDS and uses its own tile shape).
size_t seg_plan_for(rsort_ctx* ctx, const uint64_t* seg_offsets, size_t num_segs, int kb,
                    bool has_vals, size_t total, rsort::SegPlan& P)
{
    if (ctx->seg_launch == RSORT_SEG_PERSISTENT) {
        rsort::segmented_plan(seg_offsets, num_segs,
                              std::min(ctx->small_max, rsort::persist_small_max(kb)), kb, P,
                              rsort::persist_tile_shape(kb));
        return rsort::persist_ws_bytes(kb, has_vals, total, P);
    }
    rsort::segmented_plan(seg_offsets, num_segs, ctx->small_max, kb, P, ctx->seg_tile_shape);
    return rsort::segmented_ws_bytes(kb, has_vals, total, P);
}

// The segmented sort's second stream and events (default priority, made on
// first use); null when they cannot be made or RSORT_SEG_OVERLAP is 0, and
// the sort then runs on the caller's stream alone.
#ifndef RSORT_SEG_OVERLAP
#define RSORT_SEG_OVERLAP 1
#endif
const rsort::SegOverlap* seg_overlap(rsort_ctx* ctx)
{
    if (!RSORT_SEG_OVERLAP) return nullptr;
    rsort::SegOverlap& o = ctx->seg_ov;
    if (!o.aux) {
        hipStream_t st = nullptr;
        hipEvent_t f = nullptr, j = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
        if (hipEventCreateWithFlags(&f, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&j, hipEventDisableTiming) != hipSuccess) {
            if (f) (void)hipEventDestroy(f);
            (void)hipStreamDestroy(st);
            return nullptr;
        }
        o.aux = st;
        o.fork = f;
        o.join = j;
    }
    return &o;
}

}  // namespace

extern "C" {

int rsort_segmented_workspace_bytes(rsort_ctx* ctx, int key_type, int has_vals,
                                    const uint64_t* seg_offsets, size_t num_segs, size_t* bytes)
{
    if (!ctx || !bytes) return RSORT_EINVAL;
    const int kb = key_bytes_of(key_type);
    if (!kb) return fail(ctx, RSORT_EINVAL, "unknown key type %d", key_type);
    size_t total = 0;
    int rc = check_offsets(ctx, seg_offsets, num_segs, &total);
    if (rc) return rc;
    rsort::SegPlan P;
    *bytes = seg_plan_for(ctx, seg_offsets, num_segs, kb, has_vals != 0, total, P);
    return RSORT_OK;
}

int rsort_segmented_device_workspace_bytes(rsort_ctx* ctx, int key_type, int has_vals,
                                           size_t num_segs, size_t total_n, size_t* bytes)
{
    if (!ctx || !bytes) return RSORT_EINVAL;
    const int kb = key_bytes_of(key_type);
    if (!kb) return fail(ctx, RSORT_EINVAL, "unknown key type %d", key_type);
    if (total_n >= kMaxN || num_segs >= kMaxN)
        return fail(ctx, RSORT_EUNSUPPORTED, "total_n or num_segs >= 2^30");
    *bytes = rsort::devseg_layout(kb, has_vals != 0, total_n, (uint32_t)num_segs).bytes;
    return RSORT_OK;
}

int rsort_segmented_sort_device(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
                                const uint32_t* vals_in, uint32_t* vals_out,
                                const uint32_t* seg_offsets, size_t num_segs, size_t total_n,
                                void* workspace, size_t ws_bytes, void* stream)
{
    if (!ctx) return RSORT_EINVAL;
    ctx->last_error.clear();
    const int kb = key_bytes_of(key_type);
    if (!kb) return fail(ctx, RSORT_EINVAL, "unknown key type %d", key_type);
    if ((vals_in == nullptr) != (vals_out == nullptr))
        return fail(ctx, RSORT_EINVAL, "vals_in and vals_out must both be NULL or both be set");
    if ((workspace == nullptr) != (ws_bytes == 0))
        return fail(ctx, RSORT_EINVAL, "workspace and ws_bytes must both be 0 or both be set");
    if (total_n >= kMaxN || num_segs >= kMaxN)
        return fail(ctx, RSORT_EUNSUPPORTED, "total_n or num_segs >= 2^30");
    if (num_segs == 0 || total_n == 0) return RSORT_OK;
    if (!keys_in || !keys_out || !seg_offsets) return fail(ctx, RSORT_EINVAL, "NULL pointer");
    DeviceGuard g(ctx->device);
    int rc = check_arrays(ctx, kb, keys_in, keys_out, vals_in, vals_out, total_n);
    if (rc) return rc;
    if (!is_device_pointer(seg_offsets, ctx->device))
        return fail(ctx, RSORT_EINVAL, "seg_offsets must be device memory of device %d", ctx->device);
    const rsort::DevSegLayout L = rsort::devseg_layout(kb, vals_in != nullptr, total_n, (uint32_t)num_segs);
    void* ws = workspace;
    if (ws) {
        if (ws_bytes < L.bytes)
            return fail(ctx, RSORT_EINVAL, "workspace of %zu bytes < %zu needed", ws_bytes, L.bytes);
        if (!is_device_pointer(ws, ctx->device))
            return fail(ctx, RSORT_EINVAL, "workspace must be device memory");
    } else {
        rc = ensure_workspace(ctx, L.bytes, &ws);
        if (rc) return rc;
    }
    hipError_t e = rsort::devseg_sort(kb, keys_in, keys_out, vals_in, vals_out, total_n, seg_offsets,
                                      (uint32_t)num_segs, ctx->small_max, ws, L, ctx->dev_err,
                                      (hipStream_t)stream, ctx->prof, ctx->small_sort);
    return e == hipSuccess ? RSORT_OK : hip_fail(ctx, e, "kernel launch");
}

int rsort_segmented_set_small_sort(rsort_ctx* ctx, int small_sort)
{
    if (!ctx) return RSORT_EINVAL;
    if (small_sort != RSORT_SMALL_RADIX && small_sort != RSORT_SMALL_BTN &&
        small_sort != RSORT_SMALL_OET)
        return fail(ctx, RSORT_EINVAL, "unknown small-segment sorter %d", small_sort);
    ctx->small_sort = small_sort;
    return RSORT_OK;
}

int rsort_segmented_get_small_sort(rsort_ctx* ctx, int* small_sort)
{
    if (!ctx || !small_sort) return RSORT_EINVAL;
    *small_sort = ctx->small_sort;
    return RSORT_OK;
}

int rsort_set_pr4_rounds(rsort_ctx* ctx, int kind)
{
    if (!ctx) return RSORT_EINVAL;
    if (kind != RSORT_PR4_COUNTED && kind != RSORT_PR4_SINGLE_READ)
        return fail(ctx, RSORT_EINVAL, "unknown PR4 round kind %d", kind);
    ctx->pr4_rounds = kind;
    return RSORT_OK;
}

int rsort_segmented_set_tile(rsort_ctx* ctx, int tile_threads)
{
    if (!ctx) return RSORT_EINVAL;
    int shape = -1;
    if (tile_threads == 0) shape = rsort::kSegTileShapeDefault;
    else if (tile_threads == 256) shape = 0;
    else if (tile_threads == 512) shape = 1;
    else if (tile_threads == 1024) shape = 2;
    if (shape < 0) return fail(ctx, RSORT_EINVAL, "tile workgroup of %d threads (256, 512, 1024)", tile_threads);
    ctx->seg_tile_shape = shape;
    return RSORT_OK;
}

int rsort_segmented_set_launch(rsort_ctx* ctx, int launch)
{
    if (!ctx) return RSORT_EINVAL;
    if (launch != RSORT_SEG_ROUNDS && launch != RSORT_SEG_PERSISTENT)
        return fail(ctx, RSORT_EINVAL, "unknown segmented launch mode %d", launch);
    if (launch == RSORT_SEG_PERSISTENT && !kPersistentLaunch)
        return fail(ctx, RSORT_EUNSUPPORTED, "the persistent segmented launch is switched off");
    ctx->seg_launch = launch;
    return RSORT_OK;
}

int rsort_segmented_get_config(rsort_ctx* ctx, uint32_t* small_max, int* small_sort,
                               int* tile_threads, int* radix_bits, int* launch)
{
    if (!ctx) return RSORT_EINVAL;
    static const int threads[rsort::kSegTileShapes] = {256, 512, 1024};
    const bool persistent = ctx->seg_launch == RSORT_SEG_PERSISTENT;
    if (small_max) *small_max = ctx->small_max;
    if (small_sort) *small_sort = persistent ? (int)RSORT_SMALL_RADIX : ctx->small_sort;
    if (tile_threads) *tile_threads = persistent ? rsort::persist_threads() : threads[ctx->seg_tile_shape];
    if (radix_bits) *radix_bits = 8;
    if (launch) *launch = ctx->seg_launch;
    return RSORT_OK;
}

int rsort_segmented_set_split(rsort_ctx* ctx, uint32_t small_max)
{
    if (!ctx) return RSORT_EINVAL;
    if (small_max > rsort::kSmallMaxDefault)
        return fail(ctx, RSORT_EINVAL, "small_max %u above the in-LDS capacity %u", small_max,
                    rsort::kSmallMaxDefault);
    ctx->small_max = small_max;
    return RSORT_OK;
}

int rsort_segmented_sort(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
                         const uint32_t* vals_in, uint32_t* vals_out, const uint64_t* seg_offsets,
                         size_t num_segs, void* workspace, size_t ws_bytes, void* stream)
{
    if (!ctx) return RSORT_EINVAL;
    ctx->last_error.clear();
    const int kb = key_bytes_of(key_type);
    if (!kb) return fail(ctx, RSORT_EINVAL, "unknown key type %d", key_type);
    if ((vals_in == nullptr) != (vals_out == nullptr))
        return fail(ctx, RSORT_EINVAL, "vals_in and vals_out must both be NULL or both be set");
    if ((workspace == nullptr) != (ws_bytes == 0))
        return fail(ctx, RSORT_EINVAL, "workspace and ws_bytes must both be 0 or both be set");
    size_t total = 0;
    int rc = check_offsets(ctx, seg_offsets, num_segs, &total);
    if (rc) return rc;
    if (total == 0) return RSORT_OK;
    if (!keys_in || !keys_out) return fail(ctx, RSORT_EINVAL, "NULL key pointer");

    DeviceGuard g(ctx->device);
    if (!is_device_pointer(keys_in, ctx->device) || !is_device_pointer(keys_out, ctx->device))
        return fail(ctx, RSORT_EINVAL, "key arrays must be device memory of device %d", ctx->device);
    if (vals_in && (!is_device_pointer(vals_in, ctx->device) || !is_device_pointer(vals_out, ctx->device)))
        return fail(ctx, RSORT_EINVAL, "payload arrays must be device memory of device %d", ctx->device);
    const size_t kbytes = total * kb, vbytes = total * 4;
    if (overlap_partial(keys_in, kbytes, keys_out, kbytes))
        return fail(ctx, RSORT_EINVAL, "keys_in and keys_out overlap without being equal");
    if (vals_in && overlap_partial(vals_in, vbytes, vals_out, vbytes))
        return fail(ctx, RSORT_EINVAL, "vals_in and vals_out overlap without being equal");

    rsort::SegPlan& P = ctx->plan;
    const bool persistent = ctx->seg_launch == RSORT_SEG_PERSISTENT;
    const size_t need = seg_plan_for(ctx, seg_offsets, num_segs, kb, vals_in != nullptr, total, P);
    void* ws = workspace;
    if (ws) {
        if (ws_bytes < need)
            return fail(ctx, RSORT_EINVAL, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    } else {
        rc = ensure_workspace(ctx, need, &ws);
        if (rc) return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t mb = persistent ? rsort::persist_meta_bytes(P, kb) : rsort::segmented_meta_bytes(P);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) cap = hipStreamCaptureStatusNone;
    // The plan signature: what the kernels read from the workspace's plan area.
    uint64_t sig = 1469598103934665603ull;
    auto mix = [&sig](uint64_t x) { sig = (sig ^ x) * 1099511628211ull; };
    mix((uint64_t)kb);
    mix(vals_in != nullptr);
    mix(ctx->small_max);
    mix((uint64_t)ctx->seg_tile_shape);
    mix((uint64_t)ctx->seg_launch);
    mix(num_segs);
    for (size_t i = 0; i <= num_segs; ++i) mix(seg_offsets[i]);
    if (cap == hipStreamCaptureStatusActive) {
        if (persistent)
            return fail(ctx, RSORT_EUNSUPPORTED, "the persistent segmented launch is a cooperative "
                                                 "launch, which is not captured into a graph");
        // No host traffic inside a graph: the plan must already sit in this
        // workspace from an identical call made outside the capture.
        if (sig != ctx->upload_sig || ws != ctx->upload_ws)
            return fail(ctx, RSORT_EINVAL, "capturing a segmented sort needs one identical call "
                                           "with the same workspace outside the capture first");
        // one stream inside a graph: a replay of the forked form (small segments
        // on the second stream) measured slower, 1.00 against 0.73 ms on the
        // 4096-array batch
        hipError_t e = persistent
            ? rsort::persist_sort(kb, keys_in, keys_out, vals_in, vals_out, total, P, nullptr, ws,
                                  ctx->dev_err, s, nullptr)
            : rsort::segmented_sort(kb, keys_in, keys_out, vals_in, vals_out, total, P,
                                    nullptr, ws, ctx->dev_err, s, nullptr, ctx->small_sort);
        return e == hipSuccess ? RSORT_OK : hip_fail(ctx, e, "segmented sort capture");
    }
    // pinned staging of the plan: wait until its previous upload has completed
    if (ctx->meta_pending) {
        hipError_t e = hipEventSynchronize(ctx->meta_done);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize");
        ctx->meta_pending = false;
    }
    if (mb > ctx->meta_bytes) {
        if (ctx->meta_host) (void)hipHostFree(ctx->meta_host);
        ctx->meta_host = nullptr;
        ctx->meta_bytes = 0;
        size_t grow = std::max(mb, (size_t)1 << 16);
        hipError_t e = hipHostMalloc(&ctx->meta_host, grow, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipHostMalloc(plan staging)");
        ctx->meta_bytes = grow;
    }
    if (!ctx->meta_done && hipEventCreateWithFlags(&ctx->meta_done, hipEventDisableTiming) != hipSuccess)
        return fail(ctx, RSORT_EDEVICE, "hipEventCreate");
    hipError_t e;
    if (persistent) {
        rsort::persist_pack(P, kb, ctx->meta_host);
        e = rsort::persist_sort(kb, keys_in, keys_out, vals_in, vals_out, total, P, ctx->meta_host,
                                ws, ctx->dev_err, s, ctx->prof);
    } else {
        rsort::segmented_pack(P, kb, ctx->meta_host);
        e = rsort::segmented_sort(kb, keys_in, keys_out, vals_in, vals_out, total, P,
                                  ctx->meta_host, ws, ctx->dev_err, s, ctx->prof, ctx->small_sort,
                                  seg_overlap(ctx));
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "segmented sort launch");
    if (hipEventRecord(ctx->meta_done, s) == hipSuccess) ctx->meta_pending = true;
    ctx->upload_sig = sig;
    ctx->upload_ws = ws;
    return RSORT_OK;
}

int rsort_segmented_tune(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
                         const uint32_t* vals_in, uint32_t* vals_out, const uint64_t* seg_offsets,
                         size_t num_segs, int reps, void* stream, uint32_t* best_split,
                         double* best_ms)
{
    if (!ctx || !best_split) return RSORT_EINVAL;
    // A choice persisted for this architecture, key type, payload and batch
    // size class is applied (the batch is still sorted once) instead of tuning.
    rsort::TuneKey tkey;
    memset(&tkey, 0, sizeof tkey);
    const bool use_cache = !ctx->tune_cache.empty() && seg_offsets;
    if (use_cache) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess)
            return fail(ctx, RSORT_EDEVICE, "hipGetDeviceProperties");
        rsort::set_tune_arch(&tkey, prop.gcnArchName);
        tkey.key_type = key_type;
        tkey.payload = vals_in != nullptr;
        tkey.log2_keys = rsort::ceil_log2(num_segs ? seg_offsets[num_segs] - seg_offsets[0] : 0);
        tkey.log2_segs = rsort::ceil_log2(num_segs);
        rsort::TuneEntry te;
        if (rsort::lookup_tune_entry(ctx->tune_cache.c_str(), tkey, &te)) {
            const uint32_t s0 = ctx->small_max;
            const int k0 = ctx->small_sort, t0 = ctx->seg_tile_shape, l0 = ctx->seg_launch;
            if (rsort_segmented_set_launch(ctx, te.launch) == RSORT_OK &&
                rsort_segmented_set_split(ctx, te.split) == RSORT_OK &&
                rsort_segmented_set_small_sort(ctx, te.small_sort) == RSORT_OK &&
                rsort_segmented_set_tile(ctx, te.tile_threads) == RSORT_OK) {
                int rc = rsort_segmented_sort(ctx, key_type, keys_in, keys_out, vals_in, vals_out,
                                              seg_offsets, num_segs, nullptr, 0, stream);
                if (rc == RSORT_OK) rc = rsort_synchronize(ctx, stream);
                if (rc) return rc;
                *best_split = te.split;
                if (best_ms) *best_ms = te.ms;
                return RSORT_OK;
            }
            // an entry the library cannot apply (another version): tune as if there were none
            ctx->small_max = s0;
            ctx->small_sort = k0;
            ctx->seg_tile_shape = t0;
            ctx->seg_launch = l0;
            ctx->last_error.clear();
        }
    }
    static const uint32_t cands[] = {0, 1024, 4096, 8192};
    static const int sorters[] = {RSORT_SMALL_RADIX, RSORT_SMALL_BTN, RSORT_SMALL_OET};
    if (reps < 1) reps = 3;
    hipStream_t s = (hipStream_t)stream;
    DeviceGuard g(ctx->device);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(ctx, RSORT_EDEVICE, "hipEventCreate");
    }
    const uint32_t saved = ctx->small_max;
    const int saved_sort = ctx->small_sort;
    const int saved_shape = ctx->seg_tile_shape;
    const int saved_launch = ctx->seg_launch;
    double best = 1e30;
    uint32_t pick = saved;
    int pick_sort = saved_sort;
    int pick_shape = saved_shape;
    int pick_launch = saved_launch;
    int rc = RSORT_OK;
    for (int launch : {RSORT_SEG_ROUNDS, RSORT_SEG_PERSISTENT})
    if (launch == RSORT_SEG_ROUNDS || kPersistentLaunch)
    for (uint32_t c : cands)
    for (int srt : sorters)
    for (int shape = 0; shape < rsort::kSegTileShapes && !rc; ++shape) {
        if (c == 0 && srt != RSORT_SMALL_RADIX) continue;   // no small segments
        // the persistent launch has one tile shape and sorts small segments by radix rounds
        if (launch == RSORT_SEG_PERSISTENT && (srt != RSORT_SMALL_RADIX || shape != 1)) continue;
        ctx->seg_launch = launch;
        ctx->small_max = c;
        ctx->small_sort = srt;
        ctx->seg_tile_shape = shape;
        rc = rsort_segmented_sort(ctx, key_type, keys_in, keys_out, vals_in, vals_out, seg_offsets,
                                  num_segs, nullptr, 0, stream);   // warm-up, sizes the workspace
        if (rc) break;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && !rc; ++r)
            rc = rsort_segmented_sort(ctx, key_type, keys_in, keys_out, vals_in, vals_out,
                                      seg_offsets, num_segs, nullptr, 0, stream);
        (void)hipEventRecord(e1, s);
        if (rc) break;
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(ctx, RSORT_EDEVICE, "timing");
            break;
        }
        if (ms / reps < best) {
            best = ms / reps;
            pick = c;
            pick_sort = srt;
            pick_shape = shape;
            pick_launch = launch;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->small_max = rc ? saved : pick;
    ctx->small_sort = rc ? saved_sort : pick_sort;
    ctx->seg_tile_shape = rc ? saved_shape : pick_shape;
    ctx->seg_launch = rc ? saved_launch : pick_launch;
    if (rc) return rc;
    *best_split = pick;
    if (best_ms) *best_ms = best;
    if (use_cache) {   // a file that cannot be written only means tuning again next time
        static const int threads[rsort::kSegTileShapes] = {256, 512, 1024};
        rsort::TuneEntry te;
        te.key = tkey;
        te.split = pick;
        te.small_sort = pick_sort;
        te.tile_threads = threads[pick_shape];
        te.launch = pick_launch;
        te.ms = best;
        (void)rsort::append_tune_entry(ctx->tune_cache.c_str(), te);
    }
    return RSORT_OK;
}

int rsort_synchronize(rsort_ctx* ctx, void* stream)
{
    if (!ctx) return RSORT_EINVAL;
    DeviceGuard g(ctx->device);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    uint32_t err = 0;
    e = hipMemcpy(&err, ctx->dev_err, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy(error word)");
    if (err) {
        (void)hipMemset(ctx->dev_err, 0, 4);
        return fail(ctx, RSORT_EDEVICE, "device-side failure bits 0x%x%s%s", err,
                    (err & 1u) ? " (look-back wait timed out)" : "",
                    (err & 2u) ? " (invalid device segment offsets: nothing sorted)" : "");
    }
    return RSORT_OK;
}

}  // extern "C"
