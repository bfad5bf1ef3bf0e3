// Batched segmented sort in one persistent launch: the segmented sort of
// arXiv 1808.10292 Section 3.2's SR4 per segment (as in segmented.hip), every
// segment and every round inside a single kernel.
//
// A resident grid (cooperative launch: every workgroup is on the chip at
// once) walks through phases separated by grid-wide barriers; inside a phase
// workgroup b takes items b, b + G, b + 2G, ... (G workgroups):
//
//   1      the whole small segments, each sorted in LDS (one counting round
//          per digit, read once, written once); and every tile of the large
//          segments: its digit counts of round 0 and the OR of every key's
//          difference from its segment's first key (the identity words)
//   per round r of the key's digits:
//   C(r)   (r > 0) every tile: its digit counts in the round's input
//   X(r)   every large segment: (r = 0) its round plan from the identity
//          words -- a round whose digit is the same for every key of the
//          segment is skipped, the rounds that run alternate between the
//          temporary and the output so that the last one writes the output --
//          then the output start of every (tile, digit) run: segment start +
//          keys of smaller digits in the segment + keys of the digit in the
//          segment's earlier tiles
//   W(r)   every tile: a stable counting round in LDS (tile_round), then each
//          key written to its run's output start + its place in the run
//
// The barrier is a counter that only grows (the k-th barrier waits for k x G
// arrivals), cleared by a fill kernel before the launch; its wait is bounded
// (kSpinLimit polls) and a wait that gives up records kErrLookbackTimeout, so
// the launch always ends.  Every global write is bounded by the batch size.
#include <algorithm>
#include <cstring>
#include <vector>

#include "lsd_kernels.h"
#include "tile_sort.h"

namespace rsort {
namespace {

// Keys per thread of a tile (32-bit keys; 64-bit keys take half) and the
// waves per SIMD the kernel is compiled for (its registers).
#ifndef RSORT_PERSIST_ITEMS32
#define RSORT_PERSIST_ITEMS32 8
#endif
#ifndef RSORT_PERSIST_WAVES
#define RSORT_PERSIST_WAVES 4
#endif
#ifndef RSORT_PERSIST_WG
#define RSORT_PERSIST_WG 512
#endif
constexpr int kPWG = RSORT_PERSIST_WG;
constexpr int kPSmallItems = 4;   // small segments of at most kPWG * 4 keys: the short form
constexpr int kPCols = 8;         // LDS count replicas (spread the atomics of equal digits)
template <typename K> struct PCfg;
template <> struct PCfg<uint32_t> { static constexpr int ITEMS = RSORT_PERSIST_ITEMS32; };
template <> struct PCfg<uint64_t> { static constexpr int ITEMS = RSORT_PERSIST_ITEMS32 / 2; };
// The host plan cuts the large segments into tiles of one of the segmented
// sort's tile shapes (256, 512 or 1024 threads x 16 keys, x 8 for 64-bit
// keys); the persistent kernel's tile must be one of them.
static_assert(kPWG * RSORT_PERSIST_ITEMS32 == 256 * 16 || kPWG * RSORT_PERSIST_ITEMS32 == 512 * 16 ||
                  kPWG * RSORT_PERSIST_ITEMS32 == 1024 * 16,
              "the persistent tile is a tile shape of the plan");

struct PArgs {
    const void* keys_in;
    void* keys_out;
    void* keys_tmp;
    const uint32_t* vals_in;
    uint32_t* vals_out;
    uint32_t* vals_tmp;
    const uint2* small;       // {first key, end} per small segment
    const uint4* lsegs;       // {first tile, end tile, first key, 0} per large segment
    const uint2* tiles;       // {first key, end key} per tile
    const uint32_t* tile_seg; // large segment of every tile
    uint32_t nsmall, nls, nt;
    uint32_t n;               // keys in the batch
    uint32_t* cnt;            // [tile][256] digit counts of the tile in the current round
    uint32_t* start;          // [tile][256] output start of the tile's run of each digit
    uint32_t* seg_or;         // [segment][2] identity words
    RoundPlan* seg_plan;      // [segment][kMaxRounds + 1]
    uint32_t* bar;            // grid barrier counter
    int alias;
    uint32_t* err;
};

// Zero `count` words (the identity words and the barrier before the launch).
__global__ void k_persist_zero(uint32_t* words, uint32_t count)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        words[i] = 0;
}

// Every workgroup of the launch arrives here before any continues; k counts
// the barriers this workgroup has passed.  Each thread releases its own
// global writes at agent scope before the workgroup arrives, and acquires
// after the wait.
__device__ __forceinline__ void grid_barrier(const PArgs& a, uint32_t& k)
{
    ++k;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(a.bar, 1u);
        const uint32_t want = k * gridDim.x;
        uint32_t spins = 0;
        while (ld_agent(a.bar) < want) {
            if (++spins > kSpinLimit || ((spins & 255u) == 0 && (ld_agent(a.err) & kErrLookbackTimeout))) {
                atomicOr(a.err, (uint32_t)kErrLookbackTimeout);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    __threadfence();
}

template <typename K>
__device__ __forceinline__ K* pick_buf(int which, const PArgs& a)
{
    return which == 0 ? (K*)a.keys_in : which == 1 ? (K*)a.keys_out : (K*)a.keys_tmp;
}
__device__ __forceinline__ uint32_t* pick_vbuf(int which, const PArgs& a)
{
    return which == 0 ? (uint32_t*)a.vals_in : which == 1 ? a.vals_out : a.vals_tmp;
}

// Data written by other workgroups earlier in the launch (keys of the round
// before, tile counts, run starts, plans) is read with agent-scope loads, which
// the memory model makes coherent across the XCDs' L2 caches; the barrier
// orders them after the writes.
__device__ __forceinline__ RoundPlan load_plan(const RoundPlan* p)
{
    const int32_t* w = reinterpret_cast<const int32_t*>(p);
    RoundPlan r;
    r.exec = ld_agent(&w[0]);
    r.ord = ld_agent(&w[1]);
    r.src = ld_agent(&w[2]);
    r.dst = ld_agent(&w[3]);
    return r;
}

// Inclusive sum over the first 256 threads (4 waves); all threads call.
__device__ __forceinline__ uint32_t sum256(uint32_t x, uint32_t* wsum)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t incl = 0;
    if (tid < 256) {
        incl = wave_inclusive_sum(x);
        if (lane == 63) wsum[wave] = incl;
    }
    __syncthreads();
    if (tid < 256)
        for (uint32_t q = 0; q < wave; ++q) incl += wsum[q];
    __syncthreads();
    return incl;
}

// A small segment [lo, hi) sorted whole in LDS, input to output.
template <typename K, bool KV, int ITEMS>
__device__ void small_item(const PArgs& a, unsigned char* raw, uint32_t lo, uint32_t hi)
{
    auto& sm = *reinterpret_cast<TileSmem<K, KV, kPWG, ITEMS, true>*>(raw);
    const uint32_t tid = threadIdx.x;
    const uint32_t hofs = (tid >> 5) * ITEMS * 32 + (tid & 31);
    const uint32_t len = hi - lo;
    const K* kin = (const K*)a.keys_in;
    K k[ITEMS];
    uint32_t v[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t o = hofs + i * 32;
        k[i] = o < len ? kin[lo + o] : K(0);
        v[i] = KV && o < len ? a.vals_in[lo + o] : 0u;
    }
    for (uint32_t r = 0; r < sizeof(K); ++r)
        tile_round<K, KV, kPWG, ITEMS, true>(sm, k, v, len, 8u * r, 0xFFu);
    K* kout = (K*)a.keys_out;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t o = hofs + i * 32;
        if (o < len) {
            kout[lo + o] = k[i];
            if (KV) a.vals_out[lo + o] = v[i];
        }
    }
    __syncthreads();   // LDS free for the next item
}

// C(r): the digit counts of round r of tile g (round 0 also ORs every key's
// difference from its segment's first key into the identity words).
template <typename K>
__device__ void count_item(const PArgs& a, unsigned char* raw, uint32_t r, uint32_t g)
{
    constexpr int ITEMS = PCfg<K>::ITEMS;
    const uint32_t tid = threadIdx.x;
    const uint32_t s = a.tile_seg[g];
    const K* src = (const K*)a.keys_in;
    if (r > 0) {
        const RoundPlan pl = load_plan(&a.seg_plan[(size_t)s * (kMaxRounds + 1) + r]);
        if (pl.exec != 1) return;   // uniform over the workgroup
        src = pick_buf<K>(pl.src, a);
    }
    uint32_t* h = reinterpret_cast<uint32_t*>(raw);   // [256][kPCols], then 2 identity words
    for (uint32_t i = tid; i < R * kPCols + 2; i += kPWG) h[i] = 0;
    __syncthreads();
    const uint2 tr = a.tiles[g];
    const K first = ((const K*)a.keys_in)[a.lsegs[s].z];
    const uint32_t col = tid & (kPCols - 1);
    uint64_t acc = 0;
    K kk[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t i = tr.x + j * kPWG + tid;
        kk[j] = i < tr.y ? (r == 0 ? src[i] : ld_agent(&src[i])) : K(0);
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        if (tr.x + j * kPWG + tid < tr.y) {
            atomicAdd(&h[digit_of(kk[j], 8u * r, 0xFFu) * kPCols + col], 1u);
            if (r == 0) acc |= (uint64_t)(kk[j] ^ first);
        }
    }
    if (r == 0) {
        uint32_t lo = (uint32_t)acc, hi = (uint32_t)(acc >> 32);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            lo |= __shfl_xor(lo, o, 64);
            hi |= __shfl_xor(hi, o, 64);
        }
        if ((tid & 63) == 0) {
            if (lo) atomicOr(&h[R * kPCols], lo);
            if (hi) atomicOr(&h[R * kPCols + 1], hi);
        }
    }
    __syncthreads();
    if (tid < R) {
        uint32_t c = 0;
#pragma unroll
        for (int q = 0; q < kPCols; ++q) c += h[tid * kPCols + q];
        a.cnt[(size_t)g * R + tid] = c;
    }
    if (r == 0 && tid < 2) {
        const uint32_t m = h[R * kPCols + tid];
        if (m) atomicOr(&a.seg_or[2 * s + tid], m);
    }
    __syncthreads();   // LDS free for the next item
}

// X(r): large segment s -- (r = 0) its round plan; then the output start of
// every (tile, digit) run of the segment in round r.
template <typename K>
__device__ void scan_item(const PArgs& a, uint32_t* wsum, RoundPlan* plan_s, uint32_t r, uint32_t s)
{
    constexpr uint32_t NR = sizeof(K);
    const uint32_t tid = threadIdx.x;
    RoundPlan* plan = a.seg_plan + (size_t)s * (kMaxRounds + 1);
    if (tid == 0) {
        if (r == 0) {
            const uint64_t mx = (uint64_t)ld_agent(&a.seg_or[2 * s]) |
                                ((uint64_t)ld_agent(&a.seg_or[2 * s + 1]) << 32);
            int identity[kMaxRounds];
            for (uint32_t d = 0; d < NR; ++d) identity[d] = ((mx >> (8u * d)) & 0xFFull) == 0;
            plan_rounds(identity, NR, a.alias, plan);
        }
        *plan_s = load_plan(&plan[r]);
    }
    __syncthreads();
    const RoundPlan pl = *plan_s;
    __syncthreads();   // plan_s read by all before the next item rewrites it
    if (pl.exec != 1) return;
    const uint4 sg = a.lsegs[s];
    // thread v < 256: digit v over the segment's tiles, loads in batches of B
    constexpr uint32_t B = 16;
    uint32_t total = 0;
    if (tid < R) {
        for (uint32_t t = sg.x; t < sg.y; t += B) {
            uint32_t c[B];
#pragma unroll
            for (uint32_t j = 0; j < B; ++j) c[j] = t + j < sg.y ? ld_agent(&a.cnt[(size_t)(t + j) * R + tid]) : 0u;
#pragma unroll
            for (uint32_t j = 0; j < B; ++j) total += c[j];
        }
    }
    const uint32_t incl = sum256(total, wsum);
    if (tid < R) {
        uint32_t run = sg.z + incl - total;
        for (uint32_t t = sg.x; t < sg.y; t += B) {
            uint32_t c[B];
#pragma unroll
            for (uint32_t j = 0; j < B; ++j) c[j] = t + j < sg.y ? ld_agent(&a.cnt[(size_t)(t + j) * R + tid]) : 0u;
#pragma unroll
            for (uint32_t j = 0; j < B; ++j)
                if (t + j < sg.y) {
                    a.start[(size_t)(t + j) * R + tid] = run;
                    run += c[j];
                }
        }
    }
}

// W(r): tile g's round r -- stable counting round in LDS, then every key to
// its run's output start + its place in the run.
template <typename K, bool KV>
__device__ void scatter_item(const PArgs& a, unsigned char* raw, uint32_t* goff, uint32_t* wsum,
                             uint32_t r, uint32_t g)
{
    constexpr int ITEMS = PCfg<K>::ITEMS;
    auto& sm = *reinterpret_cast<TileSmem<K, KV, kPWG, ITEMS, true>*>(raw);
    const uint32_t tid = threadIdx.x;
    const uint32_t s = a.tile_seg[g];
    const RoundPlan pl = load_plan(&a.seg_plan[(size_t)s * (kMaxRounds + 1) + r]);
    if (pl.exec == 0) return;   // uniform over the workgroup
    const uint2 tr = a.tiles[g];
    const uint32_t len = tr.y - tr.x;
    if (pl.exec == 2) {
        // every round of the segment is the identity: copy the tile
        const K* kin = (const K*)a.keys_in;
        K* kout = (K*)a.keys_out;
        for (uint32_t i = tid; i < len; i += kPWG) {
            kout[tr.x + i] = kin[tr.x + i];
            if (KV) a.vals_out[tr.x + i] = a.vals_in[tr.x + i];
        }
        return;
    }
    const K* src = pick_buf<K>(pl.src, a);
    K* dst = pick_buf<K>(pl.dst, a);
    const uint32_t* vsrc = KV ? pick_vbuf(pl.src, a) : nullptr;
    uint32_t* vdst = KV ? pick_vbuf(pl.dst, a) : nullptr;
    const uint32_t hofs = (tid >> 5) * ITEMS * 32 + (tid & 31);
    K k[ITEMS];
    uint32_t v[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t o = hofs + i * 32;
        k[i] = o < len ? ld_agent(&src[tr.x + o]) : K(0);
        v[i] = KV && o < len ? ld_agent(&vsrc[tr.x + o]) : 0u;
    }
    // goff[v] = output index of sorted tile position 0 of digit v's run
    const uint32_t c = tid < R ? ld_agent(&a.cnt[(size_t)g * R + tid]) : 0u;
    const uint32_t st = tid < R ? ld_agent(&a.start[(size_t)g * R + tid]) : 0u;
    const uint32_t incl = sum256(c, wsum);
    if (tid < R) goff[tid] = st - (incl - c);
    const uint32_t shift = 8u * r;
    const bool held = tile_round<K, KV, kPWG, ITEMS, true>(sm, k, v, len, shift, 0xFFu);
    if (held) {
        // LDS holds the tile in digit order
        for (uint32_t p = tid; p < len; p += kPWG) {
            const K key = sm.keys[p];
            const uint32_t o = goff[digit_of(key, shift, 0xFFu)] + p;
            if (o < a.n) {   // always true with consistent counts
                dst[o] = key;
                if (KV) vdst[o] = sm.vals[p];
            }
        }
    } else {
        // one digit value holds the whole tile: the order is unchanged
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = hofs + i * 32;
            if (p < len) {
                const uint32_t o = goff[digit_of(k[i], shift, 0xFFu)] + p;
                if (o < a.n) {
                    dst[o] = k[i];
                    if (KV) vdst[o] = v[i];
                }
            }
        }
    }
    __syncthreads();   // LDS and goff free for the next item
}

template <typename K, bool KV>
__global__ __launch_bounds__(kPWG, RSORT_PERSIST_WAVES) void k_seg_persist(PArgs a)
{
    constexpr int ITEMS = PCfg<K>::ITEMS;
    constexpr uint32_t NR = sizeof(K);
    constexpr size_t kBig = sizeof(TileSmem<K, KV, kPWG, ITEMS, true>);
    constexpr size_t kSmall = sizeof(TileSmem<K, KV, kPWG, kPSmallItems, true>);
    constexpr size_t kCount = (R * kPCols + 2) * 4;
    constexpr size_t kBS = kBig > kSmall ? kBig : kSmall;
    constexpr size_t kRaw = kBS > kCount ? kBS : kCount;
    __shared__ alignas(16) unsigned char raw[kRaw];
    __shared__ uint32_t goff[R];
    __shared__ uint32_t wsum[4];
    __shared__ RoundPlan plan_s;
    const uint32_t b = blockIdx.x, G = gridDim.x;
    uint32_t nbar = 0;
    // 1: small segments, and round 0's tile counts with the identity words
    for (uint32_t i = b; i < a.nt + a.nsmall; i += G) {
        if (i < a.nt) {
            count_item<K>(a, raw, 0, i);
        } else {
            const uint2 sg = a.small[i - a.nt];
            if (sg.y - sg.x <= (uint32_t)(kPWG * kPSmallItems))
                small_item<K, KV, kPSmallItems>(a, raw, sg.x, sg.y);
            else
                small_item<K, KV, ITEMS>(a, raw, sg.x, sg.y);
        }
    }
    if (a.nt == 0) return;   // small segments only: nothing else to wait for
    grid_barrier(a, nbar);
    for (uint32_t r = 0; r < NR; ++r) {
        if (r > 0) {
            for (uint32_t g = b; g < a.nt; g += G) count_item<K>(a, raw, r, g);
            grid_barrier(a, nbar);
        }
        for (uint32_t s = b; s < a.nls; s += G) scan_item<K>(a, wsum, &plan_s, r, s);
        grid_barrier(a, nbar);
        for (uint32_t g = b; g < a.nt; g += G) scatter_item<K, KV>(a, raw, goff, wsum, r, g);
        if (r + 1 < NR) grid_barrier(a, nbar);
    }
}

}  // namespace

uint32_t persist_small_max(int key_bytes)
{
    return key_bytes == 8 ? kPWG * PCfg<uint64_t>::ITEMS : kPWG * PCfg<uint32_t>::ITEMS;
}

int persist_threads() { return kPWG; }

int persist_tile_shape(int key_bytes)
{
    for (int s = 0; s < kSegTileShapes; ++s)
        if (seg_tile_keys(key_bytes, s) == persist_small_max(key_bytes)) return s;
    return -1;
}

// Work lists: lsegs (uint4), tiles (uint2), tile_seg (u32), small (uint2).
size_t persist_meta_bytes(const SegPlan& P, int key_bytes)
{
    (void)key_bytes;
    const size_t nsmall = P.small[0].size() + P.small[1].size() + P.small[2].size();
    return align_up(P.lsegs.size() * sizeof(uint4)) + align_up(P.tiles.size() * sizeof(uint2)) +
           align_up(P.tile_seg.size() * sizeof(uint32_t)) + nsmall * sizeof(uint2);
}

size_t persist_ws_bytes(int key_bytes, bool has_vals, size_t total, const SegPlan& P)
{
    const size_t nt = P.tiles.size(), nls = P.lsegs.size();
    size_t o = 0;
    o = align_up(o + (nt ? total * key_bytes : 0));                 // tmp keys
    o = align_up(o + (nt && has_vals ? total * 4 : 0));             // tmp vals
    o = align_up(o + nt * R * 4);                                   // tile counts
    o = align_up(o + nt * R * 4);                                   // run output starts
    o = align_up(o + (2 * nls + 1) * 4);                            // identity words, barrier
    o = align_up(o + nls * (kMaxRounds + 1) * sizeof(RoundPlan));   // segment plans
    o = align_up(o + persist_meta_bytes(P, key_bytes));             // work lists
    return o;
}

void persist_pack(const SegPlan& P, int key_bytes, void* host)
{
    (void)key_bytes;
    uint8_t* h = (uint8_t*)host;
    memcpy(h, P.lsegs.data(), P.lsegs.size() * sizeof(uint4));
    h += align_up(P.lsegs.size() * sizeof(uint4));
    memcpy(h, P.tiles.data(), P.tiles.size() * sizeof(uint2));
    h += align_up(P.tiles.size() * sizeof(uint2));
    memcpy(h, P.tile_seg.data(), P.tile_seg.size() * sizeof(uint32_t));
    h += align_up(P.tile_seg.size() * sizeof(uint32_t));
    uint2* sm = (uint2*)h;
    for (int c = 2; c >= 0; --c)   // larger classes first
        for (const uint2& sg : P.small[c]) *sm++ = sg;
}

namespace {

template <typename K, bool KV>
hipError_t run_persist(const void* keys_in, void* keys_out, const uint32_t* vals_in,
                       uint32_t* vals_out, size_t total, const SegPlan& P, const void* host_meta,
                       void* ws, uint32_t* dev_err, hipStream_t stream, Profiler* prof)
{
    const size_t nt = P.tiles.size(), nls = P.lsegs.size();
    const size_t nsmall = P.small[0].size() + P.small[1].size() + P.small[2].size();
    if (!nt && !nsmall) return hipSuccess;
    uint8_t* w = (uint8_t*)ws;
    size_t o = 0;
    PArgs a{};
    a.keys_in = keys_in;
    a.keys_out = keys_out;
    a.vals_in = vals_in;
    a.vals_out = vals_out;
    a.keys_tmp = w + o;                 o = align_up(o + (nt ? total * sizeof(K) : 0));
    a.vals_tmp = (uint32_t*)(w + o);    o = align_up(o + (nt && KV ? total * 4 : 0));
    a.cnt = (uint32_t*)(w + o);         o = align_up(o + nt * R * 4);
    a.start = (uint32_t*)(w + o);       o = align_up(o + nt * R * 4);
    a.seg_or = (uint32_t*)(w + o);
    a.bar = a.seg_or + 2 * nls;         o = align_up(o + (2 * nls + 1) * 4);
    a.seg_plan = (RoundPlan*)(w + o);   o = align_up(o + nls * (kMaxRounds + 1) * sizeof(RoundPlan));
    uint8_t* meta = w + o;
    const size_t mb = persist_meta_bytes(P, (int)sizeof(K));
    if (host_meta) {   // null: the work lists are already in the workspace
        hipError_t e = hipMemcpyAsync(meta, host_meta, mb, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return e;
    }
    a.lsegs = (const uint4*)meta;
    a.tiles = (const uint2*)(meta + align_up(nls * sizeof(uint4)));
    a.tile_seg = (const uint32_t*)(meta + align_up(nls * sizeof(uint4)) + align_up(nt * sizeof(uint2)));
    a.small = (const uint2*)(meta + align_up(nls * sizeof(uint4)) + align_up(nt * sizeof(uint2)) +
                             align_up(nt * sizeof(uint32_t)));
    a.nsmall = (uint32_t)nsmall;
    a.nls = (uint32_t)nls;
    a.nt = (uint32_t)nt;
    a.n = (uint32_t)total;
    const bool keys_alias = keys_in == keys_out, vals_alias = KV && vals_in == vals_out;
    a.alias = (keys_alias || vals_alias ? kAliasAny : 0) | (keys_alias && (!KV || vals_alias) ? kAliasAll : 0);
    a.err = dev_err;
    const uint32_t nzero = (uint32_t)(2 * nls + 1);
    hipLaunchKernelGGL(k_persist_zero, dim3(std::min<uint32_t>(64, (nzero + 255) / 256)), dim3(256), 0,
                       stream, a.seg_or, nzero);
    // a resident grid: at most what the chip holds at once, at most the items
    static int grid_cache[2][2] = {{0, 0}, {0, 0}};
    int& resident = grid_cache[sizeof(K) == 8][KV];
    if (!resident) {
        int dev = 0, cus = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_seg_persist<K, KV>, kPWG, 0);
        resident = std::max(1, cus) * std::max(1, per);
    }
    const uint32_t grid = (uint32_t)std::min<size_t>((size_t)resident, std::max<size_t>(1, nt + nsmall));
    if (prof) profiler_mark(prof, stream, kKindRound, true);
    void* args[] = {&a};
    hipError_t e = hipLaunchCooperativeKernel((const void*)k_seg_persist<K, KV>, dim3(grid), dim3(kPWG),
                                              args, 0, stream);
    if (prof) profiler_mark(prof, stream, kKindRound, false);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace

hipError_t persist_sort(int key_bytes, const void* keys_in, void* keys_out, const uint32_t* vals_in,
                        uint32_t* vals_out, size_t total, const SegPlan& P, const void* host_meta,
                        void* ws, uint32_t* dev_err, hipStream_t stream, Profiler* prof)
{
    const bool kv = vals_in != nullptr;
    if (key_bytes == 4)
        return kv ? run_persist<uint32_t, true>(keys_in, keys_out, vals_in, vals_out, total, P, host_meta, ws, dev_err, stream, prof)
                  : run_persist<uint32_t, false>(keys_in, keys_out, vals_in, vals_out, total, P, host_meta, ws, dev_err, stream, prof);
    return kv ? run_persist<uint64_t, true>(keys_in, keys_out, vals_in, vals_out, total, P, host_meta, ws, dev_err, stream, prof)
              : run_persist<uint64_t, false>(keys_in, keys_out, vals_in, vals_out, total, P, host_meta, ws, dev_err, stream, prof);
}

}  // namespace rsort
