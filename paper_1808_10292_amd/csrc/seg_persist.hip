// Batched segmented sort in one persistent launch (the segmented sort of
// arXiv 1808.10292 Section 3.2's SR4 per segment, as in segmented.hip, with
// every segment and round in a single kernel).
//
// Workgroups stay resident and take work items from one ticket counter, in a
// fixed order in which every item depends only on items handed out before it:
//
//   H(s, t)     every tile t of every large segment s: the digit histograms of
//               all rounds and the OR of every key's difference from the
//               segment's first key (one read of the tile).  The last H item
//               of a segment (a per-segment counter) adds up the segment's
//               histograms into its digit starts for every round and makes its
//               round plan (rounds whose digit holds one value are skipped;
//               the rounds that run alternate between the temporary and the
//               output so that the last one writes the output);
//   S(lo, hi)   every small segment: sorted whole in LDS, one counting round
//               per digit, read once and written once;
//   R(r, s, t)  round by round, every tile of every large segment: wait for
//               the segment's plan and for its previous round to be complete
//               (a per-segment, per-round counter of finished tiles), count the
//               tile's digits, publish them and fold in those of the earlier
//               tiles of the same segment by decoupled look-back (flag + count
//               words, two buffers alternating by round), rank the tile stably
//               in LDS and write its digit runs to
//                   segment start + digit start in the segment
//                   + keys of the digit in earlier tiles + rank in the tile.
//
// A workgroup waits only on items with smaller tickets, which are held by
// workgroups already running, so the launch cannot deadlock whatever the grid
// size; every wait is bounded (kSpinLimit polls) and a wait that gives up
// records kErrLookbackTimeout, so the grid always drains.  The counters are
// cleared by a fill kernel before the launch; the look-back words are cleared
// by the items themselves (H clears both buffers of its tile, R of round r
// clears the buffer round r + 1 uses, whose previous contents belong to round
// r - 1, complete before round r started).
#include <algorithm>
#include <cstring>
#include <vector>

#include "lsd_kernels.h"
#include "tile_sort.h"

namespace rsort {
namespace {

constexpr int kPWG = 512;
constexpr int kPHW = kPWG / 32;          // half-waves
constexpr int kPSmallItems = 4;          // small segments of at most kPWG * 4 keys
template <typename K> struct PCfg;
template <> struct PCfg<uint32_t> { static constexpr int ITEMS = 16; };
template <> struct PCfg<uint64_t> { static constexpr int ITEMS = 8; };

enum : uint32_t { kItemHist = 0, kItemSmall = 1, kItemRound = 2, kItemEnd = 3 };

struct PArgs {
    const void* keys_in;
    void* keys_out;
    void* keys_tmp;
    const uint32_t* vals_in;
    uint32_t* vals_out;
    uint32_t* vals_tmp;
    const uint4* items;      // {kind | round << 8, a, b, 0}
    uint32_t nitems;
    const uint4* lsegs;      // {first tile, end tile, first key, 0}
    const uint2* tiles;      // {first key, end key}
    uint32_t* tile_hist;     // [tile][rounds][256]
    uint32_t* tile_or;       // [tile][2]
    uint32_t* seg_base;      // [segment][rounds][256] digit starts inside the segment
    RoundPlan* seg_plan;     // [segment][kMaxRounds + 1]
    uint32_t* state;         // [tile][2][256] look-back words
    uint32_t* ctl;           // ticket, then per segment: H done, plan ready, tiles done per round
    uint32_t nls;
    uint32_t n;              // keys in the batch
    int alias;
    uint32_t* err;
};

// Zero `count` words (the counters before the launch).
__global__ void k_persist_zero(uint32_t* words, uint32_t count)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        words[i] = 0;
}

__device__ __forceinline__ uint32_t* hist_done(const PArgs& a, uint32_t s) { return a.ctl + 1 + s; }
__device__ __forceinline__ uint32_t* plan_ready(const PArgs& a, uint32_t s) { return a.ctl + 1 + a.nls + s; }
template <uint32_t NR>
__device__ __forceinline__ uint32_t* round_done(const PArgs& a, uint32_t s, uint32_t r)
{
    return a.ctl + 1 + 2 * a.nls + (size_t)s * NR + r;
}

// Poll *p until it reaches `want` (bounded); thread 0 only.
__device__ __forceinline__ void wait_for(const uint32_t* p, uint32_t want, uint32_t* err)
{
    uint32_t spins = 0;
    while (ld_agent(p) < want) {
        if (++spins > kSpinLimit || ((spins & 255u) == 0 && (ld_agent(err) & kErrLookbackTimeout))) {
            atomicOr(err, (uint32_t)kErrLookbackTimeout);
            return;
        }
        __builtin_amdgcn_s_sleep(2);
    }
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

// A small segment [lo, hi) sorted whole in LDS.
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

// H(s, g): histograms and identity bits of tile g of large segment s.
template <typename K, bool KV>
__device__ void hist_item(const PArgs& a, unsigned char* raw, uint32_t* wsum, uint32_t* flag,
                          uint32_t s, uint32_t g)
{
    constexpr uint32_t NR = sizeof(K);
    constexpr int ITEMS = PCfg<K>::ITEMS;
    uint32_t* h = reinterpret_cast<uint32_t*>(raw);   // [NR][256], then 2 OR words
    const uint32_t tid = threadIdx.x;
    const uint4 ls = a.lsegs[s];
    const uint2 tr = a.tiles[g];
    for (uint32_t i = tid; i < NR * R + 2; i += kPWG) h[i] = 0;
    __syncthreads();
    const K* kin = (const K*)a.keys_in;
    const K first = kin[ls.z];
    uint64_t acc = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
        const uint32_t i = tr.x + j * kPWG + tid;
        if (i < tr.y) {
            const K key = kin[i];
            acc |= (uint64_t)(key ^ first);
#pragma unroll
            for (uint32_t r = 0; r < NR; ++r) atomicAdd(&h[r * R + digit_of(key, 8u * r, 0xFFu)], 1u);
        }
    }
    uint32_t lo = (uint32_t)acc, hi = (uint32_t)(acc >> 32);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        lo |= __shfl_xor(lo, o, 64);
        hi |= __shfl_xor(hi, o, 64);
    }
    if ((tid & 63) == 0) {
        if (lo) atomicOr(&h[NR * R], lo);
        if (hi) atomicOr(&h[NR * R + 1], hi);
    }
    __syncthreads();
    for (uint32_t i = tid; i < NR * R; i += kPWG) a.tile_hist[(size_t)g * NR * R + i] = h[i];
    if (tid < 2) a.tile_or[2 * g + tid] = h[NR * R + tid];
    for (uint32_t i = tid; i < 2 * R; i += kPWG) a.state[(size_t)g * 2 * R + i] = 0;
    __threadfence();
    __syncthreads();
    if (tid == 0) *flag = atomicAdd(hist_done(a, s), 1u) == ls.y - ls.x - 1;
    __syncthreads();
    if (*flag) {
        // the segment's last histogram tile: digit starts and round plan
        __threadfence();
        uint32_t orw[2] = {0, 0};
        for (uint32_t i = tid; i < NR * R; i += kPWG) {
            uint32_t t = 0;
            for (uint32_t q = ls.x; q < ls.y; ++q) t += a.tile_hist[(size_t)q * NR * R + i];
            h[i] = t;
        }
        if (tid < 2)
            for (uint32_t q = ls.x; q < ls.y; ++q) orw[tid] |= a.tile_or[2 * q + tid];
        __syncthreads();
        if (tid < 2) h[NR * R + tid] = orw[tid];
        for (uint32_t r = 0; r < NR; ++r) {
            const uint32_t c = tid < R ? h[r * R + tid] : 0u;
            const uint32_t incl = sum256(c, wsum);
            if (tid < R) a.seg_base[((size_t)s * NR + r) * R + tid] = incl - c;
        }
        if (tid == 0) {
            const uint64_t mx = (uint64_t)h[NR * R] | ((uint64_t)h[NR * R + 1] << 32);
            int identity[kMaxRounds];
            for (uint32_t r = 0; r < NR; ++r) identity[r] = ((mx >> (8u * r)) & 0xFFull) == 0;
            plan_rounds(identity, NR, a.alias, a.seg_plan + (size_t)s * (kMaxRounds + 1));
        }
        __threadfence();
        __syncthreads();
        if (tid == 0) atomicAdd(plan_ready(a, s), 1u);
    }
    __syncthreads();   // LDS free for the next item
}

// R(r, s, g): round r of tile g of large segment s.
template <typename K, bool KV>
__device__ void round_item(const PArgs& a, unsigned char* raw, uint32_t* wsum, uint32_t* goff,
                           uint32_t r, uint32_t s, uint32_t g)
{
    constexpr uint32_t NR = sizeof(K);
    constexpr int ITEMS = PCfg<K>::ITEMS;
    auto& sm = *reinterpret_cast<TileSmem<K, KV, kPWG, ITEMS, true>*>(raw);
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    const uint32_t hw = tid >> 5, hl = tid & 31;
    const uint32_t hofs = hw * ITEMS * 32 + hl;
    const uint4 ls = a.lsegs[s];
    const uint2 tr = a.tiles[g];
    const uint32_t len = tr.y - tr.x;
    const uint32_t ntl = ls.y - ls.x;
    if (tid == 0) {
        wait_for(plan_ready(a, s), 1u, a.err);
        if (r > 0) wait_for(round_done<NR>(a, s, r - 1), ntl, a.err);
    }
    __syncthreads();
    __threadfence();   // see the plan, the digit starts and the previous round's keys
    const RoundPlan pl = a.seg_plan[(size_t)s * (kMaxRounds + 1) + r];
    uint32_t* st = a.state + (size_t)g * 2 * R;
    if (pl.exec == 2) {
        // every round of the segment is the identity: copy the tile
        const K* kin = (const K*)a.keys_in;
        K* kout = (K*)a.keys_out;
        for (uint32_t i = tr.x + tid; i < tr.y; i += kPWG) {
            kout[i] = kin[i];
            if (KV) a.vals_out[i] = a.vals_in[i];
        }
    } else if (pl.exec == 1) {
        const uint32_t shift = 8u * r;
        const K* src = pick_buf<K>(pl.src, a);
        K* dst = pick_buf<K>(pl.dst, a);
        const uint32_t* vsrc = KV ? pick_vbuf(pl.src, a) : nullptr;
        uint32_t* vdst = KV ? pick_vbuf(pl.dst, a) : nullptr;
        K k[ITEMS];
        uint32_t v[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t o = hofs + i * 32;
            k[i] = o < len ? src[tr.x + o] : K(0);
            v[i] = KV && o < len ? vsrc[tr.x + o] : 0u;
        }
        for (uint32_t i = tid; i < kPHW * R / 2; i += kPWG)
            ((uint4*)&sm.slot[0][0])[i] = make_uint4(0, 0, 0, 0);
        __syncthreads();
        uint2* sl = sm.slot[hw];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const bool ok = hofs + i * 32 < len;
            const uint32_t d = digit_of(k[i], shift, 0xFFu);
            if (wave_one_digit(ok, d)) {
                if (hl == 0) atomicAdd(&sl[d].y, 32u);
                continue;
            }
            if (ok) atomicAdd(&sl[d].y, 1u);
        }
        __syncthreads();
        uint32_t total = 0;
        if (tid < R)
#pragma unroll
            for (int q = 0; q < kPHW; ++q) total += sm.slot[q][tid].y;
        const uint32_t incl = sum256(total, wsum);
        if (tid < R) {
            uint32_t run = incl - total;   // the digit's run start in the sorted tile
            // publish this tile's count, then fold in the earlier tiles'
            const uint32_t t = g - ls.x;
            uint32_t* col = a.state + (size_t)(r & 1) * R + tid;   // word of tile q: col[q * 2R]
            st_agent(&col[(size_t)g * 2 * R], (t == 0 ? kFlagPrefix : kFlagAggregate) | total);
            uint32_t excl = 0;
            if (t > 0) {
                uint32_t j = g;   // tiles j-1, j-2, ... (down to ls.x) still to be folded
                uint32_t spins = 0;
                for (;;) {
                    uint32_t lb[LB_WINDOW];
#pragma unroll
                    for (int q = 0; q < LB_WINDOW; ++q)
                        lb[q] = j - ls.x > (uint32_t)q ? ld_agent(&col[(size_t)(j - 1 - q) * 2 * R]) : kFlagPrefix;
                    uint32_t used = 0;
                    bool done = false;
#pragma unroll
                    for (int q = 0; q < LB_WINDOW; ++q) {
                        if (!done && used == (uint32_t)q) {
                            const uint32_t f = lb[q] >> kFlagShift;
                            if (f != 0) {
                                excl += lb[q] & kCountMask;
                                used = q + 1;
                                done = f == (kFlagPrefix >> kFlagShift);
                            }
                        }
                    }
                    if (done) break;
                    j -= used;
                    if (used == 0) {
                        if (++spins > kSpinLimit ||
                            ((spins & 255u) == 0 && (ld_agent(a.err) & kErrLookbackTimeout))) {
                            atomicOr(a.err, (uint32_t)kErrLookbackTimeout);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                st_agent(&col[(size_t)g * 2 * R], kFlagPrefix | ((excl + total) & kCountMask));
            }
            goff[tid] = ls.z + a.seg_base[((size_t)s * NR + r) * R + tid] + excl - run;
#pragma unroll
            for (int q = 0; q < kPHW; ++q) {
                const uint32_t c = sm.slot[q][tid].y;
                sm.slot[q][tid].y = run;
                run += c;
            }
        }
        __syncthreads();
        uint32_t pos[ITEMS];
        {
            const uint32_t bit = 1u << hl;
            const uint32_t lowsel = lane < 32 ? ~0u : 0u;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const bool ok = hofs + i * 32 < len;
                const uint32_t d = digit_of(k[i], shift, 0xFFu);
                if (wave_one_digit(ok, d)) {
                    const uint32_t c = (uint32_t)(__hip_atomic_load((uint64_t*)&sl[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >> 32);
                    pos[i] = c + hl;
                    wave_lds_order();
                    if (hl == 0)
                        __hip_atomic_store((uint64_t*)&sl[d], (uint64_t)(c + 32) << 32, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                    wave_lds_order();
                    continue;
                }
                if (ok) __hip_atomic_fetch_or(&sl[d].x, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                wave_lds_order();
                const uint64_t w = ok ? __hip_atomic_load((uint64_t*)&sl[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 0ull;
                const uint32_t m = (uint32_t)w, c = (uint32_t)(w >> 32);
                pos[i] = __builtin_amdgcn_mbcnt_hi(m, __builtin_amdgcn_mbcnt_lo(m & lowsel, c));
                wave_lds_order();
                if (ok)
                    __hip_atomic_store((uint64_t*)&sl[d], (uint64_t)(c + __builtin_popcount(m)) << 32,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                wave_lds_order();
            }
        }
        __syncthreads();   // every slot read before the keys overwrite them
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (hofs + i * 32 < len) {
                sm.keys[pos[i]] = k[i];
                if (KV) sm.vals[pos[i]] = v[i];
            }
        }
        __syncthreads();
        for (uint32_t p = tid; p < len; p += kPWG) {
            const K key = sm.keys[p];
            const uint32_t o = goff[digit_of(key, shift, 0xFFu)] + p;
            if (o < a.n) {   // always true unless a wait was abandoned
                dst[o] = key;
                if (KV) vdst[o] = sm.vals[p];
            }
        }
    }
    // the look-back words of the next round: this tile's hold round r - 1's
    for (uint32_t i = tid; i < R; i += kPWG) st[((r + 1) & 1) * R + i] = 0;
    __threadfence();
    __syncthreads();
    if (tid == 0) atomicAdd(round_done<NR>(a, s, r), 1u);
}

template <typename K, bool KV>
__global__ __launch_bounds__(kPWG) void k_seg_persist(PArgs a)
{
    constexpr int ITEMS = PCfg<K>::ITEMS;
    constexpr size_t kBig = sizeof(TileSmem<K, KV, kPWG, ITEMS, true>);
    constexpr size_t kSmall = sizeof(TileSmem<K, KV, kPWG, kPSmallItems, true>);
    constexpr size_t kHist = (sizeof(K) * R + 2) * 4;
    constexpr size_t kBS = kBig > kSmall ? kBig : kSmall;
    constexpr size_t kRaw = kBS > kHist ? kBS : kHist;
    __shared__ alignas(16) unsigned char raw[kRaw];
    __shared__ uint32_t goff[R];
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t flag;
    __shared__ uint4 item;
    const uint32_t tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            const uint32_t t = atomicAdd(&a.ctl[0], 1u);
            item = t < a.nitems ? a.items[t] : make_uint4(kItemEnd, 0, 0, 0);
        }
        __syncthreads();
        const uint4 it = item;
        __syncthreads();
        const uint32_t kind = it.x & 0xFFu;
        if (kind == kItemEnd) break;
        if (kind == kItemSmall) {
            if (it.z - it.y <= (uint32_t)(kPWG * kPSmallItems))
                small_item<K, KV, kPSmallItems>(a, raw, it.y, it.z);
            else
                small_item<K, KV, ITEMS>(a, raw, it.y, it.z);
        } else if (kind == kItemHist) {
            hist_item<K, KV>(a, raw, wsum, &flag, it.y, it.z);
        } else {
            round_item<K, KV>(a, raw, wsum, goff, it.x >> 8, it.y, it.z);
        }
    }
}

}  // namespace

uint32_t persist_small_max(int key_bytes)
{
    return key_bytes == 8 ? kPWG * PCfg<uint64_t>::ITEMS : kPWG * PCfg<uint32_t>::ITEMS;
}

// Work list and meta data: lsegs (uint4), tiles (uint2), items (uint4).
size_t persist_meta_bytes(const SegPlan& P, int key_bytes)
{
    const size_t nsmall = P.small[0].size() + P.small[1].size() + P.small[2].size();
    const size_t nitems = P.tiles.size() * (1 + (size_t)key_bytes) + nsmall;
    return align_up(P.lsegs.size() * sizeof(uint4)) + align_up(P.tiles.size() * sizeof(uint2)) +
           nitems * sizeof(uint4);
}

size_t persist_ws_bytes(int key_bytes, bool has_vals, size_t total, const SegPlan& P)
{
    const size_t nt = P.tiles.size(), nls = P.lsegs.size(), nr = key_bytes;
    size_t o = 0;
    o = align_up(o + (nt ? total * key_bytes : 0));                 // tmp keys
    o = align_up(o + (nt && has_vals ? total * 4 : 0));             // tmp vals
    o = align_up(o + nt * nr * R * 4);                              // tile histograms
    o = align_up(o + nt * 2 * 4);                                   // tile identity words
    o = align_up(o + nls * nr * R * 4);                             // segment digit starts
    o = align_up(o + nls * (kMaxRounds + 1) * sizeof(RoundPlan));   // segment plans
    o = align_up(o + nt * 2 * R * 4);                               // look-back words
    o = align_up(o + (1 + 2 * nls + nls * nr) * 4);                 // counters
    o = align_up(o + persist_meta_bytes(P, key_bytes));             // work list
    return o;
}

void persist_pack(const SegPlan& P, int key_bytes, void* host)
{
    uint8_t* h = (uint8_t*)host;
    memcpy(h, P.lsegs.data(), P.lsegs.size() * sizeof(uint4));
    h += align_up(P.lsegs.size() * sizeof(uint4));
    memcpy(h, P.tiles.data(), P.tiles.size() * sizeof(uint2));
    h += align_up(P.tiles.size() * sizeof(uint2));
    uint4* it = (uint4*)h;
    size_t n = 0;
    for (uint32_t s = 0; s < P.lsegs.size(); ++s)
        for (uint32_t g = P.lsegs[s].x; g < P.lsegs[s].y; ++g) it[n++] = make_uint4(kItemHist, s, g, 0);
    for (int c = 2; c >= 0; --c)   // larger classes first
        for (const uint2& sg : P.small[c]) it[n++] = make_uint4(kItemSmall, sg.x, sg.y, 0);
    for (uint32_t r = 0; r < (uint32_t)key_bytes; ++r)
        for (uint32_t s = 0; s < P.lsegs.size(); ++s)
            for (uint32_t g = P.lsegs[s].x; g < P.lsegs[s].y; ++g)
                it[n++] = make_uint4(kItemRound | (r << 8), s, g, 0);
}

namespace {

template <typename K, bool KV>
hipError_t run_persist(const void* keys_in, void* keys_out, const uint32_t* vals_in,
                       uint32_t* vals_out, size_t total, const SegPlan& P, const void* host_meta,
                       void* ws, uint32_t* dev_err, hipStream_t stream, Profiler* prof)
{
    constexpr size_t NR = sizeof(K);
    const size_t nt = P.tiles.size(), nls = P.lsegs.size();
    const size_t nsmall = P.small[0].size() + P.small[1].size() + P.small[2].size();
    const size_t nitems = nt * (1 + NR) + nsmall;
    if (!nitems) return hipSuccess;
    uint8_t* w = (uint8_t*)ws;
    size_t o = 0;
    PArgs a{};
    a.keys_in = keys_in;
    a.keys_out = keys_out;
    a.vals_in = vals_in;
    a.vals_out = vals_out;
    a.keys_tmp = w + o;                 o = align_up(o + (nt ? total * sizeof(K) : 0));
    a.vals_tmp = (uint32_t*)(w + o);    o = align_up(o + (nt && KV ? total * 4 : 0));
    a.tile_hist = (uint32_t*)(w + o);   o = align_up(o + nt * NR * R * 4);
    a.tile_or = (uint32_t*)(w + o);     o = align_up(o + nt * 2 * 4);
    a.seg_base = (uint32_t*)(w + o);    o = align_up(o + nls * NR * R * 4);
    a.seg_plan = (RoundPlan*)(w + o);   o = align_up(o + nls * (kMaxRounds + 1) * sizeof(RoundPlan));
    a.state = (uint32_t*)(w + o);       o = align_up(o + nt * 2 * R * 4);
    a.ctl = (uint32_t*)(w + o);
    const size_t nctl = 1 + 2 * nls + nls * NR;
    o = align_up(o + nctl * 4);
    uint8_t* meta = w + o;
    const size_t mb = persist_meta_bytes(P, (int)NR);
    if (host_meta) {   // null: the work list is already in the workspace
        hipError_t e = hipMemcpyAsync(meta, host_meta, mb, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return e;
    }
    a.lsegs = (const uint4*)meta;
    a.tiles = (const uint2*)(meta + align_up(nls * sizeof(uint4)));
    a.items = (const uint4*)(meta + align_up(nls * sizeof(uint4)) + align_up(nt * sizeof(uint2)));
    a.nitems = (uint32_t)nitems;
    a.nls = (uint32_t)nls;
    a.n = (uint32_t)total;
    const bool keys_alias = keys_in == keys_out, vals_alias = KV && vals_in == vals_out;
    a.alias = (keys_alias || vals_alias ? kAliasAny : 0) | (keys_alias && (!KV || vals_alias) ? kAliasAll : 0);
    a.err = dev_err;
    hipLaunchKernelGGL(k_persist_zero, dim3((uint32_t)std::min<size_t>(64, (nctl + 255) / 256)), dim3(256), 0,
                       stream, a.ctl, (uint32_t)nctl);
    // a resident grid: the launch's workgroups loop over the work list
    static int grid_cache[2][2] = {{0, 0}, {0, 0}};
    int& grid = grid_cache[NR == 8][KV];
    if (!grid) {
        int dev = 0, cus = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_seg_persist<K, KV>, kPWG, 0);
        grid = std::max(1, cus) * std::max(1, per);
    }
    if (prof) profiler_mark(prof, stream, kKindRound, true);
    hipLaunchKernelGGL((k_seg_persist<K, KV>), dim3((uint32_t)std::min<size_t>(nitems, (size_t)grid)),
                       dim3(kPWG), 0, stream, a);
    if (prof) profiler_mark(prof, stream, kKindRound, false);
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
