// Device kernels of the radix-2^8 count-sort rounds, shared by the plain sort
// (lsd_r8.hip) and the batched segmented sort (segmented.hip).  Everything is in
// an anonymous namespace: each translation unit instantiates what it launches.
//
// A round works on tiles of keys.  A tile is described either implicitly
// (plain sort: tile t covers keys [t*TILE, min(n, (t+1)*TILE))) or by an entry
// {first key, end} of a tile list (segmented sort: tiles never cross a segment).
#pragma once

#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "rsort_internal.h"

namespace rsort {
namespace {


constexpr uint32_t R = 256;  // radix
constexpr uint32_t kNoTile = 0xFFFFFFFFu;

// Tile shape of the count and scatter kernels: WG threads, ITEMS keys per
// thread (tile = WG * ITEMS keys).
#ifndef RSORT_R8_WG32
#define RSORT_R8_WG32 512
#endif
#ifndef RSORT_R8_ITEMS32
#define RSORT_R8_ITEMS32 16
#endif
#ifndef RSORT_R8_WG64
#define RSORT_R8_WG64 512
#endif
#ifndef RSORT_R8_ITEMS64
#define RSORT_R8_ITEMS64 8
#endif
// Scatter grid: 1 = persistent (resident workgroups loop over the tiles and
// prefetch the next tile), 0 = one workgroup per tile.
#ifndef RSORT_SCATTER_PERSIST
#define RSORT_SCATTER_PERSIST 0
#endif
// Lanes per ranking group of the scatter: 32 (64-bit slots {lane set, count})
// or 16 (32-bit slots count << 16 | lane set).
#ifndef RSORT_RANK_GROUP
#define RSORT_RANK_GROUP 32
#endif
// Scatter ranking order: 1 = rank, then bases; 0 = count, bases, then rank;
// -1 = rank first with payloads, count first without (the faster of each).
#ifndef RSORT_RANK_FIRST
#define RSORT_RANK_FIRST -1
#endif
// Waves per SIMD the scatter kernel is compiled for (bounds its registers).
#ifndef RSORT_R8_WAVES_PER_EU
#define RSORT_R8_WAVES_PER_EU 8
#endif
#ifndef RSORT_R8_WAVES_PER_EU_KV
#define RSORT_R8_WAVES_PER_EU_KV 4
#endif
#ifndef RSORT_R8_WAVES_PER_EU_KV64
#define RSORT_R8_WAVES_PER_EU_KV64 5
#endif
// LDS the scatter of 32-bit keys with payloads reserves beyond its needs (u32
// words), so that at most two of its 512-thread workgroups (4 waves per SIMD)
// share a CU.  Measured with 2^28 key-value pairs: 4.54 ms per sort at two
// workgroups per CU, 5.57 ms at three (uniform keys).
#ifndef RSORT_SCATTER_KV_LDS_RESERVE
#define RSORT_SCATTER_KV_LDS_RESERVE 6144
#endif
// Tiles per block of the tile scan, and predecessor blocks read per look-back step.
#ifndef RSORT_SCAN_BLOCK
#define RSORT_SCAN_BLOCK 64
#endif
#ifndef LB_WINDOW
#define LB_WINDOW 4
#endif
// Plain sorts of at most this many tiles skip the tile-scan kernel: each
// scatter workgroup sums the tile counts of the round itself.
#ifndef RSORT_INLINE_SCAN_TILES
#define RSORT_INLINE_SCAN_TILES 256
#endif
// Plain 32-bit sorts (counted rounds) of at most this many keys use tiles of
// kSmallWG32 x kSmallItems32 keys.
#ifndef RSORT_SMALL_TILE_MAXN
#define RSORT_SMALL_TILE_MAXN (1u << 20)
#endif
constexpr int kSmallWG32 = 512;
constexpr int kSmallItems32 = 8;
constexpr uint32_t kSmallTile32 = kSmallWG32 * kSmallItems32;

// Count kernel workgroup size (same tile, ITEMS = tile / CWG) and whether full
// tiles are read with 16-byte loads.
#ifndef RSORT_COUNT_WG
#define RSORT_COUNT_WG 512
#endif
#ifndef RSORT_COUNT_VEC
#define RSORT_COUNT_VEC 1
#endif
template <typename K> struct R8Config;
template <> struct R8Config<uint32_t> {
    static constexpr int WG = RSORT_R8_WG32;
    static constexpr int ITEMS = RSORT_R8_ITEMS32;
    static constexpr int CWG = RSORT_COUNT_WG;
    static constexpr int CITEMS = WG * ITEMS / CWG;
};
template <> struct R8Config<uint64_t> {
    static constexpr int WG = RSORT_R8_WG64;
    static constexpr int ITEMS = RSORT_R8_ITEMS64;
    static constexpr int CWG = RSORT_COUNT_WG;
    static constexpr int CITEMS = WG * ITEMS / CWG;
};

constexpr int kHistWG = 256;
constexpr int kHistUnroll = 8;
constexpr uint32_t kScanBlock = RSORT_SCAN_BLOCK;

struct RoundArgs {
    const void* keys_in;
    void* keys_out;
    void* keys_tmp;
    const uint32_t* vals_in;
    uint32_t* vals_out;
    uint32_t* vals_tmp;
    uint32_t n;
    uint32_t shift;
    uint32_t mask;
    uint32_t round;
    uint32_t ntiles;
    uint32_t* bases;         // [round][256] start of each digit's bucket (written by the tile scan)
    const RoundPlan* plan;
    uint32_t* counts;        // [ntiles][256] tile counts, then tile output starts
    uint32_t* blk_state;     // [round][nblocks][256] look-back words of k_tilescan
    uint32_t* tickets;       // [round] block tickets of k_tilescan
    uint32_t* err;
    const uint2* tiles;      // tile list {first key, end} (segmented), or null
    const uint32_t* ntiles_dev;  // tile count known only on the device (grid is an
                                 // upper bound; surplus workgroups exit), or null
    // Segmented sorts: per-segment round plans (a round whose digit is the same
    // for every key of a segment is skipped for that segment).  tile_seg[t] is
    // the large segment of tile t, seg_plan[s * (kMaxRounds + 1) + d] segment
    // s's plan of round d; seg_or (two words per segment) collects, in round
    // 0's count, the OR of every key's difference from its segment's first key
    // (lsegs[s].z); all null for the plain sort.
    const uint32_t* tile_seg = nullptr;
    const RoundPlan* seg_plan = nullptr;
    uint32_t* seg_or = nullptr;
    const uint4* lsegs = nullptr;
    // Plain sorts of few tiles: round 0's count stores tile t's identity pair
    // at mixed[2 t] (no atomics, so the words need no clearing beforehand).
    uint32_t mix_dense = 0;
    // ... and its counts stores the tile counts as 16-bit words (rows of 512
    // bytes), which the scatter's inline tile scan reads.
    uint32_t counts16 = 0;
    // Device-planned segmented sorts given a device round count (the buckets
    // of the sample sort): when it is 0 nothing is sorted, and round 0's
    // count returns at once.
    const uint32_t* dev_rounds = nullptr;
};

// The plan of round a.round for tile t: the segment's plan in a segmented
// sort, the sort's plan otherwise.
__device__ __forceinline__ RoundPlan round_plan_of(const RoundArgs& a, uint32_t t)
{
    if (a.seg_plan) return a.seg_plan[(size_t)a.tile_seg[t] * (kMaxRounds + 1) + a.round];
    return a.plan[a.round];
}

// First key and key count of tile t (at most TILE keys).
__device__ __forceinline__ uint2 tile_range(const RoundArgs& a, uint32_t t, uint32_t tile_keys)
{
    if (a.tiles) {
        const uint2 r = a.tiles[t];
        return make_uint2(r.x, r.y - r.x);
    }
    const uint32_t base = t * tile_keys;
    return make_uint2(base, min(tile_keys, a.n - base));
}

// Output stores of the scatter: streaming (non-temporal) when RSORT_NT_STORES.
#ifndef RSORT_NT_STORES
#define RSORT_NT_STORES 0
#endif
template <typename T>
__device__ __forceinline__ void store_out(T* p, T v)
{
    if (RSORT_NT_STORES) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Key loads of the count kernel and key/payload loads of the scatter kernel:
// streaming (non-temporal) or plain.  Measured: streaming speeds the count
// (every key read once, 115 -> 85 us at 2^27) and slows the scatter with
// payloads, so the defaults differ.
#ifndef RSORT_NT_LOADS_COUNT
#define RSORT_NT_LOADS_COUNT 1
#endif
#ifndef RSORT_NT_LOADS_SCATTER
#define RSORT_NT_LOADS_SCATTER 0
#endif
template <bool NT, typename T>
__device__ __forceinline__ T load_in(const T* p)
{
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

template <typename T>
__device__ __forceinline__ T* pick(int sel, const T* in, T* out, T* tmp)
{
    return sel == 0 ? const_cast<T*>(in) : (sel == 1 ? out : tmp);
}

// Tile handled by this workgroup.  Workgroups are dealt to the 8 XCDs in turn,
// so with ntiles a multiple of 8, tile = (block mod 8) * (ntiles / 8) + block / 8
// gives every XCD a contiguous run of tiles: neighbouring tiles, whose output
// runs share cache lines, then sit behind the same L2.  Other grids keep the
// plain order.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t ntiles)
{
    const uint32_t b = blockIdx.x;
    if ((ntiles & 7) != 0) return b;
    return (b & 7) * (ntiles >> 3) + (b >> 3);
}

// The value held by the lowest active lane of the wave.
__device__ __forceinline__ uint32_t first_lane_value(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint64_t first_lane_value(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Zero the global histogram copies, the block tickets and the tile-scan words.
__global__ void k_init(uint32_t* hist, uint32_t hist_words, uint32_t* tickets,
                       uint32_t nrounds, uint32_t* blk_state, size_t state_words)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t i = g; i < hist_words; i += stride) hist[i] = 0;
    for (size_t i = g; i < nrounds; i += stride) tickets[i] = 0;
    for (size_t i = g; i < state_words; i += stride) blk_state[i] = 0;
}

// The 8-bit digits of [begin_bit, end_bit), least significant first (the
// last one narrower when the range is not a multiple of 8).
struct DigitSet {
    uint32_t shift[kMaxRounds];
    uint32_t mask[kMaxRounds];
};
__device__ __forceinline__ DigitSet digit_set(uint32_t begin_bit, uint32_t end_bit)
{
    DigitSet ds;
#pragma unroll
    for (int d = 0; d < kMaxRounds; ++d) {
        const uint32_t lo = begin_bit + 8u * d;
        const uint32_t w = lo < end_bit ? min(8u, end_bit - lo) : 0u;
        ds.shift[d] = lo < end_bit ? lo : 0u;
        ds.mask[d] = (1u << w) - 1u;
    }
    return ds;
}

// Adds one key per active lane to the LDS histograms h[d * 256 + v] of every
// digit d < nrounds.  When every active lane of the wave holds the same key
// (long runs of equal keys) one lane adds the lane count: the same-address
// LDS atomics of the other lanes would serialise.
template <typename K>
__device__ __forceinline__ void hist_add(uint32_t* h, const DigitSet& ds, uint32_t nrounds, K key)
{
    const uint64_t active = __ballot(1);
    const int leader = __ffsll((unsigned long long)active) - 1;
    const K first = first_lane_value(key);
    if (__all(key == first)) {
        if ((int)(threadIdx.x & 63) == leader) {
            const uint32_t c = (uint32_t)__popcll(active);
#pragma unroll
            for (int d = 0; d < kMaxRounds; ++d)
                if ((uint32_t)d < nrounds) atomicAdd(&h[d * R + digit_of(key, ds.shift[d], ds.mask[d])], c);
        }
    } else {
#pragma unroll
        for (int d = 0; d < kMaxRounds; ++d)
            if ((uint32_t)d < nrounds) atomicAdd(&h[d * R + digit_of(key, ds.shift[d], ds.mask[d])], 1u);
    }
}

// Adds a workgroup's LDS histograms to global copy (block index mod 8), one
// atomic per nonzero bin; the copies spread contention across the XCDs.
__device__ __forceinline__ void hist_flush(const uint32_t* h, uint32_t nrounds, uint32_t* hist)
{
    uint32_t* dst = hist + (blockIdx.x % kHistReplicas) * nrounds * R;
    for (uint32_t b = threadIdx.x; b < nrounds * R; b += blockDim.x) {
        const uint32_t c = h[b];
        if (c) atomicAdd(&dst[b], c);
    }
}

// Counts of every 8-bit digit of [begin_bit, end_bit) in one pass over the
// keys (the histogram entry point; the sort takes them in its first count).
template <typename K>
__global__ __launch_bounds__(kHistWG) void k_hist(const K* __restrict__ keys, uint32_t n,
                                                  uint32_t begin_bit, uint32_t end_bit,
                                                  uint32_t nrounds, uint32_t* hist)
{
    __shared__ uint32_t h[kMaxRounds * R];
    for (uint32_t i = threadIdx.x; i < nrounds * R; i += kHistWG) h[i] = 0;
    __syncthreads();
    const DigitSet ds = digit_set(begin_bit, end_bit);
    const uint32_t stride = gridDim.x * kHistWG;
    uint32_t i = blockIdx.x * kHistWG + threadIdx.x;
    for (; i + (kHistUnroll - 1) * stride < n; i += kHistUnroll * stride) {
        K k[kHistUnroll];
#pragma unroll
        for (int u = 0; u < kHistUnroll; ++u) k[u] = keys[i + u * stride];
#pragma unroll
        for (int u = 0; u < kHistUnroll; ++u) hist_add(h, ds, nrounds, k[u]);
    }
    for (; i < n; i += stride) hist_add(h, ds, nrounds, keys[i]);
    __syncthreads();
    hist_flush(h, nrounds, hist);
}

// Block-wide (256 threads) inclusive sum; wsum is 4 words of LDS.
__device__ __forceinline__ uint32_t block256_inclusive_sum(uint32_t x, uint32_t* wsum)
{
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = wave_inclusive_sum(x);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t pre = 0;
    for (uint32_t w = 0; w < wave; ++w) pre += wsum[w];
    __syncthreads();
    return pre + incl;
}

// Round 0's count ORs every key's difference from the first key into one of
// kMixSlots pairs of words (low and high 32 bits), each pair in a cache line
// of its own, picked by workgroup index, so that the atomics of the first
// workgroups to finish do not all queue on one line.
constexpr uint32_t kMixSlots = 64;
constexpr uint32_t kMixStride = 32;   // words between pairs (128 bytes)
constexpr uint32_t kMixWords = kMixSlots * kMixStride;

// alias: bit 0 set when keys or payloads are sorted in place (keys_in ==
// keys_out or vals_in == vals_out), bit 1 set when every output array is its
// input (nothing to write when every round is the identity).
constexpr int kAliasAny = 1;
constexpr int kAliasAll = 2;

// The round plan from the identity rounds (identity[d] != 0: one digit value
// holds every key, so the stable count sort of round d is the identity).
__device__ void plan_rounds(const int* identity, uint32_t nrounds, int alias, RoundPlan* plan)
{
    const bool in_place = (alias & kAliasAny) != 0;
    int exec[kMaxRounds];
    int m = 0;
    for (uint32_t d = 0; d < nrounds; ++d) {
        exec[d] = !identity[d];
        m += exec[d];
    }
    // The last round must land in the caller's output and no round may read
    // and write the same buffer.  Rounds alternate between output and
    // temporary backwards from the last one, so: when every round is the
    // identity, a copy writes each output that is not its own input (the copy
    // moves every element to its own index, so an aliased array only rewrites
    // itself); otherwise, in place, an even number of rounds must run
    // (re-enable an identity round, or copy the input to the temporary first).
    int precopy = 0;
    if (m == 0) {
        if (!(alias & kAliasAll)) {
            exec[nrounds - 1] = 2;   // a plain copy input -> output
            m = 1;
        }
    } else if (in_place && (m & 1)) {
        int added = 0;
        for (int d = (int)nrounds - 1; d >= 0 && !added; --d)
            if (!exec[d]) { exec[d] = 1; added = 1; }
        if (added) ++m; else precopy = 1;
    }
    int ord = 0;
    int src = precopy ? 2 : 0;
    for (uint32_t d = 0; d < nrounds; ++d) {
        RoundPlan p;
        p.exec = exec[d];
        p.ord = exec[d] ? ord : -1;
        p.src = src;
        p.dst = exec[d] ? (((m - 1 - ord) & 1) ? 2 : 1) : -1;
        if (exec[d]) {
            src = p.dst;
            ++ord;
        }
        plan[d] = p;
    }
    RoundPlan pc;
    pc.exec = precopy;
    pc.ord = m;
    pc.src = 0;
    pc.dst = 2;
    plan[kMaxRounds] = pc;
}

// The round plan of the count-first path.  The OR of the kMixSlots pairs (or,
// with dense_pairs > 0, of the pairs mixed[2 i], i < dense_pairs, one per
// tile) is the OR over all keys of (key XOR first key): a round is the
// identity exactly when its digit's bits are zero there.
__global__ void k_plan(const uint32_t* mixed, uint32_t nrounds, uint32_t begin_bit,
                       uint32_t end_bit, int alias, RoundPlan* plan, uint32_t dense_pairs)
{
    const uint32_t t = threadIdx.x;   // 64 threads
    uint32_t mlo = 0, mhi = 0;
    if (dense_pairs) {
        for (uint32_t i = t; i < dense_pairs; i += 64) {
            mlo |= mixed[2 * i];
            mhi |= mixed[2 * i + 1];
        }
    } else {
        mlo = mixed[t * kMixStride];
        mhi = mixed[t * kMixStride + 1];
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        mlo |= __shfl_xor(mlo, o, 64);
        mhi |= __shfl_xor(mhi, o, 64);
    }
    const uint64_t mx = (uint64_t)mlo | ((uint64_t)mhi << 32);
    if (t == 0) {
        int identity[kMaxRounds];
        for (uint32_t d = 0; d < nrounds; ++d) {
            const uint32_t lo = begin_bit + 8u * d;
            const uint32_t w = min(8u, end_bit - lo);
            identity[d] = ((mx >> lo) & ((1ull << w) - 1ull)) == 0;
        }
        plan_rounds(identity, nrounds, alias, plan);
    }
}

// In-place sorts with an odd number of running rounds: copy input -> temporary.
constexpr int kPrecopyItems = 8;

template <typename K>
__global__ void k_precopy(const RoundPlan* plan, const K* keys, K* keys_tmp,
                          const uint32_t* vals, uint32_t* vals_tmp, uint32_t n)
{
    if (!plan[kMaxRounds].exec) return;
    // kPrecopyItems elements per thread, all loaded before the first store
    const size_t base = (size_t)blockIdx.x * blockDim.x * kPrecopyItems + threadIdx.x;
    K kk[kPrecopyItems];
    uint32_t vv[kPrecopyItems];
#pragma unroll
    for (int j = 0; j < kPrecopyItems; ++j) {
        const size_t i = base + (size_t)j * blockDim.x;
        kk[j] = i < n ? keys[i] : K(0);
        vv[j] = vals && i < n ? vals[i] : 0u;
    }
#pragma unroll
    for (int j = 0; j < kPrecopyItems; ++j) {
        const size_t i = base + (size_t)j * blockDim.x;
        if (i < n) {
            keys_tmp[i] = kk[j];
            if (vals) vals_tmp[i] = vv[j];
        }
    }
}

// ---------------------------------------------------------------------------
// k_count: counts[tile][v] = keys of digit v in the tile.
//
// Every lane counts into its own column of a [256][32] table (lane l of every
// wave uses column l mod 32), so the 32 lanes of a half-wave always hit 32
// different LDS banks; the columns are summed at the end.  Full tiles of the
// plain sort are read with 16-byte loads.
//
// FIRST (first round of the plain sort only): the same read also ORs every
// key's difference from the first key into its pair of mixed words, from which the
// planning kernel finds the identity rounds; this kernel then runs before the
// plan exists.
template <typename K, int WG, int ITEMS, bool FIRST>
__global__ __launch_bounds__(WG) void k_count(RoundArgs a, uint32_t* mixed)
{
    constexpr bool ALL = FIRST;
    constexpr uint32_t TILE = (uint32_t)WG * ITEMS;
    constexpr int VEC = 16 / sizeof(K);   // keys per 16-byte load
    static_assert(ITEMS % VEC == 0, "whole vectors per thread");
    __shared__ uint32_t h[R * 32];
    __shared__ uint32_t mix_s[2];
    // with a device-side tile count the grid (a.ntiles) is an upper bound
    const uint32_t tile = xcd_tile(a.ntiles);
    if (a.ntiles_dev && tile >= *a.ntiles_dev) return;
    RoundPlan pl;
    if (ALL) {
        if (a.dev_rounds && *a.dev_rounds == 0) return;
        pl = RoundPlan{1, 0, 0, 0};
    } else {
        pl = round_plan_of(a, tile);
        if (pl.exec != 1) return;
    }
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < R * 32 / 4; i += WG) ((uint4*)h)[i] = make_uint4(0, 0, 0, 0);
    if (ALL && tid < 2) mix_s[tid] = 0;
    __syncthreads();
    const uint2 tr = tile_range(a, tile, TILE);
    const uint32_t base = tr.x;
    const uint32_t lim = tr.y;
    const K* src = pick<K>(pl.src, (const K*)a.keys_in, (K*)a.keys_out, (K*)a.keys_tmp) + base;
    const uint32_t col = tid & 31;
    // identity test: differences from the first key of the array, or of the
    // tile's segment
    const K ref = !ALL ? K(0) : a.seg_or ? ((const K*)a.keys_in)[a.lsegs[a.tile_seg[tile]].z]
                                         : ((const K*)a.keys_in)[0];
    K acc = 0;
    K k[ITEMS];
    const bool vec = RSORT_COUNT_VEC && !a.tiles && lim == TILE && ((uintptr_t)src & 15) == 0;
    if (vec) {
#pragma unroll
        for (int q = 0; q < ITEMS / VEC; ++q) {
            typedef uint32_t v4 __attribute__((ext_vector_type(4)));
            const v4 x = load_in<RSORT_NT_LOADS_COUNT>(&((const v4*)src)[q * WG + tid]);
            const K* kx = (const K*)&x;
#pragma unroll
            for (int c = 0; c < VEC; ++c) k[q * VEC + c] = kx[c];
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            atomicAdd(&h[digit_of(k[i], a.shift, a.mask) * 32 + col], 1u);
            if (ALL) acc |= k[i] ^ ref;
        }
    } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t o = i * WG + tid;
            k[i] = o < lim ? load_in<RSORT_NT_LOADS_COUNT>(&src[o]) : K(0);
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (i * WG + tid < lim) {
                atomicAdd(&h[digit_of(k[i], a.shift, a.mask) * 32 + col], 1u);
                if (ALL) acc |= k[i] ^ ref;
            }
        }
    }
    if (ALL) {
        const uint64_t a64 = (uint64_t)acc;
        uint32_t lo = (uint32_t)a64, hi = (uint32_t)(a64 >> 32);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            lo |= __shfl_xor(lo, o, 64);
            hi |= __shfl_xor(hi, o, 64);
        }
        if ((tid & 63) == 0) {
            if (lo) atomicOr(&mix_s[0], lo);
            if (hi) atomicOr(&mix_s[1], hi);
        }
    }
    __syncthreads();
    if (ALL && tid < 2) {
        if (!a.seg_or && a.mix_dense) {
            mixed[2 * tile + tid] = mix_s[tid];
        } else {
            // only bits the workgroup's pair lacks cost an atomic
            uint32_t* mw = a.seg_or ? &a.seg_or[2 * a.tile_seg[tile] + tid]
                                    : &mixed[(blockIdx.x % kMixSlots) * kMixStride + tid];
            const uint32_t mine = mix_s[tid];
            if (mine & ~ld_agent(mw)) atomicOr(mw, mine);
        }
    }
    for (uint32_t v = tid; v < R; v += WG) {
        const uint4* r4 = (const uint4*)&h[v * 32];
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint4 x = r4[(q + v) & 7];   // rotate the start so threads spread over banks
            s += x.x + x.y + x.z + x.w;
        }
        if (a.counts16)
            ((uint16_t*)a.counts)[(size_t)tile * R + v] = (uint16_t)s;
        else
            a.counts[(size_t)tile * R + v] = s;
    }
}

// ---------------------------------------------------------------------------
// k_tilescan: replaces counts[t][v] by the sum of counts[t'][v] over t' < t,
// and (last block) writes the round's digit starts bases[v].  Workgroup = block of kScanBlock tiles taken in ticket order; thread
// v sums its digit over the block, publishes the block total, folds the totals
// of earlier blocks by decoupled look-back (a packed flag+count word per block
// and digit), publishes the inclusive prefix and rewrites its column.
__global__ __launch_bounds__(R) void k_tilescan(RoundArgs a)
{
    __shared__ uint32_t blk_s;
    const RoundPlan pl = a.plan[a.round];
    if (pl.exec != 1) return;
    const uint32_t v = threadIdx.x;
    if (v == 0) blk_s = atomicAdd(&a.tickets[a.round], 1u);
    __syncthreads();
    const uint32_t blk = blk_s;
    const uint32_t nblocks = (a.ntiles + kScanBlock - 1) / kScanBlock;
    uint32_t* state = a.blk_state + (size_t)a.round * nblocks * R;
    const uint32_t t0 = blk * kScanBlock;
    const uint32_t t1 = min(a.ntiles, t0 + kScanBlock);
    uint32_t* col = a.counts + v;

    uint32_t c[kScanBlock];
    uint32_t total = 0;
#pragma unroll
    for (uint32_t i = 0; i < kScanBlock; ++i) {
        c[i] = t0 + i < t1 ? col[(size_t)(t0 + i) * R] : 0u;
        total += c[i];
    }
    st_agent(&state[(size_t)blk * R + v], (blk == 0 ? kFlagPrefix : kFlagAggregate) | total);

    uint32_t excl = 0;
    if (blk > 0) {
        uint32_t j = blk;   // entries j-1, j-2, ... are still to be folded
        uint32_t spins = 0;
        for (;;) {
            uint32_t lb[LB_WINDOW];
#pragma unroll
            for (int q = 0; q < LB_WINDOW; ++q)
                lb[q] = (uint32_t)q < j ? ld_agent(&state[(size_t)(j - 1 - q) * R + v]) : kFlagPrefix;
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
                // Give up after kSpinLimit polls, or at once if another
                // workgroup already gave up, so the grid always drains.
                if (++spins > kSpinLimit ||
                    ((spins & 255u) == 0 && (ld_agent(a.err) & kErrLookbackTimeout))) {
                    atomicOr(a.err, (uint32_t)kErrLookbackTimeout);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        st_agent(&state[(size_t)blk * R + v], kFlagPrefix | ((excl + total) & kCountMask));
    }
    if (blk == nblocks - 1) {
        // excl + total is digit v's total over all tiles: the last block turns
        // the totals into the round's digit starts
        __shared__ uint32_t wsum[4];
        const uint32_t all = excl + total;
        a.bases[a.round * R + v] = block256_inclusive_sum(all, wsum) - all;
    }
    uint32_t run = excl;
#pragma unroll
    for (uint32_t i = 0; i < kScanBlock; ++i) {
        if (t0 + i < t1) col[(size_t)(t0 + i) * R] = run;
        run += c[i];
    }
}

// ---------------------------------------------------------------------------
// Output start of each digit's run of tile `tile` without a tile scan: the
// keys of digit v in the tiles before it plus the start of digit v (the keys
// of smaller digits in all tiles), for thread v < 256; every thread calls.
// The tile counts are 16-bit here (counts16: a tile holds fewer than 2^16
// keys), 512-byte rows read as 16-byte vectors of 8 digits, WG / 32 rows per
// step; scratch holds 2 x (WG / 32) x 256 words of LDS, wsum 4 words.  Each
// workgroup reads every row, so this is for sorts of few tiles.
template <int WG>
__device__ __forceinline__ uint32_t inline_tile_offset(const RoundArgs& a, uint32_t tile,
                                                       uint32_t* scratch, uint32_t* wsum)
{
    constexpr uint32_t RG = WG / 32;   // rows per step: 32 threads x 8 digits per row
    constexpr uint32_t ROW = R / 8;    // 16-byte vectors per row
    constexpr int U = 8;               // steps in flight
    static_assert(WG % 64 == 0 && WG >= 256, "whole rows and a thread per digit");
    const uint32_t tid = threadIdx.x, c8 = tid & 31, rg = tid >> 5;
    const uint32_t lane = tid & 63, wave = tid >> 6;
    const uint4* rows = (const uint4*)a.counts;
    uint32_t bs[8] = {0, 0, 0, 0, 0, 0, 0, 0}, ts[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t t0 = rg; t0 < a.ntiles; t0 += RG * U) {
        uint4 x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t t = t0 + u * RG;
            x[u] = t < a.ntiles ? rows[(size_t)t * ROW + c8] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t f = t0 + u * RG < tile ? ~0u : 0u;
            const uint32_t w[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t lo = w[q] & 0xFFFFu, hi = w[q] >> 16;
                ts[2 * q] += lo;
                ts[2 * q + 1] += hi;
                bs[2 * q] += lo & f;
                bs[2 * q + 1] += hi & f;
            }
        }
    }
    uint4* s4 = (uint4*)scratch;
    s4[(rg * R + 8 * c8) / 4] = make_uint4(bs[0], bs[1], bs[2], bs[3]);
    s4[(rg * R + 8 * c8) / 4 + 1] = make_uint4(bs[4], bs[5], bs[6], bs[7]);
    s4[((RG + rg) * R + 8 * c8) / 4] = make_uint4(ts[0], ts[1], ts[2], ts[3]);
    s4[((RG + rg) * R + 8 * c8) / 4 + 1] = make_uint4(ts[4], ts[5], ts[6], ts[7]);
    __syncthreads();
    uint32_t before = 0, total = 0, incl = 0;
    if (tid < R) {
#pragma unroll
        for (uint32_t g = 0; g < RG; ++g) {
            before += scratch[g * R + tid];
            total += scratch[(RG + g) * R + tid];
        }
        incl = wave_inclusive_sum(total);
        if (lane == 63) wsum[wave] = incl;
    }
    __syncthreads();
    if (tid < R)
        for (uint32_t w = 0; w < wave; ++w) incl += wsum[w];
    return incl - total + before;
}

// ---------------------------------------------------------------------------
// k_scatter: one stable count-sort round of one tile.
//
// Layout: the tile is split among half-waves (32 lanes); half-wave h owns the
// contiguous keys [h*ITEMS*32, (h+1)*ITEMS*32) of the tile, row i lane l at
// h*ITEMS*32 + i*32 + (l & 31), so "earlier in the input" is lexicographic
// (h, i, l) -- the order the ranking preserves.
// Each half-wave has one 64-bit slot per digit value: the set of its lanes
// holding that digit in the current row and the number of its keys of that
// digit in earlier rows (low and high word below digit 128, swapped above, so
// that each word kind spreads over all LDS banks).
//   rank   row by row, lanes OR their bit into the slot of their digit, read
//          the slot back -- the lanes below with the same digit plus the count
//          give the key's rank among the half-wave's keys of that digit -- and
//          write the slot back as {no lanes, count + lanes in the set};
//   bases  digit thread v turns the counts of all half-waves into slot bases
//          inside the tile (prefix over half-waves plus the tile's prefix over
//          digits), written over the counts (keys only: the counts are first
//          added up in a separate array of 4-byte words, which spreads those
//          additions over all 64 LDS banks);
//   stage  each key goes to LDS at base + rank, the tile now in digit order;
//   scatter consecutive threads write consecutive slots of a digit's run; the
//          payloads follow in a second staging pass through the same LDS.
//
// INL (plain sorts of few tiles): there is no tile scan; counts[t][v] are the
// tile counts and the workgroup sums them itself (inline_tile_offset).  A
// separate instantiation, so that the registers of the usual one stay as
// they are; with at most a few hundred tiles it needs no more than one
// workgroup per CU, so it may use more registers.
template <typename K, bool KV, int WG, int ITEMS, bool INL = false>
__global__ __launch_bounds__(WG, INL ? WG / 256 : !KV ? RSORT_R8_WAVES_PER_EU : sizeof(K) == 4 ? RSORT_R8_WAVES_PER_EU_KV : RSORT_R8_WAVES_PER_EU_KV64) void k_scatter(RoundArgs a)
{
    constexpr int G = RSORT_RANK_GROUP;         // lanes per ranking group
    constexpr int NG = WG / G;                  // ranking groups
    constexpr uint32_t TILE = (uint32_t)WG * ITEMS;
    constexpr bool rank_first = RSORT_RANK_FIRST < 0 ? KV : RSORT_RANK_FIRST != 0;
    // LDS banks: a slot is 8 bytes, so one word of every slot would sit in
    // half of the 64 banks.  Slots of digits below 128 hold {lane set,
    // count}, those of digits from 128 on {count, lane set}, so the lane-set
    // ORs of a half-wave spread over all banks; counting first adds into a
    // separate array of 4-byte counts (all banks as well).
    constexpr bool split_counts = G == 32 && !rank_first;
    static_assert(G == 16 || G == 32, "ranking groups of 16 or 32 lanes");
    static_assert(G == 32 || (uint64_t)TILE < 65536, "16-bit slot counts");
    static_assert(INL || TILE * sizeof(K) >= NG * R * (G == 32 ? 8 : 4), "staging must cover the slots");
    static_assert(!INL || 2 * NG * R >= 2 * (WG / 32) * R, "the inline tile scan's scratch fits the slot words");
    static_assert(!INL || TILE < 65536, "16-bit tile counts");
    struct Smem {
        union {
            uint2 slot[NG][R];           // 32-lane groups: {lane set, count}, then {-, slot base}
                                         // (the two words swapped for digits >= 128)
            uint32_t words[2 * NG * R];  // count first: counts at words[NG R + g R + d]
            uint32_t slot16[NG][R];      // 16-lane groups: count << 16 | lane set
            K keys[TILE];                // staging: the tile in digit order
            uint32_t vals[TILE];         // staging of the payloads (second pass)
        } u;
        uint32_t goff[R];                // output index of tile slot 0 of each digit
        uint32_t wsum[4];
        uint32_t reserve[KV && sizeof(K) == 4 && WG == 512 ? RSORT_SCATTER_KV_LDS_RESERVE : 1];   // occupancy cap, unused
    };
    __shared__ Smem sm;

    // Tile sequence of this workgroup: with a grid smaller than the tile count
    // each workgroup loops.  When both counts are multiples of 8 every XCD owns
    // a contiguous eighth of the tiles (blocks are dealt to XCDs in turn), so
    // neighbouring tiles write their shared cache lines through the same L2.
    const uint32_t b = blockIdx.x, nb = gridDim.x;
    const uint32_t ntiles = a.ntiles_dev ? *a.ntiles_dev : a.ntiles;
    const bool xcd = (a.ntiles & 7) == 0 && (nb & 7) == 0;
    const uint32_t per = a.ntiles >> 3, g8 = nb >> 3, x = b & 7;
    uint32_t tile = xcd ? x * per + (b >> 3) : b;
    // a per-segment plan needs the tile; the plain sort's plan is read even by
    // surplus workgroups (its copy round covers the whole array)
    if (a.seg_plan && tile >= ntiles) return;
    const RoundPlan pl = a.seg_plan ? round_plan_of(a, tile) : a.plan[a.round];
    if (!pl.exec) return;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    const uint32_t wave = tid >> 6;
    const uint32_t grp = tid / G;
    const uint32_t gl = tid % G;
    const uint32_t hofs = grp * ITEMS * G + gl;   // position of row 0 of this lane
    const K* src = pick<K>(pl.src, (const K*)a.keys_in, (K*)a.keys_out, (K*)a.keys_tmp);
    const uint32_t* vsrc = KV ? pick<uint32_t>(pl.src, a.vals_in, a.vals_out, a.vals_tmp) : nullptr;
    K* dst = pick<K>(pl.dst, (const K*)a.keys_in, (K*)a.keys_out, (K*)a.keys_tmp);
    uint32_t* vdst = KV ? pick<uint32_t>(pl.dst, a.vals_in, a.vals_out, a.vals_tmp) : nullptr;
    if (pl.exec == 2 && a.tiles) {   // a segment's rounds are all identities: copy the tile
        const uint2 tr = tile_range(a, tile, TILE);
        K kk[ITEMS];
        uint32_t vv[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t i = j * WG + tid;
            kk[j] = i < tr.y ? src[tr.x + i] : K(0);
            if (KV) vv[j] = i < tr.y ? vsrc[tr.x + i] : 0u;
        }
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const uint32_t i = j * WG + tid;
            if (i < tr.y) {
                dst[tr.x + i] = kk[j];
                if (KV) vdst[tr.x + i] = vv[j];
            }
        }
        return;
    }
    if (pl.exec == 2) {   // identity round standing for a copy: tile by tile, loads first
        for (uint32_t t = blockIdx.x; (size_t)t * TILE < a.n; t += gridDim.x) {
            K kk[ITEMS];
            uint32_t vv[ITEMS];
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const size_t i = (size_t)t * TILE + j * WG + tid;
                kk[j] = i < a.n ? src[i] : K(0);
                if (KV) vv[j] = i < a.n ? vsrc[i] : 0u;
            }
#pragma unroll
            for (int j = 0; j < ITEMS; ++j) {
                const size_t i = (size_t)t * TILE + j * WG + tid;
                if (i < a.n) {
                    dst[i] = kk[j];
                    if (KV) vdst[i] = vv[j];
                }
            }
        }
        return;
    }

    // full: std::true_type when the tile holds TILE keys (every tile but a
    // last or segment-end one), so that the bounds tests fold away
    auto load = [&](auto full, uint32_t t, K (&kk)[ITEMS], uint32_t (&vv)[ITEMS]) {
        const uint2 tr = tile_range(a, t, TILE);
        const uint32_t base = tr.x;
        const uint32_t lim = decltype(full)::value ? TILE : tr.y;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t o = hofs + i * G;
            kk[i] = o < lim ? load_in<RSORT_NT_LOADS_SCATTER>(&src[base + o]) : K(0);
            if (KV) vv[i] = o < lim ? load_in<RSORT_NT_LOADS_SCATTER>(&vsrc[base + o]) : 0u;
        }
    };

    // One tile whose keys are in k/v; the keys of tile tn (if any) are loaded
    // into kn/vn once k has been counted, so that those loads are in flight
    // while this tile is ranked, staged and written.
    auto process = [&](auto full, uint32_t tile, K (&k)[ITEMS], uint32_t (&v)[ITEMS], uint32_t tn,
                       K (&kn)[ITEMS], uint32_t (&vn)[ITEMS]) {
        // keys in this tile
        const uint32_t lim = decltype(full)::value ? TILE : tile_range(a, tile, TILE).y;
        constexpr uint32_t slot_u4 = NG * R * (G == 32 ? 8 : 4) / 16;
        uint32_t toff = 0;
        if constexpr (INL) {
            // the LDS scratch is read before the barrier that ends the call
            // and zeroed below only after it
            toff = inline_tile_offset<WG>(a, tile, sm.u.words, sm.wsum);
        } else if (tid < R) {
            toff = a.counts[(size_t)tile * R + tid];
            if (a.bases) toff += a.bases[a.round * R + tid];
        }
        for (uint32_t i = tid; i < slot_u4; i += WG)
            ((uint4*)&sm.u)[i] = make_uint4(0, 0, 0, 0);
        __syncthreads();

        // Rank row by row; a slot's count is advanced by the lanes of the row
        // that hold its digit.  Gives each key's rank plus the count before
        // the key's row.  (Measured: writing the slot back after its read is
        // faster than an atomic add that needs no read.)
        uint32_t pos[ITEMS];
        auto rank = [&]() {
            const uint32_t bit = 1u << gl;
            if constexpr (G == 32) {
                uint2* sl = sm.u.slot[grp];
                const uint32_t lowsel = lane < 32 ? ~0u : 0u;
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    const bool ok = hofs + i * G < lim;
                    const uint32_t d = digit_of(k[i], a.shift, a.mask);
                    const uint32_t cs = (d & 128u) ? 0u : 32u;   // bit offset of the count
                    if (wave_one_digit(ok, d)) {
                        // every lane of the wave holds this digit: no lane
                        // set to build, one lane per group moves the count
                        const uint32_t c = (uint32_t)(__hip_atomic_load((uint64_t*)&sl[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >> cs);
                        pos[i] = c + gl;
                        wave_lds_order();
                        if (gl == 0)
                            __hip_atomic_store((uint64_t*)&sl[d], (uint64_t)(c + 32) << cs,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        wave_lds_order();
                        continue;
                    }
                    if (ok) __hip_atomic_fetch_or(cs ? &sl[d].x : &sl[d].y, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    wave_lds_order();
                    const uint64_t s = ok ? __hip_atomic_load((uint64_t*)&sl[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 0ull;
                    const uint32_t m = (uint32_t)(s >> (32u - cs)), c = (uint32_t)(s >> cs);
                    pos[i] = __builtin_amdgcn_mbcnt_hi(m, __builtin_amdgcn_mbcnt_lo(m & lowsel, c));
                    wave_lds_order();
                    if (ok)
                        __hip_atomic_store((uint64_t*)&sl[d], (uint64_t)(c + __builtin_popcount(m)) << cs,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    wave_lds_order();
                }
            } else {
                uint32_t* sl = sm.u.slot16[grp];
                const uint32_t below = bit - 1u;
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    const bool ok = hofs + i * G < lim;
                    const uint32_t d = digit_of(k[i], a.shift, a.mask);
                    if (ok) __hip_atomic_fetch_or(&sl[d], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    wave_lds_order();
                    const uint32_t s = ok ? __hip_atomic_load(&sl[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 0u;
                    const uint32_t c = s >> 16;
                    pos[i] = c + __builtin_popcount(s & below);
                    wave_lds_order();
                    if (ok)
                        __hip_atomic_store(&sl[d], (c + __builtin_popcount(s & 0xFFFFu)) << 16,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    wave_lds_order();
                }
            }
        };
        auto slot_count = [&](int g, uint32_t v) -> uint32_t {
            if constexpr (G == 32) return (v & 128u) ? sm.u.slot[g][v].x : sm.u.slot[g][v].y;
            else return sm.u.slot16[g][v] >> 16;
        };
        auto set_slot_count = [&](int g, uint32_t v, uint32_t c) {
            if constexpr (G == 32) {
                if (v & 128u) sm.u.slot[g][v].x = c;
                else sm.u.slot[g][v].y = c;
            }
            else sm.u.slot16[g][v] = c << 16;
        };

        if (rank_first) {
            // rank with counts starting at zero; the counts end up in the slots
            rank();
        } else {
            // count first: the slots' counts get the per-group digit counts
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const bool ok = hofs + i * G < lim;
                const uint32_t d = digit_of(k[i], a.shift, a.mask);
                if (G == 32 && wave_one_digit(ok, d)) {   // one add per group
                    if (gl == 0) atomicAdd(&sm.u.words[NG * R + grp * R + d], 32u);
                    continue;
                }
                if (ok) {
                    if constexpr (G == 32) atomicAdd(&sm.u.words[NG * R + grp * R + d], 1u);
                    else atomicAdd(&sm.u.slot16[grp][d], 1u << 16);
                }
            }
        }
        if (RSORT_SCATTER_PERSIST && tn != kNoTile) load(std::false_type{}, tn, kn, vn);
        __syncthreads();

        // bases
        auto count_of = [&](int g, uint32_t v) -> uint32_t {
            if constexpr (split_counts) return sm.u.words[NG * R + g * R + v];
            else return slot_count(g, v);
        };
        uint32_t run = 0;
        if (tid < R) {
            uint32_t total = 0;
#pragma unroll
            for (int g = 0; g < NG; ++g) total += count_of(g, tid);
            const uint32_t incl = wave_inclusive_sum(total);
            if (lane == 63) sm.wsum[wave] = incl;
            run = incl - total;
        }
        __syncthreads();
        if constexpr (split_counts) {
            // slots of groups < NG/2 lie below the counts; the others overlap
            // them, so their counts are read before any of them is written
            uint32_t hi[NG / 2];
            if (tid < R) {
                for (uint32_t w = 0; w < wave; ++w) run += sm.wsum[w];
                sm.goff[tid] = toff - run;
#pragma unroll
                for (int g = 0; g < NG / 2; ++g) {
                    const uint32_t c = count_of(g, tid);
                    sm.u.slot[g][tid] = (tid & 128u) ? make_uint2(run, 0u) : make_uint2(0u, run);
                    run += c;
                }
#pragma unroll
                for (int g = NG / 2; g < NG; ++g) hi[g - NG / 2] = count_of(g, tid);
            }
            __syncthreads();
            if (tid < R) {
#pragma unroll
                for (int g = NG / 2; g < NG; ++g) {
                    sm.u.slot[g][tid] = (tid & 128u) ? make_uint2(run, 0u) : make_uint2(0u, run);
                    run += hi[g - NG / 2];
                }
            }
        } else if (tid < R) {
            for (uint32_t w = 0; w < wave; ++w) run += sm.wsum[w];
            sm.goff[tid] = toff - run;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const uint32_t c = slot_count(g, tid);
                set_slot_count(g, tid, run);
                run += c;
            }
        }
        __syncthreads();
        if (rank_first) {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                // Recompute the digit here rather than keep 16 slot addresses
                // alive across the bases phase (registers limit occupancy).
                __asm__ volatile("" : "+v"(k[i]));
                pos[i] += slot_count(grp, digit_of(k[i], a.shift, a.mask));
            }
        } else {
            rank();   // the counts now start at the slot bases
        }
        __syncthreads();

        // scatter
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            if (hofs + i * G < lim) sm.u.keys[pos[i]] = k[i];
        __syncthreads();
        uint32_t outi[KV ? ITEMS : 1];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = i * WG + tid;
            uint32_t o = a.n;
            if (p < lim) {
                const K key = sm.u.keys[p];
                o = sm.goff[digit_of(key, a.shift, a.mask)] + p;
                if (o < a.n) store_out(&dst[o], key);   // always true unless a tile-scan wait was abandoned
            }
            if (KV) outi[i] = o;
        }
        if (KV) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; ++i)
                if (hofs + i * G < lim) sm.u.vals[pos[i]] = v[i];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t p = i * WG + tid;
                if (p < lim && outi[i] < a.n) store_out(&vdst[outi[i]], sm.u.vals[p]);
            }
        }
        __syncthreads();   // staging and goff are free for the next tile
    };

    auto next_of = [&](uint32_t t) -> uint32_t {
        if (xcd) {
            const uint32_t l = t - x * per + g8;
            return l < per ? x * per + l : kNoTile;
        }
        return t + nb < ntiles ? t + nb : kNoTile;
    };
    if (tile >= ntiles) return;

    K ka[ITEMS];
    uint32_t va[ITEMS];
    if constexpr (!RSORT_SCATTER_PERSIST) {
        if (tile_range(a, tile, TILE).y == TILE) {
            load(std::true_type{}, tile, ka, va);
            process(std::true_type{}, tile, ka, va, kNoTile, ka, va);
        } else {
            load(std::false_type{}, tile, ka, va);
            process(std::false_type{}, tile, ka, va, kNoTile, ka, va);
        }
        return;
    }
    load(std::false_type{}, tile, ka, va);
    K kb[ITEMS];
    uint32_t vb[ITEMS];
    for (;;) {
        uint32_t tn = next_of(tile);
        process(std::false_type{}, tile, ka, va, tn, kb, vb);
        tile = tn;
        if (tile == kNoTile) break;
        tn = next_of(tile);
        process(std::false_type{}, tile, kb, vb, tn, ka, va);
        tile = tn;
        if (tile == kNoTile) break;
    }
}

}  // namespace
}  // namespace rsort
