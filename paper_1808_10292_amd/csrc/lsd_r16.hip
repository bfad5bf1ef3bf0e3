// PR2: LSD radix sort with radix r = 2^16 (arXiv 1808.10292 Section 3.2, PR2,
// equation Tp2): one stable count-sort round per 16-bit digit, two rounds for
// 32-bit keys.  A round has the paper's three parts, laid out for gfx950:
//
//   group    (rounds wider than 8 bits) the keys are first reordered, stably,
//            by the high byte of the digit: one 8-bit count-sort round of the
//            radix-256 path into a second buffer.  Counting and placement run
//            on that order (see "Grouping" below);
//   count    the keys are cut into W contiguous chunks of 8 tiles (W <= 4096),
//            one per workgroup; k_rows16 counts chunk w's digits into its own
//            row (the paper's per-processor count array).  Because the keys
//            are grouped, chunk w holds only the digits of the groups between
//            its first and last key, its window [256 g0, 256 g1 + 256); only
//            the window is counted and stored, at rows[256 w + v].  Windows of
//            consecutive chunks overlap at most in one group, so these ranges
//            never collide and all rows fit in 256 (W + 255) words;
//   prefix   rows[256 w + v] becomes the output index of chunk w's first key
//            of digit v: the sum of the totals of all digits u < v plus the
//            counts of v in chunks before w.  The chunks whose window holds v
//            are consecutive; each digit finds them by binary search of the
//            windows (column sums scanned in blocks of 256 digits, a scan of
//            the block totals, column prefixes);
//   place    k_place16: workgroup w walks its chunk in order, tile by tile.
//            Each tile is stable-sorted by the 16-bit digit in LDS (two 8-bit
//            counting sub-rounds; the second is skipped when the tile holds one
//            group), every key goes to its row entry + its rank in its digit's
//            run in the tile, and the run's last key advances the entry.  The
//            workgroup owns its row, so no atomics are needed; tiles are
//            visited in order, so the round is stable.
//
// Grouping.  Keys of equal digit keep their input order through the grouping,
// so the placement's output is that of the paper's round, but a chunk now
// holds only a few consecutive digit groups: the rows shrink to the windows, a
// tile's row entries share a few cache lines, a chunk writes each of its
// digits' output ranges front to back, and all workgroups write within a
// narrow window of the output at any time, so cache lines of the output fill
// before they are evicted.  Without it (each tile meeting a different digit at
// almost every key, 256 dense rows of 65536 counts) the placement measured 16x
// write and 10x read amplification at the L2 and took 4.8 ms per round at 2^27
// keys.  The grouping costs one more count-sort pass of coalesced traffic.
#include <algorithm>

#include "rsort_internal.h"
#include "tile_sort.h"

namespace rsort {
namespace {

constexpr uint32_t kR16 = 65536;
constexpr int kRowsWG = 1024;
constexpr uint32_t kWin = 16384;        // LDS counters of k_rows16 per pass over a chunk
constexpr uint32_t kMaxChunks = 4096;
constexpr uint32_t kChunkTiles = 8;

template <typename K> struct R16Config;
template <> struct R16Config<uint32_t> {
    static constexpr int WG = 256;
    static constexpr int ITEMS = 16;
};
template <> struct R16Config<uint64_t> {
    static constexpr int WG = 256;
    static constexpr int ITEMS = 8;
};

template <typename K>
constexpr uint32_t r16_tile() { return (uint32_t)R16Config<K>::WG * R16Config<K>::ITEMS; }

// Workgroup w counts chunk w's digits over its window (the whole digit range
// when the keys are not grouped, which happens only for rounds of at most 8
// bits), kWin digits per pass over the chunk, writes the counts of the window
// to rows[256 w + v] and the window to win[w].
template <typename K>
__global__ __launch_bounds__(kRowsWG) void k_rows16(const K* __restrict__ keys, uint32_t n,
                                                    uint32_t chunk, uint32_t shift, uint32_t mask,
                                                    uint32_t* rows, uint2* win, bool grouped)
{
    __shared__ uint32_t cnt[kWin];
    const uint32_t tid = threadIdx.x;
    const uint32_t w = blockIdx.x;
    const uint32_t lo = w * chunk, hi = min(n, lo + chunk);
    uint32_t gl = 0, gh = mask + 1;
    if (grouped) {
        gl = digit_of(keys[lo], shift, mask) & ~255u;
        gh = (digit_of(keys[hi - 1], shift, mask) | 255u) + 1u;
    }
    if (tid == 0) win[w] = make_uint2(gl, gh);
    uint32_t* row = rows + (size_t)256 * w;
    for (uint32_t p0 = gl; p0 < gh; p0 += kWin) {
        const uint32_t pw = min(kWin, gh - p0);
        for (uint32_t i = tid; i < pw; i += kRowsWG) cnt[i] = 0;
        __syncthreads();
        uint32_t i = lo + tid;
        for (; i + 3 * kRowsWG < hi; i += 4 * kRowsWG) {
            const K a = keys[i], b = keys[i + kRowsWG], c = keys[i + 2 * kRowsWG],
                    d = keys[i + 3 * kRowsWG];
            const uint32_t da = digit_of(a, shift, mask) - p0, db = digit_of(b, shift, mask) - p0;
            const uint32_t dc = digit_of(c, shift, mask) - p0, dd = digit_of(d, shift, mask) - p0;
            if (da < pw) atomicAdd(&cnt[da], 1u);
            if (db < pw) atomicAdd(&cnt[db], 1u);
            if (dc < pw) atomicAdd(&cnt[dc], 1u);
            if (dd < pw) atomicAdd(&cnt[dd], 1u);
        }
        for (; i < hi; i += kRowsWG) {
            const uint32_t d = digit_of(keys[i], shift, mask) - p0;
            if (d < pw) atomicAdd(&cnt[d], 1u);
        }
        __syncthreads();
        for (uint32_t b = tid; b < pw; b += kRowsWG) row[p0 + b] = cnt[b];
        __syncthreads();
    }
}

// The chunks whose window holds digit v: [*wa, *wb] (windows are ordered:
// both ends are nondecreasing in w).
__device__ __forceinline__ void chunks_of(const uint2* win, uint32_t nchunks, uint32_t v,
                                          uint32_t* wa, uint32_t* wb)
{
    uint32_t a = 0, b = nchunks;   // first w with win[w].y > v
    while (a < b) {
        const uint32_t m = (a + b) >> 1;
        if (win[m].y > v) b = m; else a = m + 1;
    }
    uint32_t c = a, d = nchunks;   // first w with win[w].x > v
    while (c < d) {
        const uint32_t m = (c + d) >> 1;
        if (win[m].x > v) d = m; else c = m + 1;
    }
    *wa = a;
    *wb = c;   // exclusive
}

// Column sums and their exclusive scan, in two levels: workgroup b sums the
// columns v in [256 b, 256 b + 256) over the chunks, scans them inside the
// block (excl[v]) and writes the block total; k_blockscan16 scans the block
// totals; k_colprefix16 adds them up.
__global__ __launch_bounds__(256) void k_colsum16(const uint32_t* rows, const uint2* win,
                                                  uint32_t nchunks, uint32_t nbins, uint32_t* excl,
                                                  uint32_t* block_total)
{
    __shared__ uint32_t wsum[4];
    const uint32_t v = blockIdx.x * 256 + threadIdx.x;
    uint32_t s = 0;
    if (v < nbins) {
        uint32_t wa, wb;
        chunks_of(win, nchunks, v, &wa, &wb);
        for (uint32_t w = wa; w < wb; ++w) s += rows[(size_t)256 * w + v];
    }
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t incl = wave_inclusive_sum(s);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t q = 0; q < wave; ++q) before += wsum[q];
    if (v < nbins) excl[v] = before + incl - s;
    if (threadIdx.x == 255) block_total[blockIdx.x] = before + incl;
}

// Exclusive scan of the (at most 256) block totals, in place.
__global__ __launch_bounds__(256) void k_blockscan16(uint32_t* block_total, uint32_t nblocks)
{
    __shared__ uint32_t wsum[4];
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const uint32_t x = t < nblocks ? block_total[t] : 0u;
    const uint32_t incl = wave_inclusive_sum(x);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t q = 0; q < wave; ++q) before += wsum[q];
    if (t < nblocks) block_total[t] = before + incl - x;
}

// rows[256 w + v] = (digit v's start) + sum over chunks w' < w of their counts of v.
__global__ __launch_bounds__(256) void k_colprefix16(uint32_t* rows, const uint2* win,
                                                     uint32_t nchunks, uint32_t nbins,
                                                     const uint32_t* excl, const uint32_t* block_pre)
{
    const uint32_t v = blockIdx.x * 256 + threadIdx.x;
    if (v >= nbins) return;
    uint32_t wa, wb;
    chunks_of(win, nchunks, v, &wa, &wb);
    uint32_t run = block_pre[blockIdx.x] + excl[v];
    for (uint32_t w = wa; w < wb; ++w) {
        uint32_t* p = rows + (size_t)256 * w + v;
        const uint32_t c = *p;
        *p = run;
        run += c;
    }
}

// Inclusive max over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_inclusive_max(uint32_t x)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x = max(x, y);
    }
    return x;
}

// A tile whose keys share the digit's high byte (the usual case after the
// grouping): one stable counting round on the low byte l, as in the radix-256
// rounds, with the run of l going to row[g + l] (g: the tile's group times
// 256).  The sorted tile is staged in LDS and leaves in sorted order,
// consecutive threads taking consecutive positions.  Every thread must call.
template <typename K, bool KV, int WG, int ITEMS>
__device__ __forceinline__ void place_one_group(TileSmem<K, KV, WG, ITEMS, true>& sm, uint32_t* gofs,
                                                K (&k)[ITEMS], uint32_t (&v)[ITEMS], uint32_t len,
                                                uint32_t shift, uint32_t width, uint32_t mask,
                                                uint32_t* row, uint32_t n, K first,
                                                K* __restrict__ keys_out, uint32_t* __restrict__ vals_out)
{
    static_assert(WG == 256, "one thread per low-byte value");
    constexpr int HW = WG / 32;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t hw = tid >> 5, hl = tid & 31;
    const uint32_t hofs = hw * ITEMS * 32 + hl;
    const uint32_t lmask = width < 8 ? mask : 255u;
    const uint32_t g = width > 8 ? (digit_of(first, shift, mask) & ~255u) : 0u;

    for (uint32_t i = tid; i < HW * 256 / 2; i += WG)
        ((uint4*)&sm.slot[0][0])[i] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    uint2* sl = sm.slot[hw];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const bool ok = hofs + i * 32 < len;
        const uint32_t d = digit_of(k[i], shift, lmask);
        if (wave_one_digit(ok, d)) {
            if (hl == 0) atomicAdd(&sl[d].y, 32u);
            continue;
        }
        if (ok) atomicAdd(&sl[d].y, 1u);
    }
    __syncthreads();
    {
        // thread tid = low byte l: its run's start in the tile and in the output
        uint32_t total = 0;
#pragma unroll
        for (int h = 0; h < HW; ++h) total += sm.slot[h][tid].y;
        const uint32_t incl = wave_inclusive_sum(total);
        if (lane == 63) sm.wsum[wave] = incl;
        __syncthreads();
        uint32_t run = incl - total;
        for (uint32_t q = 0; q < wave; ++q) run += sm.wsum[q];
        if (total) {
            const uint32_t r = __hip_atomic_load(&row[g + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            gofs[tid] = r - run;
            __hip_atomic_store(&row[g + tid], r + total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
#pragma unroll
        for (int h = 0; h < HW; ++h) {
            const uint32_t c = sm.slot[h][tid].y;
            sm.slot[h][tid].y = run;
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
            const uint32_t d = digit_of(k[i], shift, lmask);
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
            const uint64_t s = ok ? __hip_atomic_load((uint64_t*)&sl[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 0ull;
            const uint32_t m = (uint32_t)s, c = (uint32_t)(s >> 32);
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
    for (uint32_t p = tid; p < len; p += WG) {
        const K key = sm.keys[p];
        const uint32_t d = gofs[digit_of(key, shift, lmask)] + p;
        if (d < n) {   // always true when the rows are consistent
            keys_out[d] = key;
            if (KV) vals_out[d] = sm.vals[p];
        }
    }
    __syncthreads();   // before the next tile reuses the slots
}

// The placement of one round over chunk w (workgroup w), tile by tile in
// order; row[v] = rows[256 w + v] is the output index of the chunk's next key
// of digit v.  After the tile is sorted, each thread finds the digit runs in
// ITEMS consecutive sorted positions and records every position's output
// index in LDS; the keys then leave in sorted order, consecutive threads
// taking consecutive positions, so a wave's stores cover a few digit runs
// (a few cache lines) instead of one run per lane.
template <typename K, bool KV>
__global__ __launch_bounds__(R16Config<K>::WG) void k_place16(
    const K* __restrict__ keys_in, K* __restrict__ keys_out, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ vals_out, uint32_t n, uint32_t chunk, uint32_t shift, uint32_t width,
    uint32_t* rows)
{
    constexpr int WG = R16Config<K>::WG;
    constexpr int ITEMS = R16Config<K>::ITEMS;
    constexpr uint32_t TILE = (uint32_t)WG * ITEMS;
    static_assert(ITEMS * sizeof(K) % 16 == 0, "vector LDS reads of a thread's run");
    __shared__ alignas(16) TileSmem<K, KV, WG, ITEMS, true> sm;
    __shared__ uint32_t dest[TILE];
    __shared__ uint32_t gofs[256];
    __shared__ uint32_t wmax[WG / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t hofs = (tid >> 5) * ITEMS * 32 + (tid & 31);
    const uint32_t w = blockIdx.x;
    const uint32_t lo = w * chunk, hi = min(n, lo + chunk);
    const uint32_t mask = (1u << width) - 1u;
    const uint32_t w0 = min(width, 8u);
    uint32_t* row = rows + (size_t)256 * w;
    const uint32_t o0 = tid * ITEMS;   // this thread's consecutive positions after sorting

    for (uint32_t t0 = lo; t0 < hi; t0 += TILE) {
        const uint32_t len = min(TILE, hi - t0);
        K k[ITEMS];
        uint32_t v[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t o = hofs + i * 32;
            k[i] = o < len ? keys_in[t0 + o] : K(0);
            v[i] = KV && o < len ? vals_in[t0 + o] : 0u;
        }
        // stable sort of the tile by the digit: low 8 bits, then the rest;
        // the keys are ordered by the rest, so a tile whose first and last
        // keys agree on it needs only the first
        const bool one_group = width <= 8 || (digit_of(keys_in[t0], shift, mask) >> 8) ==
                                                 (digit_of(keys_in[t0 + len - 1], shift, mask) >> 8);
        if (one_group) {
            place_one_group<K, KV, WG, ITEMS>(sm, gofs, k, v, len, shift, width, mask, row, n,
                                              keys_in[t0], keys_out, vals_out);
            continue;
        }
        // held: LDS holds the tile in its final order (a round that finds
        // itself the identity has overwritten LDS with its slots)
        bool held = tile_round<K, KV, WG, ITEMS, true>(sm, k, v, len, shift, (1u << w0) - 1u);
        if (!one_group)
            held = tile_round<K, KV, WG, ITEMS, true>(sm, k, v, len, shift + 8, (1u << (width - 8)) - 1u);
        if (!held) {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t o = hofs + i * 32;
                if (o < len) {
                    sm.keys[o] = k[i];
                    if (KV) sm.vals[o] = v[i];
                }
            }
            __syncthreads();
        }
        // each thread takes ITEMS consecutive sorted positions
        K kk[ITEMS];
        uint32_t dg[ITEMS];
        {
            const uint4* src = (const uint4*)&sm.keys[o0];
#pragma unroll
            for (int q = 0; q < (int)(ITEMS * sizeof(K) / 16); ++q) ((uint4*)kk)[q] = src[q];
        }
        const uint32_t dprev = (o0 > 0 && o0 - 1 < len) ? digit_of(sm.keys[o0 - 1], shift, mask) : 0xFFFFFFFFu;
        const uint32_t dnext = (o0 + ITEMS < len) ? digit_of(sm.keys[o0 + ITEMS], shift, mask) : 0xFFFFFFFFu;
        uint32_t mhead = 0;   // last run start at or before this thread's positions
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            dg[i] = digit_of(kk[i], shift, mask);
            const uint32_t pd = i == 0 ? dprev : dg[i - 1];
            if (o0 + i < len && (o0 + i == 0 || pd != dg[i])) mhead = o0 + i;
        }
        // exclusive max-scan of the heads over the threads in position order
        const uint32_t incl = wave_inclusive_max(mhead);
        if (lane == 63) wmax[wave] = incl;
        uint32_t carry = __shfl_up(incl, 1, 64);
        if (lane == 0) carry = 0;
        __syncthreads();
        for (uint32_t q = 0; q < wave; ++q) carry = max(carry, wmax[q]);
        uint32_t base[ITEMS];
        uint32_t cur = carry;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t o = o0 + i;
            const uint32_t pd = i == 0 ? dprev : dg[i - 1];
            if (o < len && (o == 0 || pd != dg[i])) cur = o;
            base[i] = o < len ? __hip_atomic_load(&row[dg[i]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) + o - cur
                              : 0u;
        }
        __syncthreads();   // every read of the row precedes its updates
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t o = o0 + i;
            if (o < len) {
                dest[o] = base[i];
                const uint32_t nd = i + 1 < ITEMS ? dg[i + 1] : dnext;
                if (o + 1 == len || nd != dg[i])
                    __hip_atomic_store(&row[dg[i]], base[i] + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        __syncthreads();
        for (uint32_t p = tid; p < len; p += WG) {
            const uint32_t d = dest[p];
            if (d < n) {   // always true when the rows are consistent
                keys_out[d] = sm.keys[p];
                if (KV) vals_out[d] = sm.vals[p];
            }
        }
        __syncthreads();   // the row is this workgroup's alone: workgroup scope suffices
    }
}

template <typename K, bool KV>
hipError_t run16(const void* keys_in, void* keys_out, const uint32_t* vals_in, uint32_t* vals_out,
                 size_t n, int begin_bit, int end_bit, void* ws, const LsdR16Layout& L,
                 uint32_t* dev_err, hipStream_t stream, Profiler* prof)
{
    uint8_t* w = (uint8_t*)ws;
    K* tmp = (K*)(w + L.off_tmp_keys);
    uint32_t* vtmp = KV ? (uint32_t*)(w + L.off_tmp_vals) : nullptr;
    K* grp = (K*)(w + L.off_grp_keys);
    uint32_t* vgrp = KV ? (uint32_t*)(w + L.off_grp_vals) : nullptr;
    uint32_t* rows = (uint32_t*)(w + L.off_rows);
    uint32_t* tot = (uint32_t*)(w + L.off_tot);
    uint2* win = (uint2*)(w + L.off_win);
    const LsdR8Layout L8 = lsd_r8_layout((int)sizeof(K), KV, n, 0, 8);
    const uint32_t rounds = L.rounds;
    const K* src = (const K*)keys_in;
    const uint32_t* vsrc = vals_in;
    hipError_t e;
    if ((rounds & 1) && (keys_in == keys_out || (KV && vals_in == vals_out))) {
        // an odd round count ends in the output, so round 0 would read and
        // write the aliased array: start from a copy
        e = copy_bytes(tmp, keys_in, n * sizeof(K), stream);
        if (e == hipSuccess && KV) e = copy_bytes(vtmp, vals_in, n * 4, stream);
        if (e != hipSuccess) return e;
        src = tmp;
        vsrc = vtmp;
    }
    for (uint32_t d = 0; d < rounds; ++d) {
        const uint32_t shift = (uint32_t)begin_bit + 16u * d;
        const uint32_t width = std::min(16u, (uint32_t)end_bit - shift);
        const uint32_t mask = (1u << width) - 1u;
        const uint32_t nbins = mask + 1;
        const bool to_tmp = ((rounds - 1 - d) & 1) != 0;
        K* dst = to_tmp ? tmp : (K*)keys_out;
        uint32_t* vdst = KV ? (to_tmp ? vtmp : vals_out) : nullptr;
        const bool group = width > 8;
        if (group) {
            // stable grouping by the digit's high byte into grp
            if (prof) profiler_mark(prof, stream, kKindGroup, true);
            e = lsd_r8_sort((int)sizeof(K), src, grp, vsrc, vgrp, n, (int)shift + 8,
                            (int)(shift + width), w + L.off_r8, L8, dev_err, stream, nullptr);
            if (prof) profiler_mark(prof, stream, kKindGroup, false);
            if (e != hipSuccess) return e;
            src = grp;
            vsrc = vgrp;
        }
        if (prof) profiler_mark(prof, stream, kKindCount, true);
        hipLaunchKernelGGL(k_rows16<K>, dim3(L.nchunks), dim3(kRowsWG), 0, stream,
                           src, (uint32_t)n, L.chunk, shift, mask, rows, win, group);
        if (prof) profiler_mark(prof, stream, kKindCount, false);
        if (prof) profiler_mark(prof, stream, kKindTileScan, true);
        const uint32_t nb = (nbins + 255) / 256;
        uint32_t* btot = tot + kR16;
        hipLaunchKernelGGL(k_colsum16, dim3(nb), dim3(256), 0, stream, (const uint32_t*)rows,
                           (const uint2*)win, L.nchunks, nbins, tot, btot);
        hipLaunchKernelGGL(k_blockscan16, dim3(1), dim3(256), 0, stream, btot, nb);
        hipLaunchKernelGGL(k_colprefix16, dim3(nb), dim3(256), 0, stream, rows, (const uint2*)win,
                           L.nchunks, nbins, (const uint32_t*)tot, (const uint32_t*)btot);
        if (prof) profiler_mark(prof, stream, kKindTileScan, false);
        if (prof) profiler_mark(prof, stream, kKindRound, true);
        hipLaunchKernelGGL((k_place16<K, KV>), dim3(L.nchunks), dim3(R16Config<K>::WG), 0, stream,
                           src, dst, vsrc, vdst, (uint32_t)n, L.chunk, shift, width, rows);
        if (prof) profiler_mark(prof, stream, kKindRound, false);
        src = dst;
        vsrc = vdst;
    }
    return hipGetLastError();
}

}  // namespace

LsdR16Layout lsd_r16_layout(int key_bytes, bool has_vals, size_t n, int begin_bit, int end_bit)
{
    LsdR16Layout L{};
    L.rounds = (uint32_t)((end_bit - begin_bit + 15) / 16);
    const uint32_t tile = key_bytes == 8 ? r16_tile<uint64_t>() : r16_tile<uint32_t>();
    size_t per = (n + kMaxChunks - 1) / kMaxChunks;
    per = std::max<size_t>((size_t)kChunkTiles * tile, (per + tile - 1) / tile * tile);
    L.chunk = (uint32_t)per;
    L.nchunks = (uint32_t)std::max<size_t>(1, (n + per - 1) / per);
    size_t o = 0;
    L.off_tmp_keys = o;  o = align_up(o + n * key_bytes);
    L.off_tmp_vals = o;  o = align_up(o + (has_vals ? n * 4 : 0));
    L.off_rows = o;      o = align_up(o + (size_t)256 * (L.nchunks + 255) * 4);
    L.off_win = o;       o = align_up(o + (size_t)L.nchunks * sizeof(uint2));
    L.off_tot = o;       o = align_up(o + (size_t)(kR16 + 256) * 4);
    // the grouped keys and the radix-256 workspace of the grouping round
    // (rounds wider than 8 bits)
    const bool group = end_bit - begin_bit > 8;
    L.off_grp_keys = o;  o = align_up(o + (group ? n * key_bytes : 0));
    L.off_grp_vals = o;  o = align_up(o + (group && has_vals ? n * 4 : 0));
    L.off_r8 = o;        o = align_up(o + (group ? lsd_r8_layout(key_bytes, has_vals, n, 0, 8).bytes : 0));
    L.bytes = o;
    return L;
}

hipError_t lsd_r16_sort(int key_bytes, const void* keys_in, void* keys_out,
                        const uint32_t* vals_in, uint32_t* vals_out, size_t n, int begin_bit,
                        int end_bit, void* ws, const LsdR16Layout& L, uint32_t* dev_err,
                        hipStream_t stream, Profiler* prof)
{
    if (!n || !L.rounds) return hipSuccess;
    const bool kv = vals_in != nullptr;
    if (key_bytes == 4)
        return kv ? run16<uint32_t, true>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof)
                  : run16<uint32_t, false>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof);
    return kv ? run16<uint64_t, true>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof)
              : run16<uint64_t, false>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof);
}

}  // namespace rsort
