// PR4 on gfx950: LSD radix sort with radix 2^8, one stable count-sort round
// per 8-bit digit (arXiv 1808.10292, Section 3.2, PR4 / eq. Tp4).
//
// The paper's round (count digits, exchange the p x r counts, route keys) maps
// onto one MI355X like this:
//   k_hist   one read of the keys counts every digit of every round at once
//            (the count loops of all rounds; LDS histograms, 8 global copies);
//   k_scan   exclusive prefix of each round's 256 counts = where each digit's
//            bucket starts in the output, plus the round plan (identity rounds,
//            i.e. one digit value holding all n keys, are skipped);
//   k_round  one launch per round.  Each workgroup takes one tile of keys in
//            ticket order, ranks them stably by digit in LDS, learns how many
//            keys of each digit all earlier tiles hold through a decoupled
//            look-back over per-(tile, digit) words (the paper's count
//            exchange), stages the tile in digit order in LDS and writes every
//            key (and payload) once to its final slot (the routing).
// Keys and payloads are read once and written once per round.
#include "device_common.h"
#include "rsort_internal.h"

namespace rsort {
namespace {

constexpr uint32_t R = 256;  // radix

// Tile shape: WG threads, ITEMS keys per thread (tile = WG * ITEMS keys), and
// the number of predecessor words a look-back step reads at once.
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
#ifndef LB_WINDOW
#define LB_WINDOW 4
#endif
#ifndef RSORT_R8_WAVES_PER_EU
#define RSORT_R8_WAVES_PER_EU 6
#endif
template <typename K> struct R8Config;
template <> struct R8Config<uint32_t> {
    static constexpr int WG = RSORT_R8_WG32;
    static constexpr int ITEMS = RSORT_R8_ITEMS32;
};
template <> struct R8Config<uint64_t> {
    static constexpr int WG = RSORT_R8_WG64;
    static constexpr int ITEMS = RSORT_R8_ITEMS64;
};

constexpr int kHistWG = 256;
constexpr int kHistUnroll = 8;

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
    const uint32_t* bases;   // [round][256]
    const RoundPlan* plan;
    uint32_t* tickets;       // [round]
    uint32_t* state0;        // [ntiles][256], rounds with even ordinal
    uint32_t* state1;        // [ntiles][256], rounds with odd ordinal
    uint32_t* err;
};

template <typename T>
__device__ __forceinline__ T* pick(int sel, const T* in, T* out, T* tmp)
{
    return sel == 0 ? const_cast<T*>(in) : (sel == 1 ? out : tmp);
}

// Zero the global histogram copies, the tile tickets and the look-back words
// of the first round.
__global__ void k_init(uint32_t* hist, uint32_t hist_words, uint32_t* tickets,
                       uint32_t nrounds, uint32_t* state0, size_t state_words)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t i = g; i < hist_words; i += stride) hist[i] = 0;
    for (size_t i = g; i < nrounds; i += stride) tickets[i] = 0;
    for (size_t i = g; i < state_words; i += stride) state0[i] = 0;
}

// Counts of every 8-bit digit of [begin_bit, end_bit) in one pass over the
// keys: LDS histograms per workgroup, then one global atomic per nonzero bin
// into copy (block index mod 8), which spreads contention across the XCDs.
template <typename K>
__global__ __launch_bounds__(kHistWG) void k_hist(const K* __restrict__ keys, uint32_t n,
                                                  uint32_t begin_bit, uint32_t end_bit,
                                                  uint32_t nrounds, uint32_t* hist)
{
    __shared__ uint32_t h[kMaxRounds * R];
    for (uint32_t i = threadIdx.x; i < nrounds * R; i += kHistWG) h[i] = 0;
    __syncthreads();

    uint32_t shift[kMaxRounds], mask[kMaxRounds];
#pragma unroll
    for (int d = 0; d < kMaxRounds; ++d) {
        uint32_t lo = begin_bit + 8u * d;
        uint32_t w = lo < end_bit ? min(8u, end_bit - lo) : 0u;
        shift[d] = lo < end_bit ? lo : 0u;
        mask[d] = (1u << w) - 1u;
    }

    const uint32_t stride = gridDim.x * kHistWG;
    uint32_t i = blockIdx.x * kHistWG + threadIdx.x;
    for (; i + (kHistUnroll - 1) * stride < n; i += kHistUnroll * stride) {
        K k[kHistUnroll];
#pragma unroll
        for (int u = 0; u < kHistUnroll; ++u) k[u] = keys[i + u * stride];
#pragma unroll
        for (int u = 0; u < kHistUnroll; ++u) {
#pragma unroll
            for (int d = 0; d < kMaxRounds; ++d) {
                if ((uint32_t)d < nrounds)
                    atomicAdd(&h[d * R + digit_of(k[u], shift[d], mask[d])], 1u);
            }
        }
    }
    for (; i < n; i += stride) {
        K key = keys[i];
#pragma unroll
        for (int d = 0; d < kMaxRounds; ++d)
            if ((uint32_t)d < nrounds) atomicAdd(&h[d * R + digit_of(key, shift[d], mask[d])], 1u);
    }
    __syncthreads();
    uint32_t* dst = hist + (blockIdx.x % kHistReplicas) * nrounds * R;
    for (uint32_t b = threadIdx.x; b < nrounds * R; b += kHistWG) {
        uint32_t c = h[b];
        if (c) atomicAdd(&dst[b], c);
    }
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

// Round bases (exclusive prefix of each round's counts) and the round plan.
// One workgroup of 256 threads, thread t owns digit value t.
__global__ __launch_bounds__(R) void k_scan(const uint32_t* hist, uint32_t nrounds, uint32_t n,
                                            int in_place, uint32_t* bases, RoundPlan* plan)
{
    __shared__ uint32_t wsum[4];
    __shared__ int identity[kMaxRounds];
    const uint32_t t = threadIdx.x;
    if (t < kMaxRounds) identity[t] = 0;
    __syncthreads();
    for (uint32_t d = 0; d < nrounds; ++d) {
        uint32_t c = 0;
        for (int rep = 0; rep < kHistReplicas; ++rep) c += hist[(rep * nrounds + d) * R + t];
        uint32_t incl = block256_inclusive_sum(c, wsum);
        bases[d * R + t] = incl - c;
        if (c == n) identity[d] = 1;
    }
    __syncthreads();
    if (t == 0) {
        int exec[kMaxRounds];
        int m = 0;
        for (uint32_t d = 0; d < nrounds; ++d) {
            exec[d] = !identity[d];
            m += exec[d];
        }
        // The last round must land in the caller's output and no round may
        // read and write the same buffer.  Rounds alternate between output and
        // temporary backwards from the last one, so: without aliasing at least
        // one round must run; in place, an even number must (re-enable an
        // identity round, or copy the input to the temporary first).
        int precopy = 0;
        if (!in_place && m == 0) {
            exec[nrounds - 1] = 1;
            m = 1;
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
}

// In-place sorts with an odd number of running rounds: copy input -> temporary.
template <typename K>
__global__ void k_precopy(const RoundPlan* plan, const K* keys, K* keys_tmp,
                          const uint32_t* vals, uint32_t* vals_tmp, uint32_t n)
{
    if (!plan[kMaxRounds].exec) return;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        keys_tmp[i] = keys[i];
        if (vals) vals_tmp[i] = vals[i];
    }
}

// One stable count-sort round over all tiles (see the file comment).
//
// Layout: the tile is split among half-waves (32 lanes); half-wave h owns the
// contiguous keys [h*ITEMS*32, (h+1)*ITEMS*32) of the tile, row i lane l at
// h*ITEMS*32 + i*32 + (l & 31), so "earlier in the input" is lexicographic
// (h, i, l) -- the order the ranking below preserves.
//
// Phases of a tile:
//   count   each half-wave counts its digits into its own LDS row;
//   publish digit thread v sums the rows, publishes the tile's count of v
//           (aggregate) for later tiles, turns the rows into per-half-wave
//           slot bases, and issues the first look-back loads;
//   rank    each half-wave ranks its keys in row order: lanes OR their bit
//           into the slot of their digit, the set of lanes below with the same
//           digit gives the rank, and the digit's base advances by the set size;
//   lookback digit threads finish folding predecessor words into the number of
//           keys of v in all earlier tiles, and publish the inclusive prefix;
//   scatter the tile is staged in digit order and written out, consecutive
//           threads writing consecutive slots of a digit's run (payloads in a
//           second staging pass through the same LDS).
template <typename K, bool KV, int WG, int ITEMS>
__global__ __launch_bounds__(WG, RSORT_R8_WAVES_PER_EU) void k_round(RoundArgs a)
{
    constexpr int HW = WG / 32;                 // half-waves
    constexpr uint32_t TILE = (uint32_t)WG * ITEMS;
    constexpr uint32_t STAGE_WORDS = TILE * sizeof(K) / 4;
    constexpr uint32_t TABLE_WORDS = HW * R;
    static_assert(STAGE_WORDS >= TABLE_WORDS, "staging must cover the count table");
    static_assert(TILE <= 65536, "16-bit slot bases");
    struct Smem {
        union {
            uint32_t table[HW][R];   // counts, then lane sets of the ranking
            K keys[TILE];            // staging: the tile in digit order
            uint32_t vals[TILE];     // staging of the payloads (second pass)
        } u;
        uint16_t base[HW][R];        // next slot of digit v for half-wave h
        uint32_t goff[R];            // output index of tile slot 0 of each digit
        uint32_t wsum[4];
        uint32_t tile;
    };
    __shared__ Smem sm;

    const RoundPlan pl = a.plan[a.round];
    if (!pl.exec) return;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    const uint32_t wave = tid >> 6;
    const uint32_t hw = tid >> 5;
    const uint32_t hl = tid & 31;

    for (uint32_t i = tid; i < TABLE_WORDS; i += WG) (&sm.u.table[0][0])[i] = 0;
    if (tid == 0) sm.tile = atomicAdd(&a.tickets[a.round], 1u);
    __syncthreads();

    const uint32_t tile = sm.tile;
    const uint32_t base = tile * TILE;
    const uint32_t lim = a.n - base;   // keys in this tile (>= TILE except the last)
    const K* src = pick<K>(pl.src, (const K*)a.keys_in, (K*)a.keys_out, (K*)a.keys_tmp);
    const uint32_t* vsrc = KV ? pick<uint32_t>(pl.src, a.vals_in, a.vals_out, a.vals_tmp) : nullptr;

    const uint32_t hofs = hw * ITEMS * 32 + hl;
    K k[ITEMS];
    uint32_t v[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t o = hofs + i * 32;
        k[i] = o < lim ? src[base + o] : K(0);
        if (KV) v[i] = o < lim ? vsrc[base + o] : 0u;
    }

    // count
    uint32_t* row = sm.u.table[hw];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if (hofs + i * 32 < lim) atomicAdd(&row[digit_of(k[i], a.shift, a.mask)], 1u);
    __syncthreads();

    // publish
    uint32_t* region = (pl.ord & 1) ? a.state1 : a.state0;
    uint32_t* next_region = (pl.ord & 1) ? a.state0 : a.state1;
    uint32_t total = 0, tstart = 0;
    uint32_t lb[LB_WINDOW];
    if (tid < R) {
#pragma unroll
        for (int h = 0; h < HW; ++h) {
            const uint32_t c = sm.u.table[h][tid];
            sm.u.table[h][tid] = 0;          // the same rows hold the lane sets next
            sm.base[h][tid] = (uint16_t)total;
            total += c;
        }
        st_agent(&region[(size_t)tile * R + tid], (tile == 0 ? kFlagPrefix : kFlagAggregate) | total);
        const uint32_t incl = wave_inclusive_sum(total);
        if (lane == 63) sm.wsum[wave] = incl;
        tstart = incl - total;
#pragma unroll
        for (int q = 0; q < LB_WINDOW; ++q)
            lb[q] = (uint32_t)q < tile ? ld_agent(&region[(size_t)(tile - 1 - q) * R + tid]) : kFlagPrefix;
    }
    __syncthreads();
    if (tid < R) {
        for (uint32_t w = 0; w < wave; ++w) tstart += sm.wsum[w];
#pragma unroll
        for (int h = 0; h < HW; ++h) sm.base[h][tid] = (uint16_t)(sm.base[h][tid] + tstart);
    }
    __syncthreads();

    // rank
    uint32_t pos[ITEMS];
    {
        uint32_t* lanes = sm.u.table[hw];
        uint16_t* hb = sm.base[hw];
        const uint32_t bit = 1u << hl;
        const uint32_t lowsel = lane < 32 ? ~0u : 0u;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const bool ok = hofs + i * 32 < lim;
            const uint32_t d = digit_of(k[i], a.shift, a.mask);
            if (ok) __hip_atomic_fetch_or(&lanes[d], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            wave_lds_order();
            const uint32_t m = ok ? __hip_atomic_load(&lanes[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 0u;
            const uint32_t b = hb[d];
            pos[i] = __builtin_amdgcn_mbcnt_hi(m, __builtin_amdgcn_mbcnt_lo(m & lowsel, b));
            wave_lds_order();
            if (ok) {
                hb[d] = (uint16_t)(b + __builtin_popcount(m));
                __hip_atomic_store(&lanes[d], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            wave_lds_order();
        }
    }

    // lookback: fold predecessor words nearest first -- aggregates are added
    // and passed over, the first inclusive prefix ends the walk, a word not
    // yet published is polled again.  The first window was loaded before the
    // ranking.
    if (tid < R) {
        uint32_t excl = 0;
        if (tile > 0) {
            uint32_t j = tile;   // entries j-1, j-2, ... are still to be folded
            uint32_t spins = 0;
            for (;;) {
                uint32_t used = 0, pval = 0;
                bool done = false;
#pragma unroll
                for (int q = 0; q < LB_WINDOW; ++q) {
                    if (!done && used == (uint32_t)q) {
                        const uint32_t f = lb[q] >> kFlagShift;
                        if (f != 0) {
                            excl += lb[q] & kCountMask;
                            used = q + 1;
                            done = f == (kFlagPrefix >> kFlagShift);
                            pval = lb[q] & kCountMask;
                        }
                    }
                }
                if (done) {
                    // Help: the aggregate-only tiles folded in this window now
                    // have known inclusive prefixes; publish them so later
                    // tiles stop their walks here.  The value is unique, so a
                    // race with the owner's own store of it is harmless.
                    uint32_t run = pval;
#pragma unroll
                    for (int q = LB_WINDOW - 2; q >= 0; --q) {
                        if ((uint32_t)q + 1 < used) {
                            run += lb[q] & kCountMask;
                            st_agent(&region[(size_t)(j - 1 - q) * R + tid], kFlagPrefix | (run & kCountMask));
                        }
                    }
                    break;
                }
                j -= used;
                if (used == 0) {
                    // Give up after kSpinLimit polls, or at once if another
                    // tile already gave up, so the grid always drains.
                    if (++spins > kSpinLimit ||
                        ((spins & 255u) == 0 && (ld_agent(a.err) & kErrLookbackTimeout))) {
                        atomicOr(a.err, (uint32_t)kErrLookbackTimeout);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
#pragma unroll
                for (int q = 0; q < LB_WINDOW; ++q)
                    lb[q] = (uint32_t)q < j ? ld_agent(&region[(size_t)(j - 1 - q) * R + tid]) : kFlagPrefix;
            }
            st_agent(&region[(size_t)tile * R + tid], kFlagPrefix | ((excl + total) & kCountMask));
        }
        next_region[(size_t)tile * R + tid] = 0u;
        sm.goff[tid] = a.bases[a.round * R + tid] + excl - tstart;
    }
    __syncthreads();

    // scatter
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if (hofs + i * 32 < lim) sm.u.keys[pos[i]] = k[i];
    __syncthreads();
    K* dst = pick<K>(pl.dst, (const K*)a.keys_in, (K*)a.keys_out, (K*)a.keys_tmp);
    uint32_t outi[KV ? ITEMS : 1];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = i * WG + tid;
        uint32_t o = a.n;
        if (p < lim) {
            const K key = sm.u.keys[p];
            o = sm.goff[digit_of(key, a.shift, a.mask)] + p;
            if (o < a.n) dst[o] = key;   // always true unless a look-back wait was abandoned
        }
        if (KV) outi[i] = o;
    }
    if (KV) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            if (hofs + i * 32 < lim) sm.u.vals[pos[i]] = v[i];
        __syncthreads();
        uint32_t* vdst = pick<uint32_t>(pl.dst, a.vals_in, a.vals_out, a.vals_tmp);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = i * WG + tid;
            if (p < lim && outi[i] < a.n) vdst[outi[i]] = sm.u.vals[p];
        }
    }
}

__global__ void k_copy_bytes(const uint8_t* src, uint8_t* dst, size_t bytes)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < bytes; i += stride)
        dst[i] = src[i];
}

uint32_t rounds_of(int begin_bit, int end_bit, int digit_bits)
{
    return end_bit > begin_bit ? (uint32_t)((end_bit - begin_bit + digit_bits - 1) / digit_bits) : 0u;
}

uint32_t hist_grid(size_t n)
{
    size_t per = (size_t)kHistWG * 16;
    size_t g = (n + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 1024) g = 1024;
    return (uint32_t)g;
}

template <typename K, bool KV>
hipError_t run(const void* keys_in, void* keys_out, const uint32_t* vals_in, uint32_t* vals_out,
               size_t n, int begin_bit, int end_bit, void* ws, const LsdR8Layout& L,
               uint32_t* dev_err, hipStream_t stream, Profiler* prof)
{
    constexpr int WG = R8Config<K>::WG;
    constexpr int ITEMS = R8Config<K>::ITEMS;
    uint8_t* w = (uint8_t*)ws;
    uint32_t* hist = (uint32_t*)(w + L.off_hist);
    uint32_t* bases = (uint32_t*)(w + L.off_bases);
    RoundPlan* plan = (RoundPlan*)(w + L.off_plan);
    uint32_t* tickets = (uint32_t*)(w + L.off_tickets);
    uint32_t* state0 = (uint32_t*)(w + L.off_state0);
    uint32_t* state1 = (uint32_t*)(w + L.off_state1);
    K* keys_tmp = (K*)(w + L.off_tmp_keys);
    uint32_t* vals_tmp = KV ? (uint32_t*)(w + L.off_tmp_vals) : nullptr;
    const uint32_t nr = L.rounds;
    const bool in_place = keys_in == keys_out || (KV && vals_in == vals_out);

    hipLaunchKernelGGL(k_init, dim3(256), dim3(256), 0, stream, hist,
                       (uint32_t)(kHistReplicas * nr * R), tickets, nr, state0,
                       (size_t)L.ntiles * R);
    if (prof) profiler_mark(prof, stream, kKindHist, true);
    if (prof) profiler_mark(prof, stream, kKindHist, true);
    hipLaunchKernelGGL(k_hist<K>, dim3(hist_grid(n)), dim3(kHistWG), 0, stream,
                       (const K*)keys_in, (uint32_t)n, (uint32_t)begin_bit, (uint32_t)end_bit, nr, hist);
    if (prof) profiler_mark(prof, stream, kKindHist, false);
    if (prof) profiler_mark(prof, stream, kKindHist, false);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(R), 0, stream, (const uint32_t*)hist, nr,
                       (uint32_t)n, (int)in_place, bases, plan);
    if (in_place && (nr & 1)) {
        uint32_t g = (uint32_t)std::min<size_t>((n + 255) / 256, 2048);
        hipLaunchKernelGGL(k_precopy<K>, dim3(g), dim3(256), 0, stream, (const RoundPlan*)plan,
                           (const K*)keys_in, keys_tmp, KV ? vals_in : nullptr, vals_tmp, (uint32_t)n);
    }
    for (uint32_t d = 0; d < nr; ++d) {
        RoundArgs a;
        a.keys_in = keys_in;
        a.keys_out = keys_out;
        a.keys_tmp = keys_tmp;
        a.vals_in = vals_in;
        a.vals_out = vals_out;
        a.vals_tmp = vals_tmp;
        a.n = (uint32_t)n;
        a.shift = (uint32_t)begin_bit + 8u * d;
        a.mask = (1u << std::min(8u, (uint32_t)end_bit - a.shift)) - 1u;
        a.round = d;
        a.bases = bases;
        a.plan = plan;
        a.tickets = tickets;
        a.state0 = state0;
        a.state1 = state1;
        a.err = dev_err;
        if (prof) profiler_mark(prof, stream, kKindRound, true);
        if (prof) profiler_mark(prof, stream, kKindRound, true);
        hipLaunchKernelGGL((k_round<K, KV, WG, ITEMS>), dim3(L.ntiles), dim3(WG), 0, stream, a);
        if (prof) profiler_mark(prof, stream, kKindRound, false);
        if (prof) profiler_mark(prof, stream, kKindRound, false);
    }
    return hipGetLastError();
}

}  // namespace

LsdR8Layout lsd_r8_layout(int key_bytes, bool has_vals, size_t n, int begin_bit, int end_bit)
{
    LsdR8Layout L{};
    L.rounds = rounds_of(begin_bit, end_bit, 8);
    L.tile = key_bytes == 8 ? R8Config<uint64_t>::WG * R8Config<uint64_t>::ITEMS
                            : R8Config<uint32_t>::WG * R8Config<uint32_t>::ITEMS;
    L.ntiles = (uint32_t)((n + L.tile - 1) / L.tile);
    size_t o = 0;
    L.off_tmp_keys = o; o = align_up(o + n * key_bytes);
    L.off_tmp_vals = o; o = align_up(o + (has_vals ? n * 4 : 0));
    L.off_state0 = o;   o = align_up(o + (size_t)L.ntiles * R * 4);
    L.off_state1 = o;   o = align_up(o + (size_t)L.ntiles * R * 4);
    L.off_hist = o;     o = align_up(o + (size_t)kHistReplicas * kMaxRounds * R * 4);
    L.off_bases = o;    o = align_up(o + (size_t)kMaxRounds * R * 4);
    L.off_plan = o;     o = align_up(o + (kMaxRounds + 1) * sizeof(RoundPlan));
    L.off_tickets = o;  o = align_up(o + kMaxRounds * 4);
    L.bytes = o;
    return L;
}

hipError_t lsd_r8_sort(int key_bytes, const void* keys_in, void* keys_out,
                       const uint32_t* vals_in, uint32_t* vals_out, size_t n,
                       int begin_bit, int end_bit, void* ws, const LsdR8Layout& L,
                       uint32_t* dev_err, hipStream_t stream, Profiler* prof)
{
    const bool kv = vals_in != nullptr;
    if (key_bytes == 4)
        return kv ? run<uint32_t, true>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof)
                  : run<uint32_t, false>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof);
    return kv ? run<uint64_t, true>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof)
              : run<uint64_t, false>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof);
}

hipError_t copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t stream)
{
    if (!bytes || dst == src) return hipSuccess;
    uint32_t g = (uint32_t)std::min<size_t>((bytes + 255) / 256, 4096);
    hipLaunchKernelGGL(k_copy_bytes, dim3(g), dim3(256), 0, stream, (const uint8_t*)src,
                       (uint8_t*)dst, bytes);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stand-alone digit histograms (8-bit: the k_hist above; 16-bit: LDS halves).

namespace {

__global__ void k_zero(uint32_t* p, size_t words)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = 0;
}

__global__ void k_hist_reduce(const uint32_t* reps, uint32_t words, uint32_t* out)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= words) return;
    uint32_t s = 0;
    for (int r = 0; r < kHistReplicas; ++r) s += reps[r * words + i];
    out[i] = s;
}

// 16-bit digits: 65536 bins do not fit LDS as 32-bit counters, so each
// workgroup counts one half of the digit values (32768 bins, 128 KiB) of one
// round over a contiguous chunk, then adds its nonzero bins to the output.
constexpr int kH16WG = 1024;
constexpr uint32_t kH16Bins = 32768;

template <typename K>
__global__ __launch_bounds__(kH16WG) void k_hist16(const K* __restrict__ keys, uint32_t n,
                                                   uint32_t begin_bit, uint32_t end_bit,
                                                   uint32_t chunk, uint32_t* out)
{
    extern __shared__ uint32_t h16[];
    const uint32_t round = blockIdx.y >> 1, half = blockIdx.y & 1;
    const uint32_t shift = begin_bit + 16u * round;
    const uint32_t width = min(16u, end_bit - shift);
    const uint32_t mask = (1u << width) - 1u;
    for (uint32_t i = threadIdx.x; i < kH16Bins; i += kH16WG) h16[i] = 0;
    __syncthreads();
    const uint32_t lo = blockIdx.x * chunk;
    const uint32_t hi = min(n, lo + chunk);
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kH16WG) {
        const uint32_t d = digit_of(keys[i], shift, mask);
        if ((d >> 15) == half) atomicAdd(&h16[d & (kH16Bins - 1)], 1u);
    }
    __syncthreads();
    uint32_t* o = out + (size_t)round * 65536 + half * kH16Bins;
    for (uint32_t b = threadIdx.x; b < kH16Bins; b += kH16WG) {
        const uint32_t c = h16[b];
        if (c) atomicAdd(&o[b], c);
    }
}

}  // namespace

size_t histogram_ws_bytes(int digit_bits, int begin_bit, int end_bit)
{
    if (digit_bits == 8) return (size_t)kHistReplicas * kMaxRounds * R * 4;
    return 0;
}

hipError_t histogram(int key_bytes, const void* keys, size_t n, int digit_bits,
                     int begin_bit, int end_bit, uint32_t* hist_out, void* ws,
                     hipStream_t stream)
{
    const uint32_t nr = rounds_of(begin_bit, end_bit, digit_bits);
    if (nr == 0) return hipSuccess;
    if (digit_bits == 8) {
        uint32_t* reps = (uint32_t*)ws;
        const uint32_t words = nr * R;
        hipLaunchKernelGGL(k_zero, dim3(64), dim3(256), 0, stream, reps, (size_t)kHistReplicas * words);
        if (key_bytes == 4)
            hipLaunchKernelGGL(k_hist<uint32_t>, dim3(hist_grid(n)), dim3(kHistWG), 0, stream,
                               (const uint32_t*)keys, (uint32_t)n, (uint32_t)begin_bit, (uint32_t)end_bit, nr, reps);
        else
            hipLaunchKernelGGL(k_hist<uint64_t>, dim3(hist_grid(n)), dim3(kHistWG), 0, stream,
                               (const uint64_t*)keys, (uint32_t)n, (uint32_t)begin_bit, (uint32_t)end_bit, nr, reps);
        hipLaunchKernelGGL(k_hist_reduce, dim3((words + 255) / 256), dim3(256), 0, stream,
                           (const uint32_t*)reps, words, hist_out);
        return hipGetLastError();
    }
    // 16-bit digits
    hipLaunchKernelGGL(k_zero, dim3(256), dim3(256), 0, stream, hist_out, (size_t)nr * 65536);
    const uint32_t chunk = 1u << 20;
    const uint32_t nchunks = (uint32_t)std::max<size_t>(1, (n + chunk - 1) / chunk);
    const size_t lds = kH16Bins * 4;
    (void)hipFuncSetAttribute((const void*)k_hist16<uint32_t>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void*)k_hist16<uint64_t>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (key_bytes == 4)
        hipLaunchKernelGGL(k_hist16<uint32_t>, dim3(nchunks, 2 * nr), dim3(kH16WG), lds, stream,
                           (const uint32_t*)keys, (uint32_t)n, (uint32_t)begin_bit, (uint32_t)end_bit, chunk, hist_out);
    else
        hipLaunchKernelGGL(k_hist16<uint64_t>, dim3(nchunks, 2 * nr), dim3(kH16WG), lds, stream,
                           (const uint64_t*)keys, (uint32_t)n, (uint32_t)begin_bit, (uint32_t)end_bit, chunk, hist_out);
    return hipGetLastError();
}

}  // namespace rsort
