// Single-read count-sort rounds of the plain radix-2^8 sort (Section 3.2,
// PR4): every round reads each key once and writes it once.
//
// A round of the paper counts, exchanges the p x r counts and routes.  Here a
// tile of keys counts its digits, learns how many keys of each digit precede
// it from its predecessor tiles (a decoupled look-back over published counts)
// and routes its keys, all in one kernel.  What keeps the look-back short on a
// chip whose cross-XCD publish-to-observe time is about a microsecond is that
// the tiles of a round are split into independent chains whose totals are
// known before the round starts:
//
//   * the first round that runs reads the input in its original order; its
//     chains are the contiguous chunks the counting pass read, and the counts
//     of every digit per chunk come out of that pass;
//   * a later round reads the output of the round before it, which is ordered
//     by that round's digit.  Its chains are the key ranges that share the top
//     kChainBits bits of the previous digit: contiguous in the round's input,
//     with digit counts given by the joint histogram of (top bits of digit
//     d - 1, digit d), a histogram of a 12-bit window of the key that the
//     counting pass also takes.
//
// So output index = digit start + keys of that digit in earlier chains (known
// in advance) + keys of that digit in earlier tiles of the same chain (look-
// back) + rank inside the tile.  Tiles of different chains are dealt out
// interleaved, so a tile's predecessor in its chain started several tiles
// earlier and has usually published its inclusive count by the time the tile
// looks back.  Each chain is dealt to one of 8 ticket queues (one per XCD,
// picked by block index), so that the neighbouring tiles of a chain, whose
// output runs share cache lines, write through the same L2; a workgroup whose
// queue is empty takes a ticket from another one.
//
// Kernels per sort: k_os_init, k_os_count (one read: identity test, per-chunk
// digit counts, joint histograms), k_os_reduce (column sums and chunk
// prefixes), k_os_plan (round plan, digit starts, chains, ticket tables), then
// one k_onesweep per round.
#pragma once

#include "lsd_kernels.h"

namespace rsort {
namespace {

constexpr uint32_t kChainBits = 4;                    // top bits of the previous digit
constexpr uint32_t kJointChains = 1u << kChainBits;   // 16
constexpr uint32_t kJointBins = kJointChains * R;     // 4096 per round
constexpr uint32_t kQueues = 8;                       // ticket queues (XCDs)
constexpr uint32_t kQueueStride = 32;                 // words between ticket counters
// Chunk chains dealt together in one queue (0: all of the queue's chains).
// More chains in flight shorten the look-back walks but space out the tiles
// of a chain, whose output runs share cache lines, beyond what the L2 merges:
// measured at 2^27 keys (first round, chunk chains) 233 us per round without
// look-back at 4 or 8 chains, 244 at 16; with look-back 300 us at 8, 324 at
// 16, 377 at 32, 385 with all 64.
#ifndef RSORT_OS_CHUNK_GROUP
#define RSORT_OS_CHUNK_GROUP 8
#endif
constexpr int kOsCountWG = 512;
constexpr int kOsReduceWG = 1024;
constexpr int kOsPlanWG = 1024;
constexpr uint32_t kOsMaxChunks = 512;                // chunks of the counting pass
constexpr uint32_t kOsMinChunkTiles = 8;
constexpr int kOsMaxJoint = 3;                        // 32-bit keys: rounds 1..3
constexpr uint32_t kNoRow = 0xFFFFFFFFu;

enum ChainKind : uint32_t { kChainChunk = 0, kChainJoint = 1, kChainSingle = 2 };

// Per round, written by k_os_plan.
struct OsRound {
    uint32_t kind;
    uint32_t nchains;
    uint32_t ntiles;                 // tickets of the round
    uint32_t qoff[kQueues + 1];      // ticket-table offsets of the queues
};

struct OsArgs {
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
    const RoundPlan* plan;
    const OsRound* rinfo;      // [round]
    const uint4* tt;           // this round's ticket table {start, keys, row, chain}
    const uint32_t* row0;      // this round's first row per chain (chain table)
    const uint32_t* cb_chunk;  // this round's chain bases for chunk chains [chain][256]
    const uint32_t* cb_joint;  // this round's chain bases for joint / single chains [chain][256]
    const uint32_t* bases;     // [round][256] digit starts
    uint32_t* state;           // [2][maxrows][256] look-back words
    uint32_t maxrows;
    uint32_t* tick;            // this round's kQueues counters (kQueueStride apart)
    uint32_t* err;
};

// Workspace sizes that depend only on n and the key type.
struct OsShape {
    uint32_t nchunks;       // chunks of the counting pass (= chunk chains)
    uint32_t chunk_keys;    // keys per chunk (a multiple of the tile)
    uint32_t roww;          // words per chunk row
    uint32_t maxrows;       // upper bound of the tiles of a round
    uint32_t cmax;          // upper bound of the chains of a round
};

// ---------------------------------------------------------------------------
// k_os_init: zero the identity words and the ticket counters.
__global__ void k_os_init(uint32_t* mixed, uint32_t mixed_words, uint32_t* tick, uint32_t tick_words)
{
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = g; i < mixed_words; i += stride) mixed[i] = 0;
    for (uint32_t i = g; i < tick_words; i += stride) tick[i] = 0;
}

// Adds c to h[bin] for every valid lane; when every lane of the wave holds the
// same bin one lane adds the lane count (same-address LDS atomics of a wave
// are serialised).
__device__ __forceinline__ void lds_count(uint32_t* h, uint32_t bin, bool valid)
{
    const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)bin);
    const uint64_t same = __builtin_amdgcn_ballot_w64(valid && bin == b0);
    const uint64_t act = __builtin_amdgcn_ballot_w64(valid);
    if (same == act) {
        if (act && (threadIdx.x & 63) == (uint32_t)(__ffsll((unsigned long long)act) - 1))
            atomicAdd(&h[b0], (uint32_t)__popcll(act));
    } else if (valid) {
        atomicAdd(&h[bin], 1u);
    }
}

// ---------------------------------------------------------------------------
// k_os_count: workgroup w reads chunk w = [w * chunk, (w + 1) * chunk) once.
// Row w of `rows` (roww words) receives
//   [d * 256 + v]                      keys of digit d = v in the chunk, d < nr
//   [nr * 256 + (d - 1) * 4096 + i]    joint counts of round d >= 1, bin i =
//                                      digit d << 4 | top 4 bits of digit d - 1
// The same read ORs every key's difference from the first key into the
// identity words (as k_count does for the counted rounds) and zeroes a slice
// of the look-back words of the first round.
template <typename K>
__global__ __launch_bounds__(kOsCountWG) void k_os_count(const K* __restrict__ keys, uint32_t n,
                                                         uint32_t chunk, uint32_t begin_bit,
                                                         uint32_t end_bit, uint32_t nr,
                                                         uint32_t* rows, uint32_t roww,
                                                         uint32_t* mixed, uint32_t* state0,
                                                         uint32_t state_words)
{
    static_assert(sizeof(K) == 4, "joint histograms of 32-bit keys");
    constexpr int VEC = 4;       // keys per 16-byte load
    constexpr int ITEMS = 16;    // keys per thread and step
    constexpr uint32_t STEP = kOsCountWG * ITEMS;
    __shared__ uint32_t h0[R * 8];                       // digit 0, 8 columns by lane
    __shared__ uint32_t hj[kOsMaxJoint * kJointBins];    // joint counts of rounds 1..3
    __shared__ uint32_t mix_s[2];
    const uint32_t tid = threadIdx.x;
    const uint32_t w = blockIdx.x;
    for (uint32_t i = tid; i < R * 8; i += kOsCountWG) h0[i] = 0;
    for (uint32_t i = tid; i < (nr - 1) * kJointBins; i += kOsCountWG) hj[i] = 0;
    if (tid < 2) mix_s[tid] = 0;

    // this workgroup's slice of the first round's look-back words
    {
        const uint32_t per = (state_words / 4 + gridDim.x - 1) / gridDim.x;
        uint4* s4 = (uint4*)state0;
        const uint32_t lo = w * per, hi = min(state_words / 4, lo + per);
        for (uint32_t i = lo + tid; i < hi; i += kOsCountWG) s4[i] = make_uint4(0, 0, 0, 0);
    }
    __syncthreads();

    const DigitSet ds = digit_set(begin_bit, end_bit);
    uint32_t jshift[kOsMaxJoint], jmask[kOsMaxJoint];
#pragma unroll
    for (int d = 1; d <= kOsMaxJoint; ++d) {
        jshift[d - 1] = ds.shift[d] - kChainBits;
        jmask[d - 1] = (ds.mask[d] << kChainBits) | (kJointChains - 1);
    }
    const uint32_t col = tid & 7;
    const K ref = keys[0];
    K acc = 0;
    const uint32_t c0 = w * chunk;
    const uint32_t c1 = min(n, c0 + chunk);

    auto count_key = [&](K k, bool valid) {
        if (valid) acc |= k ^ ref;
        if (valid) atomicAdd(&h0[digit_of(k, ds.shift[0], ds.mask[0]) * 8 + col], 1u);
#pragma unroll
        for (int d = 0; d < kOsMaxJoint; ++d)
            if ((uint32_t)d + 1 < nr)
                lds_count(&hj[d * kJointBins], ((uint32_t)k >> jshift[d]) & jmask[d], valid);
    };

    typedef uint32_t v4 __attribute__((ext_vector_type(4)));
    const bool aligned = (((uintptr_t)keys) & 15) == 0;
    for (uint32_t s = c0; s < c1; s += STEP) {
        if (aligned && s + STEP <= c1) {
            K k[ITEMS];
#pragma unroll
            for (int q = 0; q < ITEMS / VEC; ++q) {
                const v4 x = __builtin_nontemporal_load(&((const v4*)(keys + s))[q * kOsCountWG + tid]);
#pragma unroll
                for (int e = 0; e < VEC; ++e) k[q * VEC + e] = x[e];
            }
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) count_key(k[i], true);
        } else {
            K k[ITEMS];
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t o = s + i * kOsCountWG + tid;
                k[i] = o < c1 ? keys[o] : K(0);
            }
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) count_key(k[i], s + i * kOsCountWG + tid < c1);
        }
    }
    {
        uint32_t lo = (uint32_t)acc;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) lo |= __shfl_xor(lo, o, 64);
        if ((tid & 63) == 0 && lo) atomicOr(&mix_s[0], lo);
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t* mw = &mixed[(w % kMixSlots) * kMixStride];
        const uint32_t mine = mix_s[0];
        if (mine & ~ld_agent(mw)) atomicOr(mw, mine);
    }
    uint32_t* row = rows + (size_t)w * roww;
    if (tid < R) {
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) s += h0[tid * 8 + ((q + tid) & 7)];
        row[tid] = s;
        for (uint32_t d = 1; d < nr; ++d) {
            uint32_t t = 0;
#pragma unroll
            for (uint32_t c = 0; c < kJointChains; ++c) t += hj[(d - 1) * kJointBins + tid * kJointChains + c];
            row[d * R + tid] = t;
        }
    }
    for (uint32_t i = tid; i < (nr - 1) * kJointBins; i += kOsCountWG) row[nr * R + i] = hj[i];
}

// ---------------------------------------------------------------------------
// k_os_reduce: column sums over the chunk rows.  Columns below nr * 256 (the
// per-chunk digit counts) also get their exclusive prefix over chunks:
// cbx[d][w][v] = keys of digit v in chunks before w; tot[d][v] = all keys of
// digit v.  The joint columns are summed into J[d][i] (d >= 1).
// Workgroup = 64 columns; 16 row groups of 64 threads each.
__global__ __launch_bounds__(kOsReduceWG) void k_os_reduce(const uint32_t* rows, uint32_t nchunks,
                                                           uint32_t roww, uint32_t nr,
                                                           uint32_t* cbx, uint32_t* tot, uint32_t* J)
{
    constexpr int NRG = kOsReduceWG / 64;
    __shared__ uint32_t part[NRG][64];
    const uint32_t tid = threadIdx.x;
    const uint32_t cl = tid & 63, rg = tid >> 6;
    const uint32_t colx = blockIdx.x * 64 + cl;
    const bool have = colx < roww;
    const uint32_t poscols = nr * R;
    const uint32_t per = (nchunks + NRG - 1) / NRG;
    const uint32_t r0 = min(nchunks, rg * per), r1 = min(nchunks, r0 + per);
    uint32_t s = 0;
    {
        uint32_t r = r0;
        for (; r + 8 <= r1; r += 8) {
            uint32_t x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = have ? rows[(size_t)(r + u) * roww + colx] : 0u;
#pragma unroll
            for (int u = 0; u < 8; ++u) s += x[u];
        }
        for (; r < r1; ++r) s += have ? rows[(size_t)r * roww + colx] : 0u;
    }
    part[rg][cl] = s;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int g = 0; g < NRG; ++g) {
        const uint32_t p = part[g][cl];
        if ((uint32_t)g < rg) before += p;
        all += p;
    }
    if (!have) return;
    if (colx < poscols) {
        const uint32_t d = colx / R, v = colx % R;
        if (rg == 0) tot[colx] = all;
        uint32_t run = before;
        uint32_t r = r0;
        for (; r + 8 <= r1; r += 8) {
            uint32_t x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = rows[(size_t)(r + u) * roww + colx];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                cbx[((size_t)d * nchunks + r + u) * R + v] = run;
                run += x[u];
            }
        }
        for (; r < r1; ++r) {
            cbx[((size_t)d * nchunks + r) * R + v] = run;
            run += rows[(size_t)r * roww + colx];
        }
    } else if (rg == 0) {
        J[kJointBins + (colx - poscols)] = all;   // J[d] for d >= 1
    }
}

// ---------------------------------------------------------------------------
// k_os_plan (one workgroup): identity rounds -> round plan; digit starts; for
// every round that runs, its chains (start, tiles, first row, queue) and their
// bases.  k_os_tickets then writes the ticket tables.
//
// Ticket order: queue x holds a contiguous range of chains, in groups of A
// consecutive chains (by default A = all of the queue's chains); groups are dealt one after another, and the tiles of a
// group in the order of their fractional position j / m_c inside their chain
// (ties by chain), so that every chain advances at the same pace and a tile's
// predecessor always has an earlier ticket of the same queue.

// Exclusive sum over the kOsPlanWG threads of the workgroup; wsum holds one
// word per wave.  Every thread must call it.
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t x, uint32_t* wsum)
{
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t incl = wave_inclusive_sum(x);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t pre = 0;
    for (uint32_t w = 0; w < wave; ++w) pre += wsum[w];
    __syncthreads();
    return pre + incl - x;
}

__global__ __launch_bounds__(kOsPlanWG) void k_os_plan(
    const uint32_t* mixed, uint32_t nr, uint32_t begin_bit, uint32_t end_bit, int alias, uint32_t n,
    uint32_t tile, OsShape sh, RoundPlan* plan, const uint32_t* tot, const uint32_t* J,
    uint32_t* bases, uint32_t* jx, OsRound* rinfo, uint32_t* chain_tab)
{
    __shared__ RoundPlan pl_s[kMaxRounds + 1];
    __shared__ uint32_t jl_s[kJointBins];      // joint counts of one round, [digit][chain]
    __shared__ uint32_t len_s[kJointChains];
    __shared__ uint32_t r0_s[kOsMaxChunks + 1];
    __shared__ uint32_t wsum[kOsPlanWG / 64];
    const uint32_t tid = threadIdx.x;
    if (tid < 64) {
        uint32_t mlo = mixed[tid * kMixStride];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) mlo |= __shfl_xor(mlo, o, 64);
        if (tid == 0) {
            int identity[kMaxRounds];
            for (uint32_t d = 0; d < nr; ++d) {
                const uint32_t lo = begin_bit + 8u * d;
                const uint32_t wd = min(8u, end_bit - lo);
                identity[d] = ((mlo >> lo) & ((1u << wd) - 1u)) == 0;
            }
            plan_rounds(identity, nr, alias, plan);
            for (uint32_t d = 0; d <= (uint32_t)kMaxRounds; ++d) pl_s[d] = plan[d];
        }
    }
    // digit starts of every round (exclusive scan over the 256 digits)
    for (uint32_t d = 0; d < nr; ++d) {
        const uint32_t x = tid < R ? tot[d * R + tid] : 0u;
        const uint32_t ex = block_exclusive_sum(x, wsum);
        if (tid < R) bases[d * R + tid] = ex;
    }
    __syncthreads();

    for (uint32_t d = 0; d < nr; ++d) {
        const RoundPlan pl = pl_s[d];
        if (pl.exec != 1) continue;
        uint32_t kind, C;
        if (pl.ord == 0) { kind = kChainChunk; C = sh.nchunks; }
        else if (d > 0 && pl_s[d - 1].exec == 1) { kind = kChainJoint; C = kJointChains; }
        else { kind = kChainSingle; C = 1; }
        if (kind == kChainJoint) {
            for (uint32_t i = tid; i < kJointBins; i += kOsPlanWG) jl_s[i] = J[(size_t)d * kJointBins + i];
            __syncthreads();
            // chain lengths; chain bases jx[d][c][v] = keys of digit v in chains before c
            if (tid < kJointChains) {
                uint32_t l = 0;
                for (uint32_t v = 0; v < R; ++v) l += jl_s[v * kJointChains + tid];
                len_s[tid] = l;
            }
            if (tid < R) {
                uint32_t run = 0;
#pragma unroll
                for (uint32_t c = 0; c < kJointChains; ++c) {
                    jx[((size_t)d * kJointChains + c) * R + tid] = run;
                    run += jl_s[tid * kJointChains + c];
                }
            }
            __syncthreads();
        } else if (kind == kChainSingle) {
            if (tid < R) jx[(size_t)d * kJointChains * R + tid] = 0;
        }
        // chain starts, tiles and first rows (block scans over the chains)
        const uint32_t c = tid;
        uint32_t len = 0;
        if (c < C) {
            if (kind == kChainChunk) len = min(sh.chunk_keys, n - c * sh.chunk_keys);
            else if (kind == kChainJoint) len = len_s[c];
            else len = n;
        }
        const uint32_t m = (len + tile - 1) / tile;
        const uint32_t ls = block_exclusive_sum(len, wsum);
        const uint32_t ms = block_exclusive_sum(m, wsum);
        uint32_t* ch_start = chain_tab + (size_t)(3 * d + 0) * sh.cmax;
        uint32_t* ch_tiles = chain_tab + (size_t)(3 * d + 1) * sh.cmax;
        uint32_t* ch_row0 = chain_tab + (size_t)(3 * d + 2) * sh.cmax;
        if (c < C) {
            ch_start[c] = ls;
            ch_tiles[c] = m;
            ch_row0[c] = ms;
            r0_s[c] = ms;
        }
        if (c == C - 1) r0_s[C] = ms + m;
        __syncthreads();
        if (tid == 0) {
            OsRound ri;
            ri.kind = kind;
            ri.nchains = C;
            ri.ntiles = r0_s[C];
            // queue x holds chains [ceil(x C / 8), ceil((x + 1) C / 8)) (the single
            // chain goes to queue 0)
            for (uint32_t x = 0; x <= kQueues; ++x) {
                const uint32_t qc = kind == kChainSingle ? (x == 0 ? 0u : 1u) : (x * C + kQueues - 1) / kQueues;
                ri.qoff[x] = r0_s[qc];
            }
            rinfo[d] = ri;
        }
        __syncthreads();
    }
}

// Rank of tile j of chain c among the tiles of chains [g0, g1) ordered by
// (j' / m_i, i): j plus, for every other chain i, its tiles j' with j' m_c <=
// j m_i (i < c) or j' m_c < j m_i (i > c).
__device__ __forceinline__ uint32_t os_rank_in_group(const uint32_t* m, uint32_t g0, uint32_t g1,
                                                     uint32_t c, uint32_t j)
{
    const uint32_t mc = m[c];
    uint32_t r = j;
    for (uint32_t i = g0; i < g1; ++i) {
        if (i == c) continue;
        const uint32_t mi = m[i];
        const uint64_t num = (uint64_t)j * mi;
        // floor(num / mc) from a double estimate, corrected (num < 2^53)
        uint64_t f = (uint64_t)((double)num / (double)mc);
        while (f * mc > num) --f;
        while ((f + 1) * mc <= num) ++f;
        const uint64_t k = i < c ? f + 1 : f + (f * mc != num ? 1u : 0u);
        r += (uint32_t)min<uint64_t>(mi, k);
    }
    return r;
}

// k_os_tickets: ticket table of round blockIdx.y, one row per thread.
constexpr int kOsTicketWG = 256;
__global__ __launch_bounds__(kOsTicketWG) void k_os_tickets(const RoundPlan* plan, const OsRound* rinfo,
                                                            const uint32_t* chain_tab, uint32_t cmax,
                                                            uint32_t maxrows, uint32_t n, uint32_t tile,
                                                            uint4* tt)
{
    __shared__ uint32_t st_s[kOsMaxChunks];
    __shared__ uint32_t m_s[kOsMaxChunks];
    __shared__ uint32_t r0_s[kOsMaxChunks + 1];
    const uint32_t d = blockIdx.y;
    if (plan[d].exec != 1) return;
    const OsRound ri = rinfo[d];
    const uint32_t C = ri.nchains;
    const uint32_t tid = threadIdx.x;
    if (blockIdx.x * kOsTicketWG >= ri.ntiles) return;
    for (uint32_t c = tid; c < C; c += kOsTicketWG) {
        st_s[c] = chain_tab[(size_t)(3 * d + 0) * cmax + c];
        m_s[c] = chain_tab[(size_t)(3 * d + 1) * cmax + c];
        r0_s[c] = chain_tab[(size_t)(3 * d + 2) * cmax + c];
    }
    if (tid == 0) r0_s[C] = ri.ntiles;
    __syncthreads();
    const uint32_t row = blockIdx.x * kOsTicketWG + tid;
    if (row >= ri.ntiles) return;
    // chain of this row: last c with r0_s[c] <= row (never an empty chain)
    uint32_t lo = 0, hi = C - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (r0_s[mid] <= row) lo = mid; else hi = mid - 1;
    }
    const uint32_t c = lo;
    const uint32_t j = row - r0_s[c];
    const uint32_t x = ri.kind == kChainSingle ? 0u : (uint32_t)(((uint64_t)c * kQueues) / C);
    const uint32_t qa = ri.kind == kChainSingle ? 0u : (x * C + kQueues - 1) / kQueues;
    const uint32_t qb = ri.kind == kChainSingle ? 1u : ((x + 1) * C + kQueues - 1) / kQueues;
    const uint32_t A = ri.kind == kChainChunk && RSORT_OS_CHUNK_GROUP ? RSORT_OS_CHUNK_GROUP : (qb - qa);
    const uint32_t g0 = qa + ((c - qa) / A) * A;
    const uint32_t g1 = min(qb, g0 + A);
    const uint32_t ticket = ri.qoff[x] + (r0_s[g0] - r0_s[qa]) + os_rank_in_group(m_s, g0, g1, c, j);
    const uint32_t start = st_s[c] + j * tile;
    const uint32_t end = c + 1 < C ? st_s[c + 1] : n;
    if (ticket < maxrows) tt[(size_t)d * maxrows + ticket] = make_uint4(start, min(tile, end - start), row, c);
}

// ---------------------------------------------------------------------------
// k_onesweep: one stable count-sort round of one tile, with the tile's output
// offsets found by look-back inside its chain.  The ranking, staging and
// writing are those of k_scatter (count first, 32-lane ranking groups with
// 64-bit {lane set, count} slots, tile staged in digit order in LDS).
//
//   ticket   thread 0 takes a ticket from its queue (or another) -> tile
//   load     the tile's keys (and payloads)
//   count    per-group digit counts in LDS
//   publish  digit thread v publishes the tile's count of v (its inclusive
//            count at once when it is the chain's first tile), then the slot
//            bases are laid out
//   rank     stable rank in the tile
//   stage    digit thread v reads its nearest predecessor's word; the tile is
//            staged in digit order in LDS while that read is in flight
//   resolve  fold the predecessors' words nearest first (counts added, the
//            first inclusive count ends the walk, a word not yet published is
//            polled again, further words 4 at a time), publish the inclusive
//            count, output offsets
//   write    consecutive threads write consecutive keys
#ifndef RSORT_OS_WAVES_PER_EU
#define RSORT_OS_WAVES_PER_EU 8
#endif
#ifndef RSORT_OS_WAVES_PER_EU_KV
#define RSORT_OS_WAVES_PER_EU_KV 4
#endif
#ifndef RSORT_OS_KV_LDS_RESERVE
#define RSORT_OS_KV_LDS_RESERVE 6144
#endif
constexpr int kOsWindow = 4;   // predecessor words per look-back step after the first

template <typename K, bool KV, int WG, int ITEMS>
__global__ __launch_bounds__(WG, KV ? RSORT_OS_WAVES_PER_EU_KV : RSORT_OS_WAVES_PER_EU) void k_onesweep(OsArgs a)
{
    constexpr int G = 32;
    constexpr int NG = WG / G;
    constexpr uint32_t TILE = (uint32_t)WG * ITEMS;
    static_assert(WG == 2 * (int)R, "two look-back halves of 256 digit threads");
    static_assert(TILE * sizeof(K) >= NG * R * 8, "staging must cover the slots");
    struct Smem {
        union {
            uint2 slot[NG][R];           // {lane set, count} (swapped for digits >= 128)
            uint32_t words[2 * NG * R];  // counts first at words[NG R + g R + d]
            K keys[TILE];
            uint32_t vals[TILE];
        } u;
        uint32_t goff[R];
        uint32_t wsum[4];
        uint4 e;
        uint32_t reserve[KV ? RSORT_OS_KV_LDS_RESERVE : 1];
    };
    __shared__ Smem sm;

    const RoundPlan pl = a.plan[a.round];
    if (!pl.exec) return;
    const uint32_t tid = threadIdx.x;
    const K* src = pick<K>(pl.src, (const K*)a.keys_in, (K*)a.keys_out, (K*)a.keys_tmp);
    const uint32_t* vsrc = KV ? pick<uint32_t>(pl.src, a.vals_in, a.vals_out, a.vals_tmp) : nullptr;
    K* dst = pick<K>(pl.dst, (const K*)a.keys_in, (K*)a.keys_out, (K*)a.keys_tmp);
    uint32_t* vdst = KV ? pick<uint32_t>(pl.dst, a.vals_in, a.vals_out, a.vals_tmp) : nullptr;
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

    uint32_t* st = a.state + (size_t)(pl.ord & 1) * a.maxrows * R;
    {
        // the next round's look-back words (written two rounds ago) start at zero
        uint4* nx = (uint4*)(a.state + (size_t)((pl.ord + 1) & 1) * a.maxrows * R);
        for (uint32_t r = blockIdx.x; r < a.maxrows; r += gridDim.x)
            if (tid < R / 4) nx[(size_t)r * (R / 4) + tid] = make_uint4(0, 0, 0, 0);
    }
    if (tid == 0) {
        const OsRound& ri = a.rinfo[a.round];
        uint4 e = make_uint4(0, 0, kNoRow, 0);
        const uint32_t x0 = blockIdx.x & (kQueues - 1);
        for (uint32_t q = 0; q < kQueues; ++q) {
            const uint32_t x = (x0 + q) & (kQueues - 1);
            const uint32_t qlen = ri.qoff[x + 1] - ri.qoff[x];
            if (qlen == 0) continue;
            uint32_t* ctr = &a.tick[x * kQueueStride];
            if (q > 0 && ld_agent(ctr) >= qlen) continue;   // exhausted: no atomic
            const uint32_t t = atomicAdd(ctr, 1u);
            if (t < qlen) {
                e = a.tt[ri.qoff[x] + t];
                break;
            }
        }
        sm.e = e;
    }
    constexpr uint32_t slot_u4 = NG * R * 8 / 16;
    for (uint32_t i = tid; i < slot_u4; i += WG) ((uint4*)&sm.u)[i] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    const uint4 e = sm.e;
    if (e.z == kNoRow) return;
    if (e.x >= a.n || e.y == 0 || e.y > TILE || e.y > a.n - e.x || e.z >= a.maxrows ||
        e.w >= a.rinfo[a.round].nchains) {
        if (tid == 0) atomicOr(a.err, (uint32_t)kErrBadPlan);   // a malformed ticket entry
        return;
    }
    const uint32_t base = e.x, lim = e.y, row = e.z, chain = e.w;
    const uint32_t jpre = row - a.row0[chain];   // predecessors in the chain

    const uint32_t lane = tid & 63;
    const uint32_t wave = tid >> 6;
    const uint32_t grp = tid / G;
    const uint32_t gl = tid % G;
    const uint32_t hofs = grp * ITEMS * G + gl;
    K k[ITEMS];
    uint32_t v[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t o = hofs + i * G;
        k[i] = o < lim ? src[base + o] : K(0);
        if (KV) v[i] = o < lim ? vsrc[base + o] : 0u;
    }
    // chain base and digit start of digit thread tid (latency hidden by the count)
    const uint32_t* cb = (a.rinfo[a.round].kind == kChainChunk ? a.cb_chunk : a.cb_joint) + (size_t)chain * R;
    uint32_t gbase = 0;
    if (tid < R) gbase = cb[tid] + a.bases[a.round * R + tid];

    // count: per-group digit counts
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const bool ok = hofs + i * G < lim;
        const uint32_t d = digit_of(k[i], a.shift, a.mask);
        if (wave_one_digit(ok, d)) {
            if (gl == 0) atomicAdd(&sm.u.words[NG * R + grp * R + d], 32u);
            continue;
        }
        if (ok) atomicAdd(&sm.u.words[NG * R + grp * R + d], 1u);
    }
    __syncthreads();

    // publish, look-back loads, slot bases
    uint32_t total = 0, run = 0;
    if (tid < R) {
#pragma unroll
        for (int g = 0; g < NG; ++g) total += sm.u.words[NG * R + g * R + tid];
        st_agent(&st[(size_t)row * R + tid], (jpre == 0 ? kFlagPrefix : kFlagAggregate) | total);
        const uint32_t incl = wave_inclusive_sum(total);
        if (lane == 63) sm.wsum[wave] = incl;
        run = incl - total;
    }
    __syncthreads();
    uint32_t hi[NG / 2];
    uint32_t tstart = 0;   // tile-local start of digit tid
    if (tid < R) {
        for (uint32_t w = 0; w < wave; ++w) run += sm.wsum[w];
        tstart = run;
#pragma unroll
        for (int g = 0; g < NG / 2; ++g) {
            const uint32_t c = sm.u.words[NG * R + g * R + tid];
            sm.u.slot[g][tid] = (tid & 128u) ? make_uint2(run, 0u) : make_uint2(0u, run);
            run += c;
        }
#pragma unroll
        for (int g = NG / 2; g < NG; ++g) hi[g - NG / 2] = sm.u.words[NG * R + g * R + tid];
    }
    __syncthreads();
    if (tid < R) {
#pragma unroll
        for (int g = NG / 2; g < NG; ++g) {
            sm.u.slot[g][tid] = (tid & 128u) ? make_uint2(run, 0u) : make_uint2(0u, run);
            run += hi[g - NG / 2];
        }
    }
    __syncthreads();

    // rank
    uint32_t pos[ITEMS];
    {
        const uint32_t bit = 1u << gl;
        uint2* sl = sm.u.slot[grp];
        const uint32_t lowsel = lane < 32 ? ~0u : 0u;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const bool ok = hofs + i * G < lim;
            const uint32_t d = digit_of(k[i], a.shift, a.mask);
            const uint32_t cs = (d & 128u) ? 0u : 32u;
            if (wave_one_digit(ok, d)) {
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
    }

    // the nearest predecessor's word, read after the ranking (predecessors get
    // that long to publish) and folded after the staging
    uint32_t w0 = 0;
    if (tid < R && jpre > 0) w0 = ld_agent(&st[(size_t)(row - 1) * R + tid]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if (hofs + i * G < lim) sm.u.keys[pos[i]] = k[i];

    // resolve the look-back: fold predecessor words nearest first -- counts
    // are added and passed over, the first inclusive count ends the walk, a
    // word not yet published is polled again
    if (tid < R) {
        uint32_t excl = 0;
        if (jpre > 0) {
            uint32_t q = 0;   // next predecessor to fold
            bool done = false;
            {
                const uint32_t f = w0 >> kFlagShift;
                if (f != 0) {
                    excl = w0 & kCountMask;
                    q = 1;
                    done = f == (kFlagPrefix >> kFlagShift);
                }
            }
            uint32_t spins = 0;
            while (!done) {
                // q < jpre here: the chain's first tile publishes an inclusive count
                uint32_t w4[kOsWindow];
#pragma unroll
                for (int i = 0; i < kOsWindow; ++i)
                    w4[i] = q + i < jpre ? ld_agent(&st[(size_t)(row - 1 - q - i) * R + tid]) : 0u;
                uint32_t used = 0;
                bool gap = false;
#pragma unroll
                for (int i = 0; i < kOsWindow; ++i) {
                    if (!done && !gap && q + i < jpre) {
                        const uint32_t f = w4[i] >> kFlagShift;
                        if (f == 0) {
                            gap = true;
                        } else {
                            excl += w4[i] & kCountMask;
                            used = i + 1;
                            done = f == (kFlagPrefix >> kFlagShift);
                        }
                    }
                }
                q += used;
                if (!done && used == 0) {
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
            st_agent(&st[(size_t)row * R + tid], kFlagPrefix | ((excl + total) & kCountMask));
        }
        sm.goff[tid] = gbase + excl - tstart;
    }
    __syncthreads();

    // write: consecutive threads store consecutive keys of the staged tile
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
            if (hofs + i * G < lim) sm.u.vals[pos[i]] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = i * WG + tid;
            if (p < lim && outi[i] < a.n) vdst[outi[i]] = sm.u.vals[p];
        }
    }
}

}  // namespace
}  // namespace rsort
