// Batched segmented sorting: many independent arrays (CSR segments of one key
// array) sorted in one call, each by the stable LSD radix-2^8 sort of
// arXiv 1808.10292 Section 3.2 (SR4 applied per segment).
//
// Segments are split by size on the host:
//   small (<= 8192 keys): one workgroup sorts the whole segment in LDS --
//           every round is count, bases, rank and restage inside the
//           workgroup, so the segment is read from HBM once and written once
//           (k_seg_small, three tile capacities: 1024, 4096, 8192 keys);
//   large:  split into tiles of 8192 keys that never cross a segment; each
//           round is the plain sort's k_count and k_scatter over the tile list,
//           with k_segscan turning the tile counts of every segment into output
//           starts (one workgroup per segment).
// The size split is a parameter the tuner (rsort_segmented_tune) chooses.
#include <algorithm>
#include <cstring>
#include <vector>

#include "lsd_kernels.h"
#include "tile_sort.h"

namespace rsort {
namespace {

// ---------------------------------------------------------------------------
// k_seg_small: one workgroup sorts segment blockIdx.x of the list in LDS, one
// tile_round per 8-bit digit (whole keys), then writes it back once.
template <typename K, bool KV, int WG, int ITEMS>
__global__ __launch_bounds__(WG) void k_seg_small(const K* __restrict__ keys_in, K* keys_out,
                                                  const uint32_t* __restrict__ vals_in,
                                                  uint32_t* vals_out, const uint2* segs,
                                                  uint32_t nrounds)
{
    __shared__ TileSmem<K, KV, WG, ITEMS, true> sm;
    const uint32_t tid = threadIdx.x;
    const uint32_t hofs = (tid >> 5) * ITEMS * 32 + (tid & 31);
    const uint2 seg = segs[blockIdx.x];
    const uint32_t base = seg.x;
    const uint32_t len = seg.y - seg.x;

    K k[ITEMS];
    uint32_t v[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t o = hofs + i * 32;
        k[i] = o < len ? keys_in[base + o] : K(0);
        v[i] = KV && o < len ? vals_in[base + o] : 0u;
    }
    for (uint32_t r = 0; r < nrounds; ++r)
        tile_round<K, KV, WG, ITEMS>(sm, k, v, len, 8u * r, 0xFFu);
    // write out: each thread holds positions hofs + 32 i in the final order
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t o = hofs + i * 32;
        if (o < len) {
            keys_out[base + o] = k[i];
            if (KV) vals_out[base + o] = v[i];
        }
    }
}

// k_segscan: one workgroup per large segment {first tile, end tile, first key}.
// Thread v sums its digit over the segment's tiles, the 256 totals are scanned
// into the digit starts inside the segment, and every tile count is replaced
// by the output index of the tile's first key of digit v.
__global__ __launch_bounds__(R) void k_segscan(RoundArgs a, const uint4* lsegs)
{
    __shared__ uint32_t wsum[4];
    const RoundPlan pl = a.seg_plan ? a.seg_plan[(size_t)blockIdx.x * (kMaxRounds + 1) + a.round]
                                    : a.plan[a.round];
    if (pl.exec != 1) return;
    const uint4 sg = lsegs[blockIdx.x];
    const uint32_t v = threadIdx.x;
    uint32_t* col = a.counts + v;
    // the column in batches of B tiles, each batch's loads issued together
    constexpr uint32_t B = 16;
    uint32_t total = 0;
    for (uint32_t t = sg.x; t < sg.y; t += B) {
        uint32_t c[B];
#pragma unroll
        for (uint32_t j = 0; j < B; ++j) c[j] = t + j < sg.y ? col[(size_t)(t + j) * R] : 0u;
#pragma unroll
        for (uint32_t j = 0; j < B; ++j) total += c[j];
    }
    const uint32_t lane = v & 63, wave = v >> 6;
    const uint32_t incl = wave_inclusive_sum(total);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t run = sg.z + incl - total;
    for (uint32_t w = 0; w < wave; ++w) run += wsum[w];
    for (uint32_t t = sg.x; t < sg.y; t += B) {
        uint32_t c[B];
#pragma unroll
        for (uint32_t j = 0; j < B; ++j) c[j] = t + j < sg.y ? col[(size_t)(t + j) * R] : 0u;
#pragma unroll
        for (uint32_t j = 0; j < B; ++j)
            if (t + j < sg.y) {
                col[(size_t)(t + j) * R] = run;
                run += c[j];
            }
    }
}

// Zero `words` words (the segments' identity words before round 0's count).
__global__ void k_zero_words(uint32_t* words, uint32_t count)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        words[i] = 0;
}

// k_seg_plans: thread s turns segment s's identity words (the OR of every key's
// difference from the segment's first key, from round 0's count) into its
// round plan: a round whose digit bits are zero there is the identity for the
// segment and is skipped, with the rounds that run alternating between the
// temporary and the output so that the last one writes the output.  With a
// device round count of 0 (dev_rounds) the caller writes the output itself:
// no round runs and nothing is copied.
__global__ void k_seg_plans(const uint32_t* seg_or, uint32_t nseg, uint32_t nrounds, int alias,
                            RoundPlan* seg_plan, const uint32_t* dev_rounds)
{
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    if (dev_rounds && *dev_rounds == 0) {
        RoundPlan* pl = seg_plan + (size_t)s * (kMaxRounds + 1);
        for (uint32_t d = 0; d < nrounds; ++d) pl[d] = RoundPlan{0, -1, 0, -1};
        pl[kMaxRounds] = RoundPlan{0, 0, 0, 2};
        return;
    }
    const uint64_t mx = (uint64_t)seg_or[2 * s] | ((uint64_t)seg_or[2 * s + 1] << 32);
    int identity[kMaxRounds];
    for (uint32_t d = 0; d < nrounds; ++d) identity[d] = ((mx >> (8u * d)) & 0xFFull) == 0;
    plan_rounds(identity, nrounds, alias, seg_plan + (size_t)s * (kMaxRounds + 1));
}

// Small-segment kernel classes: capacity = WG * ITEMS keys.
struct SmallClass {
    int wg, items;
};
constexpr SmallClass kSmallClasses[3] = {{256, 4}, {512, 8}, {512, 16}};
// Keys per tile of the large path: the tile of the plain sort's round kernels.
uint32_t large_tile(int key_bytes)
{
    return key_bytes == 8 ? R8Config<uint64_t>::WG * R8Config<uint64_t>::ITEMS
                          : R8Config<uint32_t>::WG * R8Config<uint32_t>::ITEMS;
}


// ---------------------------------------------------------------------------
// BTN and OET (Section 2) as whole-segment sorts inside one workgroup, the
// alternatives to the in-LDS radix rounds for small segments (32-bit keys,
// up to 4096 keys).  The P threads are the paper's processors: thread t holds
// the run of segment positions [t R, t R + R) as (key, position) composites,
// sorts it (a register sorting network; the paper sorts the runs by SR4),
// then the runs are ordered as P 'keys':
//   BTN  lg P (lg P + 1) / 2 stages of Batcher's bitonic sorter;
//   OET  P rounds of odd-even transposition;
// where comparing two runs means merging them and giving the lower R
// composites to the lower-indexed thread of the pair (the upper to the
// other).  Composites are unique, so the result is the stable sort; payloads
// are staged in LDS by position and gathered at the end (in place is safe).

__device__ __forceinline__ bool comp_lt(uint32_t a, uint32_t ai, uint32_t b, uint32_t bi)
{
    return a < b || (a == b && ai < bi);
}

// (k[a], x[a]) <= (k[b], x[b]) afterwards.
template <int R>
__device__ __forceinline__ void comp_order(uint32_t (&k)[R], uint32_t (&x)[R], int a, int b)
{
    const bool sw = comp_lt(k[b], x[b], k[a], x[a]);
    const uint32_t ka = k[a], kb = k[b], xa = x[a], xb = x[b];
    k[a] = sw ? kb : ka;
    k[b] = sw ? ka : kb;
    x[a] = sw ? xb : xa;
    x[b] = sw ? xa : xb;
}

// Bitonic sorting network on R registers, ascending.
template <int R>
__device__ __forceinline__ void reg_sort(uint32_t (&k)[R], uint32_t (&x)[R])
{
#pragma unroll
    for (int size = 2; size <= R; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int j = i ^ stride;
                if (j > i) {
                    if ((i & size) == 0) comp_order<R>(k, x, i, j);
                    else comp_order<R>(k, x, j, i);
                }
            }
}

// A bitonic sequence of R registers sorted ascending (half-cleaners).
template <int R>
__device__ __forceinline__ void reg_bitonic_merge(uint32_t (&k)[R], uint32_t (&x)[R])
{
#pragma unroll
    for (int stride = R >> 1; stride > 0; stride >>= 1)
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int j = i ^ stride;
            if (j > i) comp_order<R>(k, x, i, j);
        }
}

template <bool KV, int P, int R, bool OET>
__global__ __launch_bounds__(P) void k_seg_network(const uint32_t* __restrict__ keys_in,
                                                   uint32_t* keys_out,
                                                   const uint32_t* __restrict__ vals_in,
                                                   uint32_t* vals_out, const uint2* segs)
{
    __shared__ uint32_t xk[R][P];   // run exchange, register i of thread t at [i][t]
    __shared__ uint32_t xi[R][P];
    __shared__ uint32_t vst[KV ? P * R : 1];
    const uint2 seg = segs[blockIdx.x];
    const uint32_t base = seg.x, len = seg.y - seg.x;
    if (len == 0) return;
    const uint32_t t = threadIdx.x;
    uint32_t k[R], x[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t u = t * R + i;
        k[i] = u < len ? keys_in[base + u] : 0xFFFFFFFFu;   // padding sorts last: position >= len
        x[i] = u;
    }
    if (KV)
        for (uint32_t u = t; u < len; u += P) vst[u] = vals_in[base + u];
    reg_sort<R>(k, x);
    // run t against run `partner`: keep the lower (or upper) R of the two
    auto merge_split = [&](bool active, uint32_t partner, bool lower) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            xk[i][t] = k[i];
            xi[i][t] = x[i];
        }
        __syncthreads();
        if (active) {
            uint32_t bk[R], bx[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                bk[i] = xk[R - 1 - i][partner];
                bx[i] = xi[R - 1 - i][partner];
            }
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const bool mine = comp_lt(k[i], x[i], bk[i], bx[i]) == lower;
                k[i] = mine ? k[i] : bk[i];
                x[i] = mine ? x[i] : bx[i];
            }
            reg_bitonic_merge<R>(k, x);
        }
        __syncthreads();
    };
    if (!OET) {
        for (uint32_t size = 2; size <= P; size <<= 1)
            for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                const uint32_t partner = t ^ stride;
                const bool asc = (t & size) == 0;
                merge_split(true, partner, (t < partner) == asc);
            }
    } else {
        for (uint32_t r = 0; r < P; ++r) {
            const bool left = (t & 1) == (r & 1);   // pairs (t, t + 1) with t of this round's parity
            const uint32_t partner = left ? t + 1 : t - 1;
            merge_split(left ? t + 1 < P : t > 0, partner, left);
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t u = t * R + i;
        if (u < len) {
            keys_out[base + u] = k[i];
            if (KV) vals_out[base + u] = vst[x[i]];
        }
    }
}

// Small-segment class cls (capacities 1024, 4096, 8192).  small_sort picks
// the in-LDS radix rounds (0), BTN (1) or OET (2); the two networks take
// 32-bit keys in the first two classes, other segments take the radix rounds.
template <typename K, bool KV>
void launch_small(int cls, const void* ki, void* ko, const uint32_t* vi, uint32_t* vo,
                  const uint2* segs, uint32_t nsegs, uint32_t nrounds, hipStream_t s,
                  int small_sort = 0)
{
    if (!nsegs) return;
    if (small_sort != 0 && sizeof(K) == 4 && cls < 2) {
        const uint32_t* k32 = (const uint32_t*)ki;
        uint32_t* o32 = (uint32_t*)ko;
        const bool oet = small_sort == 2;
        if (cls == 0) {
            if (oet) hipLaunchKernelGGL((k_seg_network<KV, 256, 4, true>), dim3(nsegs), dim3(256), 0, s, k32, o32, vi, vo, segs);
            else hipLaunchKernelGGL((k_seg_network<KV, 256, 4, false>), dim3(nsegs), dim3(256), 0, s, k32, o32, vi, vo, segs);
        } else {
            if (oet) hipLaunchKernelGGL((k_seg_network<KV, 512, 8, true>), dim3(nsegs), dim3(512), 0, s, k32, o32, vi, vo, segs);
            else hipLaunchKernelGGL((k_seg_network<KV, 512, 8, false>), dim3(nsegs), dim3(512), 0, s, k32, o32, vi, vo, segs);
        }
        return;
    }
    switch (cls) {
    case 0:
        hipLaunchKernelGGL((k_seg_small<K, KV, 256, 4>), dim3(nsegs), dim3(256), 0, s,
                           (const K*)ki, (K*)ko, vi, vo, segs, nrounds);
        break;
    case 1:
        hipLaunchKernelGGL((k_seg_small<K, KV, 512, 8>), dim3(nsegs), dim3(512), 0, s,
                           (const K*)ki, (K*)ko, vi, vo, segs, nrounds);
        break;
    default:
        hipLaunchKernelGGL((k_seg_small<K, KV, 512, 16>), dim3(nsegs), dim3(512), 0, s,
                           (const K*)ki, (K*)ko, vi, vo, segs, nrounds);
        break;
    }
}

}  // namespace

// Host-side plan: which segments go to which small class, the large tiles and
// the large segments.  Built from host CSR offsets.
uint32_t seg_tile_keys(int key_bytes, int shape)
{
    static const uint32_t wg[kSegTileShapes] = {256, 512, 1024};
    const int s = shape >= 0 && shape < kSegTileShapes ? shape : kSegTileShapeDefault;
    return wg[s] * (key_bytes == 8 ? 8u : 16u);
}

void segmented_plan(const uint64_t* off, size_t nsegs, uint32_t small_max, int key_bytes,
                    SegPlan& P, int tile_shape)
{
    P.tile_shape = tile_shape >= 0 && tile_shape < kSegTileShapes ? tile_shape : kSegTileShapeDefault;
    P.small[0].clear();
    P.small[1].clear();
    P.small[2].clear();
    P.tiles.clear();
    P.lsegs.clear();
    P.tile_seg.clear();
    const uint32_t tile = seg_tile_keys(key_bytes, P.tile_shape);
    for (size_t s = 0; s < nsegs; ++s) {
        const uint32_t lo = (uint32_t)off[s], hi = (uint32_t)off[s + 1];
        const uint32_t len = hi - lo;
        if (len == 0) continue;
        if (len <= small_max) {
            int cls = 2;
            for (int c = 0; c < 3; ++c)
                if (len <= (uint32_t)(kSmallClasses[c].wg * kSmallClasses[c].items)) { cls = c; break; }
            P.small[cls].push_back(make_uint2(lo, hi));
        } else {
            const uint32_t t0 = (uint32_t)P.tiles.size();
            for (uint32_t b = lo; b < hi; b += tile) {
                P.tiles.push_back(make_uint2(b, std::min(hi, b + tile)));
                P.tile_seg.push_back((uint32_t)P.lsegs.size());
            }
            P.lsegs.push_back(make_uint4(t0, (uint32_t)P.tiles.size(), lo, 0));
        }
    }
}

size_t segmented_ws_bytes(int key_bytes, bool has_vals, size_t total, const SegPlan& P)
{
    const size_t nt = P.tiles.size();
    size_t o = 0;
    o = align_up(o + (P.tiles.empty() ? 0 : total * key_bytes));          // tmp keys
    o = align_up(o + (P.tiles.empty() || !has_vals ? 0 : total * 4));      // tmp vals
    o = align_up(o + nt * R * 4);                                          // tile counts
    o = align_up(o + P.lsegs.size() * 2 * 4);                              // segment identity words
    o = align_up(o + P.lsegs.size() * (kMaxRounds + 1) * sizeof(RoundPlan)); // segment plans
    o = align_up(o + segmented_meta_bytes(P));                             // plan + lists
    return o;
}

size_t segmented_meta_bytes(const SegPlan& P)
{
    return align_up((kMaxRounds + 1) * sizeof(RoundPlan), 16) +
           (P.small[0].size() + P.small[1].size() + P.small[2].size() + P.tiles.size()) * sizeof(uint2) +
           P.lsegs.size() * sizeof(uint4) + P.tile_seg.size() * sizeof(uint32_t);
}

// Pack the round plan and the lists into `host` (pinned): plan, small[0..2],
// tiles, lsegs, tile_seg.  The large segments' rounds follow per-segment plans
// made on the device after round 0's count (k_seg_plans); the static plan here
// (every round runs; an even number of rounds ends in the output) is the
// reference layout of the lists only.
void segmented_pack(const SegPlan& P, int key_bytes, void* host)
{
    uint8_t* h = (uint8_t*)host;
    RoundPlan* plan = (RoundPlan*)h;
    const int rounds = key_bytes;
    int src = 0;
    for (int d = 0; d < kMaxRounds; ++d) {
        RoundPlan r{0, -1, 0, -1};
        if (d < rounds) {
            r.exec = 1;
            r.ord = d;
            r.src = src;
            r.dst = ((rounds - 1 - d) & 1) ? 2 : 1;
            src = r.dst;
        }
        plan[d] = r;
    }
    plan[kMaxRounds] = RoundPlan{0, 0, 0, 2};
    h += align_up((kMaxRounds + 1) * sizeof(RoundPlan), 16);
    for (int c = 0; c < 3; ++c) {
        memcpy(h, P.small[c].data(), P.small[c].size() * sizeof(uint2));
        h += P.small[c].size() * sizeof(uint2);
    }
    memcpy(h, P.tiles.data(), P.tiles.size() * sizeof(uint2));
    h += P.tiles.size() * sizeof(uint2);
    memcpy(h, P.lsegs.data(), P.lsegs.size() * sizeof(uint4));
    h += P.lsegs.size() * sizeof(uint4);
    memcpy(h, P.tile_seg.data(), P.tile_seg.size() * sizeof(uint32_t));
}

namespace {

// The large segments' rounds with tiles of WG * ITEMS keys: round 0's count
// also takes every segment's identity words, from which k_seg_plans makes the
// per-segment round plans; then per round the tile counts, the per-segment
// scan and the scatter, each reading its tile's segment plan.
struct LargeArgs {
    const void* keys_in;
    void* keys_out;
    void* keys_tmp;
    const uint32_t* vals_in;
    uint32_t* vals_out;
    uint32_t* vals_tmp;
    size_t total;
    size_t nt;
    uint32_t nls;
    const RoundPlan* plan;
    uint32_t* counts;
    uint32_t* seg_or;
    RoundPlan* seg_plan;
    const uint2* tiles;
    const uint4* lsegs;
    const uint32_t* tile_seg;
    int alias;
    uint32_t* dev_err;
    hipStream_t stream;
    Profiler* prof;
};

template <typename K, bool KV, int WG, int ITEMS>
void run_large(const LargeArgs& L)
{
    const int rounds = (int)sizeof(K);   // 8-bit digits over the whole key
    const uint32_t nrounds = sizeof(K);
    for (int d = 0; d < rounds; ++d) {
        RoundArgs a;
        a.keys_in = L.keys_in;
        a.keys_out = L.keys_out;
        a.keys_tmp = L.keys_tmp;
        a.vals_in = L.vals_in;
        a.vals_out = L.vals_out;
        a.vals_tmp = L.vals_tmp;
        a.n = (uint32_t)L.total;
        a.shift = 8u * d;
        a.mask = 0xFFu;
        a.round = d;
        a.ntiles = (uint32_t)L.nt;
        a.bases = nullptr;
        a.plan = L.plan;
        a.counts = L.counts;
        a.blk_state = nullptr;
        a.tickets = nullptr;
        a.err = L.dev_err;
        a.tiles = L.tiles;
        a.ntiles_dev = nullptr;
        a.tile_seg = L.tile_seg;
        a.seg_plan = L.seg_plan;
        a.lsegs = L.lsegs;
        if (L.prof) profiler_mark(L.prof, L.stream, kKindCount, true);
        if (d == 0) {
            a.seg_or = L.seg_or;
            hipLaunchKernelGGL((k_count<K, WG, ITEMS, true>), dim3(L.nt), dim3(WG), 0, L.stream, a, nullptr);
            a.seg_or = nullptr;
            hipLaunchKernelGGL(k_seg_plans, dim3((L.nls + 255) / 256), dim3(256), 0, L.stream,
                               (const uint32_t*)L.seg_or, L.nls, nrounds, L.alias, L.seg_plan,
                               (const uint32_t*)nullptr);
        } else {
            hipLaunchKernelGGL((k_count<K, WG, ITEMS, false>), dim3(L.nt), dim3(WG), 0, L.stream, a, nullptr);
        }
        if (L.prof) profiler_mark(L.prof, L.stream, kKindCount, false);
        if (L.prof) profiler_mark(L.prof, L.stream, kKindTileScan, true);
        hipLaunchKernelGGL(k_segscan, dim3(L.nls), dim3(R), 0, L.stream, a, L.lsegs);
        if (L.prof) profiler_mark(L.prof, L.stream, kKindTileScan, false);
        if (L.prof) profiler_mark(L.prof, L.stream, kKindRound, true);
        hipLaunchKernelGGL((k_scatter<K, KV, WG, ITEMS>), dim3(L.nt), dim3(WG), 0, L.stream, a);
        if (L.prof) profiler_mark(L.prof, L.stream, kKindRound, false);
    }
}

template <typename K, bool KV>
hipError_t run_segmented(const void* keys_in, void* keys_out, const uint32_t* vals_in,
                         uint32_t* vals_out, size_t total, const SegPlan& P, const void* host_meta,
                         void* ws, uint32_t* dev_err, hipStream_t stream, Profiler* prof,
                         int small_sort, const SegOverlap* ov)
{
    const uint32_t nrounds = sizeof(K);   // 8-bit digits over the whole key
    const size_t nt = P.tiles.size();
    uint8_t* w = (uint8_t*)ws;
    size_t o = 0;
    K* keys_tmp = (K*)(w + o);          o = align_up(o + (nt ? total * sizeof(K) : 0));
    uint32_t* vals_tmp = (uint32_t*)(w + o); o = align_up(o + (nt && KV ? total * 4 : 0));
    uint32_t* counts = (uint32_t*)(w + o);   o = align_up(o + nt * R * 4);
    const uint32_t nls = (uint32_t)P.lsegs.size();
    uint32_t* seg_or = (uint32_t*)(w + o);   o = align_up(o + nls * 2 * 4);
    RoundPlan* seg_plan = (RoundPlan*)(w + o); o = align_up(o + nls * (kMaxRounds + 1) * sizeof(RoundPlan));
    uint8_t* meta = w + o;
    const size_t meta_bytes = segmented_meta_bytes(P);
    hipError_t e = hipSuccess;
    if (meta_bytes && host_meta) {   // null: the plan is already in the workspace
        e = hipMemcpyAsync(meta, host_meta, meta_bytes, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return e;
    }
    const RoundPlan* plan = (const RoundPlan*)meta;
    const uint2* small[3];
    uint8_t* m = meta + align_up((kMaxRounds + 1) * sizeof(RoundPlan), 16);
    for (int c = 0; c < 3; ++c) {
        small[c] = (const uint2*)m;
        m += P.small[c].size() * sizeof(uint2);
    }
    const uint2* tiles = (const uint2*)m;
    m += nt * sizeof(uint2);
    const uint4* lsegs = (const uint4*)m;
    m += nls * sizeof(uint4);
    const uint32_t* tile_seg = (const uint32_t*)m;

    // The whole-segment sorts and the large segments' rounds touch disjoint
    // key ranges (and the workspace only for the plan, read by both): with an
    // aux stream the small ones run beside the rounds.
    const size_t nsmall = P.small[0].size() + P.small[1].size() + P.small[2].size();
    const bool fork = ov && ov->aux && nsmall && nt;
    hipStream_t ss = stream;
    if (fork) {
        e = hipEventRecord(ov->fork, stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(ov->aux, ov->fork, 0);
        if (e != hipSuccess) return e;
        ss = ov->aux;
    }
    if (prof) profiler_mark(prof, ss, kKindSmall, true);
    for (int c = 0; c < 3; ++c)
        launch_small<K, KV>(c, keys_in, keys_out, KV ? vals_in : nullptr, KV ? vals_out : nullptr,
                            small[c], (uint32_t)P.small[c].size(), nrounds, ss, small_sort);
    if (prof) profiler_mark(prof, ss, kKindSmall, false);
    if (fork) {
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(ov->join, ov->aux);
        if (e != hipSuccess) return e;
    }
    if (!nt) return hipGetLastError();

    const bool keys_alias = keys_in == keys_out, vals_alias = KV && vals_in == vals_out;
    const int alias = (keys_alias || vals_alias ? kAliasAny : 0) |
                      (keys_alias && (!KV || vals_alias) ? kAliasAll : 0);
    hipLaunchKernelGGL(k_zero_words, dim3((2 * nls + 255) / 256), dim3(256), 0, stream, seg_or, 2 * nls);
    LargeArgs la{keys_in, keys_out, keys_tmp, vals_in, vals_out, vals_tmp, total, nt, nls, plan,
                 counts, seg_or, seg_plan, tiles, lsegs, tile_seg, alias, dev_err, stream, prof};
    constexpr int IT = sizeof(K) == 8 ? 8 : 16;
    switch (P.tile_shape) {
    case 0: run_large<K, KV, 256, IT>(la); break;
    case 2: run_large<K, KV, 1024, IT>(la); break;
    default: run_large<K, KV, 512, IT>(la); break;
    }
    e = hipGetLastError();
    if (e == hipSuccess && fork) e = hipStreamWaitEvent(stream, ov->join, 0);
    return e;
}

}  // namespace

hipError_t segmented_sort(int key_bytes, const void* keys_in, void* keys_out,
                          const uint32_t* vals_in, uint32_t* vals_out, size_t total,
                          const SegPlan& P, const void* host_meta, void* ws, uint32_t* dev_err,
                          hipStream_t stream, Profiler* prof, int small_sort, const SegOverlap* ov)
{
    const bool kv = vals_in != nullptr;
    if (key_bytes == 4)
        return kv ? run_segmented<uint32_t, true>(keys_in, keys_out, vals_in, vals_out, total, P, host_meta, ws, dev_err, stream, prof, small_sort, ov)
                  : run_segmented<uint32_t, false>(keys_in, keys_out, vals_in, vals_out, total, P, host_meta, ws, dev_err, stream, prof, small_sort, ov);
    return kv ? run_segmented<uint64_t, true>(keys_in, keys_out, vals_in, vals_out, total, P, host_meta, ws, dev_err, stream, prof, small_sort, ov)
              : run_segmented<uint64_t, false>(keys_in, keys_out, vals_in, vals_out, total, P, host_meta, ws, dev_err, stream, prof, small_sort, ov);
}


// ---------------------------------------------------------------------------
// Device-planned segmented sort: the segment offsets live in device memory
// and are known to no host code (the sample sort's blocks and buckets).  One
// planning workgroup classifies the segments and writes the small-segment
// lists, the tile list, the per-segment tile ranges, the tile count and the
// round plan into the workspace; the round kernels are launched over an upper
// bound of the tile count and surplus workgroups exit at once.  No host
// traffic, so the sequence can be captured in a graph.
namespace {

constexpr int kPlanWG = 1024;

// Block-wide exclusive sum over kPlanWG threads; *total receives the sum.
__device__ uint32_t plan_exclusive_sum(uint32_t x, uint32_t* wsum, uint32_t* total)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t incl = wave_inclusive_sum(x);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (uint32_t w = 0; w < kPlanWG / 64; ++w) {
        const uint32_t v = wsum[w];
        before += w < wave ? v : 0u;
        all += v;
    }
    __syncthreads();
    *total = all;
    return before + incl - x;
}

__global__ __launch_bounds__(kPlanWG) void k_devseg_plan(const uint32_t* off, uint32_t nseg,
                                                         uint32_t n, uint32_t small_max,
                                                         uint32_t tile, uint32_t key_rounds,
                                                         const uint32_t* dev_rounds,
                                                         RoundPlan* plan, uint2* small,
                                                         uint2* tiles, uint4* lsegs,
                                                         uint32_t* tile_seg,
                                                         uint32_t* ntiles, uint32_t* err)
{
    __shared__ uint32_t wsum[kPlanWG / 64];
    const uint32_t tid = threadIdx.x;
    // Offsets must be nondecreasing and end within the arrays; otherwise
    // nothing is sorted (every round disabled, no segment) and the error word
    // records a bad plan.
    bool bad = false;
    for (uint32_t j = tid; j < nseg; j += kPlanWG) bad |= off[j + 1] < off[j];
    if (tid == 0) bad |= off[nseg] > n;
    if (__syncthreads_or(bad)) {
        if (tid <= (uint32_t)kMaxRounds) plan[tid] = RoundPlan{0, -1, 0, -1};
        for (uint32_t j = tid; j < nseg; j += kPlanWG) {
            for (uint32_t k = 0; k < 3; ++k) small[(size_t)k * nseg + j] = make_uint2(0, 0);
            lsegs[j] = make_uint4(0, 0, 0, 0);
        }
        if (tid == 0) {
            *ntiles = 0;
            atomicOr(err, (uint32_t)kErrBadPlan);
        }
        return;
    }
    // the large segments' rounds: the low digits the keys can differ in
    // (dev_rounds, when given), so the last one still writes the output; with
    // none the caller writes the output itself, so no segment is sorted whole
    // either
    const uint32_t rounds = dev_rounds ? min(key_rounds, *dev_rounds) : key_rounds;
    const bool none = dev_rounds && rounds == 0;
    if (tid <= (uint32_t)kMaxRounds) {
        RoundPlan r{0, -1, 0, -1};
        if (tid < rounds) {
            r.exec = 1;
            r.ord = (int32_t)tid;
            r.src = tid == 0 ? 0 : (((rounds - tid) & 1) ? 2 : 1);
            r.dst = ((rounds - 1 - tid) & 1) ? 2 : 1;
        }
        if (tid == (uint32_t)kMaxRounds) r = RoundPlan{0, 0, 0, 2};
        plan[tid] = r;
    }
    uint32_t base = 0;
    for (uint32_t c = 0; c < nseg; c += kPlanWG) {
        const uint32_t j = c + tid;
        uint32_t lo = 0, hi = 0, nt = 0;
        if (j < nseg) {
            lo = off[j];
            hi = off[j + 1];
            const uint32_t len = hi - lo;
            nt = len > small_max ? (len + tile - 1) / tile : 0u;
            // class c takes len in (cap[c-1], cap[c]]; other classes see an empty segment
            uint32_t cls = 3;
            if (len && len <= small_max && !none)
                for (uint32_t k = 0; k < 3; ++k)
                    if (len <= (uint32_t)(kSmallClasses[k].wg * kSmallClasses[k].items)) { cls = k; break; }
            for (uint32_t k = 0; k < 3; ++k)
                small[(size_t)k * nseg + j] = make_uint2(lo, k == cls ? hi : lo);
        }
        uint32_t total;
        const uint32_t t0 = base + plan_exclusive_sum(nt, wsum, &total);
        if (j < nseg) {
            lsegs[j] = make_uint4(t0, t0 + nt, lo, 0);
            for (uint32_t b = 0; b < nt; ++b) {
                const uint32_t first = lo + b * tile;
                tiles[t0 + b] = make_uint2(first, min(hi, first + tile));
                tile_seg[t0 + b] = j;
            }
        }
        base += total;
    }
    if (tid == 0) *ntiles = base;
}

template <typename K, bool KV>
hipError_t run_devseg(const void* keys_in, void* keys_out, const uint32_t* vals_in,
                      uint32_t* vals_out, size_t n, const uint32_t* off, uint32_t nseg,
                      uint32_t small_max, void* ws, const DevSegLayout& L, uint32_t* dev_err,
                      hipStream_t stream, Profiler* prof, int small_sort,
                      const uint32_t* dev_rounds)
{
    uint8_t* w = (uint8_t*)ws;
    K* keys_tmp = (K*)(w + L.off_tmp_keys);
    uint32_t* vals_tmp = KV ? (uint32_t*)(w + L.off_tmp_vals) : nullptr;
    uint32_t* counts = (uint32_t*)(w + L.off_counts);
    RoundPlan* plan = (RoundPlan*)(w + L.off_plan);
    uint2* small = (uint2*)(w + L.off_small);
    uint2* tiles = (uint2*)(w + L.off_tiles);
    uint4* lsegs = (uint4*)(w + L.off_lsegs);
    uint32_t* ntiles = (uint32_t*)(w + L.off_ntiles);
    uint32_t* tile_seg = (uint32_t*)(w + L.off_tile_seg);
    uint32_t* seg_or = (uint32_t*)(w + L.off_seg_or);
    RoundPlan* seg_plan = (RoundPlan*)(w + L.off_seg_plan);
    const uint32_t rounds = sizeof(K);
    hipLaunchKernelGGL(k_devseg_plan, dim3(1), dim3(kPlanWG), 0, stream, off, nseg, (uint32_t)n,
                       small_max, large_tile(sizeof(K)), rounds, dev_rounds, plan, small, tiles,
                       lsegs, tile_seg, ntiles, dev_err);
    hipLaunchKernelGGL(k_zero_words, dim3((2 * nseg + 255) / 256), dim3(256), 0, stream, seg_or, 2 * nseg);
    if (prof) profiler_mark(prof, stream, kKindSmall, true);
    for (int c = 0; c < 3; ++c)
        launch_small<K, KV>(c, keys_in, keys_out, KV ? vals_in : nullptr, KV ? vals_out : nullptr,
                            small + (size_t)c * nseg, nseg, rounds, stream, small_sort);
    if (prof) profiler_mark(prof, stream, kKindSmall, false);
    constexpr int WG = R8Config<K>::WG;
    constexpr int ITEMS = R8Config<K>::ITEMS;
    const bool keys_alias = keys_in == keys_out, vals_alias = KV && vals_in == vals_out;
    const int alias = (keys_alias || vals_alias ? kAliasAny : 0) |
                      (keys_alias && (!KV || vals_alias) ? kAliasAll : 0);
    for (uint32_t d = 0; d < rounds; ++d) {
        RoundArgs a;
        a.keys_in = keys_in;
        a.keys_out = keys_out;
        a.keys_tmp = keys_tmp;
        a.vals_in = vals_in;
        a.vals_out = vals_out;
        a.vals_tmp = vals_tmp;
        a.n = (uint32_t)n;
        a.shift = 8u * d;
        a.mask = 0xFFu;
        a.round = (int)d;
        a.ntiles = L.max_tiles;
        a.bases = nullptr;
        a.plan = plan;
        a.counts = counts;
        a.blk_state = nullptr;
        a.tickets = nullptr;
        a.err = dev_err;
        a.tiles = tiles;
        a.ntiles_dev = ntiles;
        a.tile_seg = tile_seg;
        a.seg_plan = seg_plan;
        a.lsegs = lsegs;
        a.dev_rounds = dev_rounds;
        if (prof) profiler_mark(prof, stream, kKindCount, true);
        if (d == 0) {
            // round 0's count also takes the segments' identity words, from
            // which every large segment gets its own round plan
            a.seg_or = seg_or;
            hipLaunchKernelGGL((k_count<K, R8Config<K>::CWG, R8Config<K>::CITEMS, true>), dim3(L.max_tiles), dim3(R8Config<K>::CWG), 0, stream, a, nullptr);
            a.seg_or = nullptr;
            hipLaunchKernelGGL(k_seg_plans, dim3((nseg + 255) / 256), dim3(256), 0, stream,
                               (const uint32_t*)seg_or, nseg, rounds, alias, seg_plan, dev_rounds);
        } else {
            hipLaunchKernelGGL((k_count<K, R8Config<K>::CWG, R8Config<K>::CITEMS, false>), dim3(L.max_tiles), dim3(R8Config<K>::CWG), 0, stream, a, nullptr);
        }
        if (prof) profiler_mark(prof, stream, kKindCount, false);
        if (prof) profiler_mark(prof, stream, kKindTileScan, true);
        hipLaunchKernelGGL(k_segscan, dim3(nseg), dim3(R), 0, stream, a, (const uint4*)lsegs);
        if (prof) profiler_mark(prof, stream, kKindTileScan, false);
        if (prof) profiler_mark(prof, stream, kKindRound, true);
        hipLaunchKernelGGL((k_scatter<K, KV, WG, ITEMS>), dim3(L.max_tiles), dim3(WG), 0, stream, a);
        if (prof) profiler_mark(prof, stream, kKindRound, false);
    }
    return hipGetLastError();
}

}  // namespace

DevSegLayout devseg_layout(int key_bytes, bool has_vals, size_t n, uint32_t nseg)
{
    DevSegLayout L;
    const uint32_t tile = large_tile(key_bytes);
    L.max_tiles = ((uint32_t)((n + tile - 1) / tile) + nseg + 7) & ~7u;   // multiple of 8: XCD slices
    size_t o = 0;
    L.off_tmp_keys = o;  o = align_up(o + n * key_bytes);
    L.off_tmp_vals = o;  o = align_up(o + (has_vals ? n * 4 : 0));
    L.off_counts = o;    o = align_up(o + (size_t)L.max_tiles * R * 4);
    L.off_plan = o;      o = align_up(o + (kMaxRounds + 1) * sizeof(RoundPlan));
    L.off_small = o;     o = align_up(o + (size_t)3 * nseg * sizeof(uint2));
    L.off_tiles = o;     o = align_up(o + (size_t)L.max_tiles * sizeof(uint2));
    L.off_lsegs = o;     o = align_up(o + (size_t)nseg * sizeof(uint4));
    L.off_ntiles = o;    o = align_up(o + 4);
    L.off_tile_seg = o;  o = align_up(o + (size_t)L.max_tiles * 4);
    L.off_seg_or = o;    o = align_up(o + (size_t)nseg * 2 * 4);
    L.off_seg_plan = o;  o = align_up(o + (size_t)nseg * (kMaxRounds + 1) * sizeof(RoundPlan));
    L.bytes = o;
    return L;
}

hipError_t devseg_sort(int key_bytes, const void* keys_in, void* keys_out, const uint32_t* vals_in,
                       uint32_t* vals_out, size_t n, const uint32_t* off, uint32_t nseg,
                       uint32_t small_max, void* ws, const DevSegLayout& L, uint32_t* dev_err,
                       hipStream_t stream, Profiler* prof, int small_sort,
                       const uint32_t* dev_rounds)
{
    if (!nseg || !n) return hipSuccess;
    const bool kv = vals_in != nullptr;
    if (key_bytes == 4)
        return kv ? run_devseg<uint32_t, true>(keys_in, keys_out, vals_in, vals_out, n, off, nseg, small_max, ws, L, dev_err, stream, prof, small_sort, dev_rounds)
                  : run_devseg<uint32_t, false>(keys_in, keys_out, vals_in, vals_out, n, off, nseg, small_max, ws, L, dev_err, stream, prof, small_sort, dev_rounds);
    return kv ? run_devseg<uint64_t, true>(keys_in, keys_out, vals_in, vals_out, n, off, nseg, small_max, ws, L, dev_err, stream, prof, small_sort, dev_rounds)
              : run_devseg<uint64_t, false>(keys_in, keys_out, vals_in, vals_out, n, off, nseg, small_max, ws, L, dev_err, stream, prof, small_sort, dev_rounds);
}

}  // namespace rsort
