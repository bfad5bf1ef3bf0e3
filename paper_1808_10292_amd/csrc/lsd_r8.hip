// PR4 on gfx950: LSD radix sort with radix 2^8, one stable count-sort round
// per 8-bit digit (arXiv 1808.10292, Section 3.2, PR4 and eq. Tp / Tp4).
//
// The paper's parallel round has three steps: every processor counts the
// digits of its block of keys, the p x r counts are exchanged so that each
// processor knows where its keys of each digit go, and the keys are routed
// there.  On one MI355X a "processor" is a tile of keys handled by one
// workgroup, and a round is three kernels:
//
//   k_count    per-tile digit counts (the count loop; one read of the keys);
//   k_tilescan the count exchange: for every tile t and digit v, the output
//              index of the tile's first key of digit v, i.e. the digit's
//              global start plus the keys of v in tiles before t (a scan over
//              tiles per digit, blocks of tiles chained by a decoupled
//              look-back);
//   k_scatter  the output loop: the tile is ranked stably by digit in LDS,
//              staged in digit order and written out -- consecutive threads
//              write consecutive slots of each digit's run -- with the payload
//              moved alongside.
//
// The first round's k_count also ORs together every key's difference from the
// first key in the same read, and k_plan derives the round plan from it: a
// round whose digit is the same for all n keys is the identity and is
// skipped.  Each round's digit starts come out of its own tile scan.
//
// No tile of a round waits for another tile: the dependencies are kernel
// boundaries, except the chain of tile blocks inside k_tilescan.
#include "lsd_kernels.h"
#include "onesweep_kernels.h"

namespace rsort {
namespace {

// Plain copy: each workgroup moves 4 consecutive 4 KiB blocks of 16-byte words
// per step (four loads in flight per thread, streaming hints) when both
// pointers are 16-byte aligned; bytes otherwise.
#ifndef RSORT_COPY_NT
#define RSORT_COPY_NT 1
#endif
#ifndef RSORT_COPY_BLOCKS
#define RSORT_COPY_BLOCKS 16384
#endif
constexpr int kCopyWG = 256;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kCopyWG) void k_copy_bytes(const uint8_t* src, uint8_t* dst, size_t bytes)
{
    constexpr int U = 4;
    size_t head = 0;
    if ((((uintptr_t)src | (uintptr_t)dst) & 15) == 0) {
        const size_t words = bytes / 16;
        const u32x4* s4 = (const u32x4*)src;
        u32x4* d4 = (u32x4*)dst;
        const size_t step = (size_t)gridDim.x * kCopyWG * U;
        for (size_t i = (size_t)blockIdx.x * kCopyWG * U + threadIdx.x; i < words; i += step) {
            u32x4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t j = i + (size_t)u * kCopyWG;
                if (j < words) v[u] = RSORT_COPY_NT ? __builtin_nontemporal_load(&s4[j]) : s4[j];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t j = i + (size_t)u * kCopyWG;
                if (j < words) {
                    if (RSORT_COPY_NT) __builtin_nontemporal_store(v[u], &d4[j]);
                    else d4[j] = v[u];
                }
            }
        }
        head = words * 16;
    }
    const size_t stride = (size_t)gridDim.x * kCopyWG;
    for (size_t i = head + (size_t)blockIdx.x * kCopyWG + threadIdx.x; i < bytes; i += stride)
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

uint32_t nblocks_of(uint32_t ntiles) { return (ntiles + kScanBlock - 1) / kScanBlock; }

// Workgroups that fit on the device at once for a kernel (cached per kernel).
uint32_t persistent_blocks(const void* kernel, int wg)
{
    static const void* cached_kernel[16];
    static uint32_t cached_value[16];
    for (int i = 0; i < 16; ++i)
        if (cached_kernel[i] == kernel) return cached_value[i];
    int dev = 0, cus = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, wg, 0) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    const uint32_t v = (uint32_t)(cus * per_cu);
    for (int i = 0; i < 16; ++i)
        if (!cached_kernel[i]) {
            cached_kernel[i] = kernel;
            cached_value[i] = v;
            break;
        }
    return v;
}

RoundArgs round_args(const void* keys_in, void* keys_out, void* keys_tmp, const uint32_t* vals_in,
                     uint32_t* vals_out, uint32_t* vals_tmp, size_t n, int begin_bit, int end_bit,
                     uint32_t d, const LsdR8Layout& L, uint32_t* bases, RoundPlan* plan,
                     uint32_t* counts, uint32_t* blk_state, uint32_t* tickets, uint32_t* dev_err)
{
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
    a.ntiles = L.ntiles;
    a.bases = bases;
    a.plan = plan;
    a.counts = counts;
    a.blk_state = blk_state;
    a.tickets = tickets;
    a.err = dev_err;
    a.tiles = nullptr;
    a.ntiles_dev = nullptr;
    return a;
}

template <typename K, bool KV, int WG = R8Config<K>::WG, int ITEMS = R8Config<K>::ITEMS>
hipError_t run(const void* keys_in, void* keys_out, const uint32_t* vals_in, uint32_t* vals_out,
               size_t n, int begin_bit, int end_bit, void* ws, const LsdR8Layout& L,
               uint32_t* dev_err, hipStream_t stream, Profiler* prof)
{
    constexpr int CWG = R8Config<K>::CWG;          // count kernel: same tile
    constexpr int CITEMS = WG * ITEMS / CWG;
    uint8_t* w = (uint8_t*)ws;
    uint32_t* hist = (uint32_t*)(w + L.off_hist);
    uint32_t* bases = (uint32_t*)(w + L.off_bases);
    RoundPlan* plan = (RoundPlan*)(w + L.off_plan);
    uint32_t* tickets = (uint32_t*)(w + L.off_tickets);
    uint32_t* counts = (uint32_t*)(w + L.off_counts);
    uint32_t* blk_state = (uint32_t*)(w + L.off_blk_state);
    K* keys_tmp = (K*)(w + L.off_tmp_keys);
    uint32_t* vals_tmp = KV ? (uint32_t*)(w + L.off_tmp_vals) : nullptr;
    const uint32_t nr = L.rounds;
    const bool keys_alias = keys_in == keys_out, vals_alias = KV && vals_in == vals_out;
    const bool in_place = keys_alias || vals_alias;
    const int alias = (in_place ? kAliasAny : 0) | (keys_alias && (!KV || vals_alias) ? kAliasAll : 0);
    const uint32_t nblk = nblocks_of(L.ntiles);

    uint32_t* mixed = hist;   // kMixWords words
    static_assert(kMixWords <= (size_t)kHistReplicas * kMaxRounds * R, "identity words fit");
    // Scatter grid: one workgroup per tile, or RSORT_SCATTER_WAVES resident
    // workgroups per CU looping over the tiles.
    // The small-tile shape exists only for sorts of few tiles (inline scan).
    constexpr bool kSmallShape = sizeof(K) == 4 && WG == kSmallWG32 && ITEMS == kSmallItems32;
    static_assert((size_t)RSORT_SMALL_TILE_MAXN <= (size_t)RSORT_INLINE_SCAN_TILES * kSmallTile32,
                  "small-tile sorts have few enough tiles for the inline scan");
    uint32_t sgrid = L.ntiles;
    if constexpr (RSORT_SCATTER_PERSIST && !kSmallShape) {
        const uint32_t resident = persistent_blocks((const void*)k_scatter<K, KV, WG, ITEMS>, WG);
        sgrid = std::min<uint32_t>(L.ntiles, resident & ~7u ? resident & ~7u : resident);
    }
    // Few tiles: no tile-scan kernel (the scatter sums the tile counts
    // itself) and one identity pair per tile, stored without atomics, so
    // nothing needs clearing before round 0's count.
    const bool inline_scan = L.ntiles <= RSORT_INLINE_SCAN_TILES && sgrid == L.ntiles;
    static_assert(2 * RSORT_INLINE_SCAN_TILES <= (size_t)kHistReplicas * kMaxRounds * R,
                  "one identity pair per tile fits");
    if (!inline_scan)
        hipLaunchKernelGGL(k_init, dim3(256), dim3(256), 0, stream, mixed, kMixWords, tickets, nr,
                           blk_state, (size_t)nr * nblk * R);
    // Round 0's tile counts and the identity test of every round in one read.
    {
        RoundArgs a0 = round_args(keys_in, keys_out, keys_tmp, vals_in, vals_out, vals_tmp, n,
                                  begin_bit, end_bit, 0, L, bases, plan, counts, blk_state,
                                  tickets, dev_err);
        a0.mix_dense = inline_scan ? 1u : 0u;
        a0.counts16 = inline_scan ? 1u : 0u;
        if (prof) profiler_mark(prof, stream, kKindHist, true);
        hipLaunchKernelGGL((k_count<K, CWG, CITEMS, true>), dim3(L.ntiles), dim3(R8Config<K>::CWG), 0, stream, a0,
                           mixed);
        if (prof) profiler_mark(prof, stream, kKindHist, false);
    }
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(64), 0, stream, (const uint32_t*)mixed, nr,
                       (uint32_t)begin_bit, (uint32_t)end_bit, alias, plan,
                       inline_scan ? L.ntiles : 0u);
    if (in_place && (nr & 1)) {
        const uint32_t g = (uint32_t)((n + 256 * kPrecopyItems - 1) / (256 * kPrecopyItems));
        hipLaunchKernelGGL(k_precopy<K>, dim3(g), dim3(256), 0, stream, (const RoundPlan*)plan,
                           (const K*)keys_in, keys_tmp, KV ? vals_in : nullptr, vals_tmp, (uint32_t)n);
    }
    for (uint32_t d = 0; d < nr; ++d) {
        RoundArgs a = round_args(keys_in, keys_out, keys_tmp, vals_in, vals_out, vals_tmp, n,
                                 begin_bit, end_bit, d, L, bases, plan, counts, blk_state,
                                 tickets, dev_err);
        a.counts16 = inline_scan ? 1u : 0u;
        if (d > 0) {   // round 0 was counted with the histograms
            if (prof) profiler_mark(prof, stream, kKindCount, true);
            hipLaunchKernelGGL((k_count<K, CWG, CITEMS, false>), dim3(L.ntiles), dim3(R8Config<K>::CWG), 0, stream,
                               a, nullptr);
            if (prof) profiler_mark(prof, stream, kKindCount, false);
        }
        if (!inline_scan) {
            if (prof) profiler_mark(prof, stream, kKindTileScan, true);
            hipLaunchKernelGGL(k_tilescan, dim3(nblk), dim3(R), 0, stream, a);
            if (prof) profiler_mark(prof, stream, kKindTileScan, false);
        }
        if (prof) profiler_mark(prof, stream, kKindRound, true);
        if constexpr (kSmallShape) {
            hipLaunchKernelGGL((k_scatter<K, KV, WG, ITEMS, true>), dim3(sgrid), dim3(WG), 0, stream, a);
        } else {
            if (inline_scan)
                hipLaunchKernelGGL((k_scatter<K, KV, WG, ITEMS, true>), dim3(sgrid), dim3(WG), 0, stream, a);
            else
                hipLaunchKernelGGL((k_scatter<K, KV, WG, ITEMS>), dim3(sgrid), dim3(WG), 0, stream, a);
        }
        if (prof) profiler_mark(prof, stream, kKindRound, false);
    }
    return hipGetLastError();
}

// Single-read rounds of 32-bit keys (onesweep_kernels.h).
template <bool KV>
hipError_t run_os(const void* keys_in, void* keys_out, const uint32_t* vals_in, uint32_t* vals_out,
                  size_t n, int begin_bit, int end_bit, void* ws, const LsdR8Layout& L,
                  uint32_t* dev_err, hipStream_t stream, Profiler* prof)
{
    typedef uint32_t K;
    constexpr int WG = R8Config<K>::WG;
    constexpr int ITEMS = R8Config<K>::ITEMS;
    uint8_t* w = (uint8_t*)ws;
    uint32_t* mixed = (uint32_t*)(w + L.off_hist);
    uint32_t* bases = (uint32_t*)(w + L.off_bases);
    RoundPlan* plan = (RoundPlan*)(w + L.off_plan);
    uint32_t* rows = (uint32_t*)(w + L.off_os_rows);
    uint32_t* cbx = (uint32_t*)(w + L.off_os_cbx);
    uint32_t* tot = (uint32_t*)(w + L.off_os_tot);
    uint32_t* J = (uint32_t*)(w + L.off_os_J);
    uint32_t* jx = (uint32_t*)(w + L.off_os_jx);
    OsRound* rinfo = (OsRound*)(w + L.off_os_rinfo);
    uint4* tt = (uint4*)(w + L.off_os_tt);
    uint32_t* chains = (uint32_t*)(w + L.off_os_chains);
    uint32_t* state = (uint32_t*)(w + L.off_os_state);
    uint32_t* tick = (uint32_t*)(w + L.off_os_tick);
    K* keys_tmp = (K*)(w + L.off_tmp_keys);
    uint32_t* vals_tmp = KV ? (uint32_t*)(w + L.off_tmp_vals) : nullptr;
    const uint32_t nr = L.rounds;
    const bool keys_alias = keys_in == keys_out, vals_alias = KV && vals_in == vals_out;
    const bool in_place = keys_alias || vals_alias;
    const int alias = (in_place ? kAliasAny : 0) | (keys_alias && (!KV || vals_alias) ? kAliasAll : 0);
    OsShape sh;
    sh.nchunks = L.os_nchunks;
    sh.chunk_keys = L.os_chunk_keys;
    sh.roww = L.os_roww;
    sh.maxrows = L.os_maxrows;
    sh.cmax = L.os_cmax;
    const uint32_t state_words = sh.maxrows * R;

    hipLaunchKernelGGL(k_os_init, dim3(16), dim3(256), 0, stream, mixed, kMixWords, tick,
                       nr * kQueues * kQueueStride);
    if (prof) profiler_mark(prof, stream, kKindHist, true);
    hipLaunchKernelGGL(k_os_count<K>, dim3(sh.nchunks), dim3(kOsCountWG), 0, stream, (const K*)keys_in,
                       (uint32_t)n, sh.chunk_keys, (uint32_t)begin_bit, (uint32_t)end_bit, nr, rows,
                       sh.roww, mixed, state, state_words);
    if (prof) profiler_mark(prof, stream, kKindHist, false);
    if (prof) profiler_mark(prof, stream, kKindTileScan, true);
    hipLaunchKernelGGL(k_os_reduce, dim3((sh.roww + 63) / 64), dim3(kOsReduceWG), 0, stream,
                       (const uint32_t*)rows, sh.nchunks, sh.roww, nr, cbx, tot, J);
    hipLaunchKernelGGL(k_os_plan, dim3(1), dim3(kOsPlanWG), 0, stream, (const uint32_t*)mixed, nr,
                       (uint32_t)begin_bit, (uint32_t)end_bit, alias, (uint32_t)n, L.tile, sh, plan,
                       (const uint32_t*)tot, (const uint32_t*)J, bases, jx, rinfo, chains);
    hipLaunchKernelGGL(k_os_tickets, dim3((sh.maxrows + kOsTicketWG - 1) / kOsTicketWG, nr),
                       dim3(kOsTicketWG), 0, stream, (const RoundPlan*)plan, (const OsRound*)rinfo,
                       (const uint32_t*)chains, sh.cmax, sh.maxrows, (uint32_t)n, L.tile, tt);
    if (prof) profiler_mark(prof, stream, kKindTileScan, false);
    if (in_place && (nr & 1)) {
        const uint32_t g = (uint32_t)((n + 256 * kPrecopyItems - 1) / (256 * kPrecopyItems));
        hipLaunchKernelGGL(k_precopy<K>, dim3(g), dim3(256), 0, stream, (const RoundPlan*)plan,
                           (const K*)keys_in, keys_tmp, KV ? vals_in : nullptr, vals_tmp, (uint32_t)n);
    }
    for (uint32_t d = 0; d < nr; ++d) {
        OsArgs a;
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
        a.plan = plan;
        a.rinfo = rinfo;
        a.tt = tt + (size_t)d * sh.maxrows;
        a.row0 = chains + (size_t)(3 * d + 2) * sh.cmax;
        a.cb_chunk = cbx + (size_t)d * sh.nchunks * R;
        a.cb_joint = jx + (size_t)d * kJointChains * R;
        a.bases = bases;
        a.state = state;
        a.maxrows = sh.maxrows;
        a.tick = tick + (size_t)d * kQueues * kQueueStride;
        a.err = dev_err;
        if (prof) profiler_mark(prof, stream, kKindRound, true);
        hipLaunchKernelGGL((k_onesweep<K, KV, WG, ITEMS>), dim3(sh.maxrows), dim3(WG), 0, stream, a);
        if (prof) profiler_mark(prof, stream, kKindRound, false);
    }
    return hipGetLastError();
}

}  // namespace

LsdR8Layout lsd_r8_layout(int key_bytes, bool has_vals, size_t n, int begin_bit, int end_bit,
                          bool single_read)
{
    LsdR8Layout L{};
    L.rounds = rounds_of(begin_bit, end_bit, 8);
    L.tile = key_bytes == 8 ? R8Config<uint64_t>::WG * R8Config<uint64_t>::ITEMS
                            : R8Config<uint32_t>::WG * R8Config<uint32_t>::ITEMS;
    // small 32-bit sorts (counted rounds): tiles of half the keys, so that
    // twice as many workgroups share the work of a round and each ranks half
    // as many rows
    if (key_bytes == 4 && !single_read && n <= (size_t)RSORT_SMALL_TILE_MAXN) L.tile = kSmallTile32;
    L.ntiles = (uint32_t)((n + L.tile - 1) / L.tile);
    const uint32_t nblk = nblocks_of(L.ntiles);
    size_t o = 0;
    L.off_tmp_keys = o;  o = align_up(o + n * key_bytes);
    L.off_tmp_vals = o;  o = align_up(o + (has_vals ? n * 4 : 0));
    L.off_counts = o;    o = align_up(o + (size_t)L.ntiles * R * 4);
    L.off_blk_state = o; o = align_up(o + (size_t)std::max(1u, L.rounds) * nblk * R * 4);
    L.off_hist = o;      o = align_up(o + (size_t)kHistReplicas * kMaxRounds * R * 4);
    L.off_bases = o;     o = align_up(o + (size_t)kMaxRounds * R * 4);
    L.off_plan = o;      o = align_up(o + (kMaxRounds + 1) * sizeof(RoundPlan));
    L.off_tickets = o;   o = align_up(o + kMaxRounds * 4);
    L.onesweep = single_read && key_bytes == 4 && L.rounds > 0 && L.rounds <= 4;
    if (L.onesweep) {
        const uint32_t cpt = std::max<uint32_t>(kOsMinChunkTiles, (L.ntiles + kOsMaxChunks - 1) / kOsMaxChunks);
        L.os_nchunks = std::max<uint32_t>(1, (L.ntiles + cpt - 1) / cpt);
        L.os_chunk_keys = cpt * L.tile;
        L.os_roww = L.rounds * R + (L.rounds - 1) * kJointBins;
        L.os_maxrows = (L.ntiles + kJointChains + 7) & ~7u;
        L.os_cmax = std::max<uint32_t>(L.os_nchunks, kJointChains);
        const size_t nr = L.rounds;
        L.off_os_rows = o;   o = align_up(o + (size_t)L.os_nchunks * L.os_roww * 4);
        L.off_os_cbx = o;    o = align_up(o + nr * L.os_nchunks * R * 4);
        L.off_os_tot = o;    o = align_up(o + nr * R * 4);
        L.off_os_J = o;      o = align_up(o + nr * kJointBins * 4);
        L.off_os_jx = o;     o = align_up(o + nr * kJointChains * R * 4);
        L.off_os_rinfo = o;  o = align_up(o + nr * sizeof(OsRound));
        L.off_os_tt = o;     o = align_up(o + nr * L.os_maxrows * sizeof(uint4));
        L.off_os_chains = o; o = align_up(o + 3 * nr * L.os_cmax * 4);
        L.off_os_state = o;  o = align_up(o + 2 * (size_t)L.os_maxrows * R * 4);
        L.off_os_tick = o;   o = align_up(o + nr * kQueues * kQueueStride * 4);
    }
    L.bytes = o;
    return L;
}

hipError_t lsd_r8_sort(int key_bytes, const void* keys_in, void* keys_out,
                       const uint32_t* vals_in, uint32_t* vals_out, size_t n,
                       int begin_bit, int end_bit, void* ws, const LsdR8Layout& L,
                       uint32_t* dev_err, hipStream_t stream, Profiler* prof)
{
    const bool kv = vals_in != nullptr;
    if (L.onesweep)
        return kv ? run_os<true>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof)
                  : run_os<false>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof);
    if (key_bytes == 4 && L.tile == kSmallTile32)
        return kv ? run<uint32_t, true, kSmallWG32, kSmallItems32>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof)
                  : run<uint32_t, false, kSmallWG32, kSmallItems32>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof);
    if (key_bytes == 4)
        return kv ? run<uint32_t, true>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof)
                  : run<uint32_t, false>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof);
    return kv ? run<uint64_t, true>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof)
              : run<uint64_t, false>(keys_in, keys_out, vals_in, vals_out, n, begin_bit, end_bit, ws, L, dev_err, stream, prof);
}

hipError_t copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t stream)
{
    if (!bytes || dst == src) return hipSuccess;
    uint32_t g = (uint32_t)std::min<size_t>((bytes + 16383) / 16384, RSORT_COPY_BLOCKS);
    hipLaunchKernelGGL(k_copy_bytes, dim3(g), dim3(kCopyWG), 0, stream, (const uint8_t*)src,
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
    (void)begin_bit;
    (void)end_bit;
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
