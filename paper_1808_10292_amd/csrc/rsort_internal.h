// Host-side interfaces between the C ABI (api.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace rsort {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// One entry per count-sort round, written on the device by the scan kernel:
// whether the round runs (it is skipped when one digit value holds every key,
// which makes the round the identity), its ordinal among the rounds that run,
// and where it reads and writes: 0 = caller input, 1 = caller output,
// 2 = workspace temporary.
struct RoundPlan {
    int32_t exec;
    int32_t ord;
    int32_t src;
    int32_t dst;
};

constexpr int kMaxRounds = 8;      // 64-bit keys, 8-bit digits
constexpr int kHistReplicas = 8;   // global histogram copies, picked by block index

// Optional kernel timing: HIP events recorded on the launch stream around the
// kernels of one kind (implemented in api.hip).  nullptr disables it.
enum KernelKind { kKindRound = 0, kKindHist = 1, kKindCount = 2, kKindTileScan = 3, kKindSmall = 4,
                  kKindGroup = 5, kNumKinds = 6 };
struct Profiler;
void profiler_mark(Profiler* p, hipStream_t s, int kind, bool begin);

// ---------------------------------------------------------------------------
// Radix 2^8 LSD (PR4).  Counted rounds (per-tile counts, a scan over tiles,
// then the routing kernel) for every key type; 32-bit keys can instead run
// single-read rounds (onesweep_kernels.h: one counting pass, then per round
// one kernel that counts, looks back inside its chain of tiles and routes).
struct LsdR8Layout {
    uint32_t rounds;     // number of 8-bit (or narrower, last) digits
    uint32_t tile;       // keys per tile in a round
    uint32_t ntiles;
    size_t off_tmp_keys, off_tmp_vals, off_counts, off_blk_state;
    size_t off_hist, off_bases, off_plan, off_tickets;
    // single-read rounds (onesweep == true)
    bool onesweep;
    uint32_t os_nchunks, os_chunk_keys, os_roww, os_maxrows, os_cmax;
    size_t off_os_rows, off_os_cbx, off_os_tot, off_os_J, off_os_jx, off_os_rinfo, off_os_tt,
        off_os_chains, off_os_state, off_os_tick;
    size_t bytes;
};

// single_read: 32-bit keys with at most four rounds use the single-read
// rounds (other requests keep the counted rounds).
LsdR8Layout lsd_r8_layout(int key_bytes, bool has_vals, size_t n, int begin_bit, int end_bit,
                          bool single_read = false);

// Enqueue the whole sort on `stream`.  ws must hold layout.bytes bytes.
hipError_t lsd_r8_sort(int key_bytes, const void* keys_in, void* keys_out,
                       const uint32_t* vals_in, uint32_t* vals_out, size_t n,
                       int begin_bit, int end_bit, void* ws, const LsdR8Layout& L,
                       uint32_t* dev_err, hipStream_t stream, Profiler* prof);

// ---------------------------------------------------------------------------
// Radix 2^16 LSD (PR2, lsd_r16.hip): per round, chunk rows of 65536 counts,
// column prefixes, and a chunk-ordered placement through LDS-sorted tiles.
struct LsdR16Layout {
    uint32_t rounds;    // 16-bit (last one narrower) digits
    uint32_t chunk;     // keys per chunk (a multiple of the tile)
    uint32_t nchunks;   // workgroups / count rows (<= 4096)
    size_t off_tmp_keys, off_tmp_vals, off_rows, off_win, off_tot;
    size_t off_grp_keys, off_grp_vals, off_r8;   // grouped keys, grouping round
    size_t bytes;
};
LsdR16Layout lsd_r16_layout(int key_bytes, bool has_vals, size_t n, int begin_bit, int end_bit);
hipError_t lsd_r16_sort(int key_bytes, const void* keys_in, void* keys_out,
                        const uint32_t* vals_in, uint32_t* vals_out, size_t n, int begin_bit,
                        int end_bit, void* ws, const LsdR16Layout& L, uint32_t* dev_err,
                        hipStream_t stream, Profiler* prof);

// Digit histograms of every digit (8- or 16-bit) of [begin_bit, end_bit).
size_t histogram_ws_bytes(int digit_bits, int begin_bit, int end_bit);
hipError_t histogram(int key_bytes, const void* keys, size_t n, int digit_bits,
                     int begin_bit, int end_bit, uint32_t* hist_out, void* ws,
                     hipStream_t stream);

// ---------------------------------------------------------------------------
// Batched segmented sort (segmented.hip).  Segments of at most small_max keys
// are sorted whole in LDS by one workgroup (three capacity classes); larger
// ones are cut into tiles for the round kernels.
// Tile shapes of the large-segment path (workgroup size; keys per thread are
// 16 for 32-bit and 8 for 64-bit keys): 256, 512 (default) or 1024 threads.
constexpr int kSegTileShapes = 3;
constexpr int kSegTileShapeDefault = 1;
uint32_t seg_tile_keys(int key_bytes, int shape);
struct SegPlan {
    std::vector<uint2> small[3];   // {first key, end} per small segment, by class
    std::vector<uint2> tiles;      // {first key, end} per tile of the large segments
    std::vector<uint4> lsegs;      // {first tile, end tile, first key, 0} per large segment
    std::vector<uint32_t> tile_seg;   // large segment (index into lsegs) of every tile
    int tile_shape = kSegTileShapeDefault;   // of the large path's tiles
};
constexpr uint32_t kSmallMaxDefault = 8192;
void segmented_plan(const uint64_t* offsets, size_t num_segs, uint32_t small_max, int key_bytes,
                    SegPlan& P, int tile_shape = kSegTileShapeDefault);
size_t segmented_meta_bytes(const SegPlan& P);
size_t segmented_ws_bytes(int key_bytes, bool has_vals, size_t total, const SegPlan& P);
void segmented_pack(const SegPlan& P, int key_bytes, void* host);
// small_sort: the sorter of the small segments (0 radix rounds, 1 BTN, 2 OET).
// Overlap (optional): the whole-segment sorts run on `aux`, forked from and
// joined back into `stream` with the two events, while the large segments'
// rounds run on `stream` (the two touch disjoint key ranges).
struct SegOverlap {
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
hipError_t segmented_sort(int key_bytes, const void* keys_in, void* keys_out,
                          const uint32_t* vals_in, uint32_t* vals_out, size_t total,
                          const SegPlan& P, const void* host_meta, void* ws, uint32_t* dev_err,
                          hipStream_t stream, Profiler* prof, int small_sort = 0,
                          const SegOverlap* ov = nullptr);

// The same sort in one persistent launch (seg_persist.hip): a resident grid
// takes histogram, small-segment and round items from one ticket counter.
// Small segments are those of at most persist_small_max keys (and at most the
// plan's small_max); plan with segmented_plan(..., persist_tile_shape(...)).
uint32_t persist_small_max(int key_bytes);
int persist_tile_shape(int key_bytes);   // the plan's tile shape: tiles of persist_small_max keys
int persist_threads();                    // workgroup size of the persistent kernel
size_t persist_meta_bytes(const SegPlan& P, int key_bytes);
size_t persist_ws_bytes(int key_bytes, bool has_vals, size_t total, const SegPlan& P);
void persist_pack(const SegPlan& P, int key_bytes, void* host);
hipError_t persist_sort(int key_bytes, const void* keys_in, void* keys_out, const uint32_t* vals_in,
                        uint32_t* vals_out, size_t total, const SegPlan& P, const void* host_meta,
                        void* ws, uint32_t* dev_err, hipStream_t stream, Profiler* prof);

// Device-planned segmented sort: offsets (nseg + 1 u32, nondecreasing) live in
// device memory.  ws must hold devseg_layout(...).bytes bytes.
struct DevSegLayout {
    uint32_t max_tiles;   // upper bound of the tile count: ceil(n / tile) + nseg, rounded up to 8
    size_t off_tmp_keys, off_tmp_vals, off_counts, off_plan, off_small, off_tiles, off_lsegs,
        off_ntiles, off_tile_seg, off_seg_or, off_seg_plan;
    size_t bytes;
};
DevSegLayout devseg_layout(int key_bytes, bool has_vals, size_t n, uint32_t nseg);
hipError_t devseg_sort(int key_bytes, const void* keys_in, void* keys_out, const uint32_t* vals_in,
                       uint32_t* vals_out, size_t n, const uint32_t* off, uint32_t nseg,
                       uint32_t small_max, void* ws, const DevSegLayout& L, uint32_t* dev_err,
                       hipStream_t stream, Profiler* prof, int small_sort = 0,
                       const uint32_t* dev_rounds = nullptr);

// ---------------------------------------------------------------------------
// Oversampling sample sorts (sample_sort.hip), 32-bit keys: GSD (regular
// sample of the sorted blocks), GER (random sample of the sorted blocks) and
// GVR (random sample of the input, no local sort, the input split around the
// splitters by a count sort on the bucket index).
enum SampleKind { kGSD = 0, kGER = 1, kGVR = 2 };
constexpr uint32_t kGvrMaxP = 256;   // GVR buckets: one 8-bit routing digit
struct GsdLayout {
    uint32_t p;                 // blocks = buckets (the request clamped to n)
    uint32_t s;                 // samples per block (r p for GSD)
    uint32_t tiles_per_block;   // route workgroups per block
    size_t nT;                  // sample size: p s (GSD), s p - 1 (GER, GVR)
    int kind;                   // SampleKind
    LsdR8Layout LT;             // the sample's sort by key (with positions)
    LsdR8Layout LTk;            // GER, GVR: the sort of the drawn positions
    DevSegLayout LS;            // local sort and bucket finish
    size_t off_lo, off_boff, off_bsize, off_coloff, off_Tk, off_Tg, off_Sk, off_Sg, off_lsd,
        off_Y, off_YV, off_seg;
    // GSD step 5 as a merge (p <= 256): pieces cut at a sorted regular sample
    // of the sorted blocks (GSD: its own sample; GER: a second one, s2 per
    // block, sorted with LT2; GSD's s2 is s), each of its p intervals of s2
    // elements cut into q parts: M = p q boundaries, F = (M + 2) x p run bounds
    bool merge;
    uint32_t q, M, s2;
    size_t nT2;
    LsdR8Layout LT2;
    size_t off_F, off_BK, off_large, off_R;
    // GVR route: tile counts, tile-scan state, round plan + ticket, bucket
    // starts, one bucket byte per key, the bucket-search table, and the
    // bucket key offsets (+ the round count), the tiles' key minima / maxima
    uint32_t route_tpb, route_ntiles;
    size_t off_rcounts, off_rstate, off_rplan, off_rbases, off_bkt, off_rtab, off_rshift,
        off_rmm;
    size_t bytes;
};
GsdLayout gsd_layout(bool has_vals, size_t n, uint32_t p, uint32_t r);
GsdLayout ger_layout(bool has_vals, size_t n, uint32_t p, uint32_t s);
GsdLayout gvr_layout(bool has_vals, size_t n, uint32_t p, uint32_t s);
// Statistics area (device, u32): split bounds p x (p+1), splitter keys (p),
// splitter indexes (p).
size_t gsd_stats_words(uint32_t p);
hipError_t gsd_sort(const uint32_t* keys_in, uint32_t* keys_out, const uint32_t* vals_in,
                    uint32_t* vals_out, size_t n, const GsdLayout& L, uint64_t seed, void* ws,
                    uint32_t* stats, uint32_t* dev_err, hipStream_t stream, Profiler* prof);

// Order-preserving maps of signed / IEEE float keys onto unsigned ones
// (key_order.hip); inverse = true restores the keys.  in == out is allowed.
enum KeyKind { kKeyUnsigned = 0, kKeySigned = 1, kKeyFloat = 2 };
hipError_t map_keys(int key_bytes, int kind, bool inverse, const void* in, void* out, size_t n,
                    hipStream_t stream);

// Plain device copy used when a sort moves nothing (empty bit range).
hipError_t copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t stream);

// Device memory for the library's own buffers (workspaces, error words,
// descriptors).  hipMalloc, except that a test hook can make one allocation
// fail as out of memory: rsort_debug_fail_alloc(k), or RSORT_FAULT_ALLOC=k in
// the environment when the library first allocates, fails the k-th call from
// then on.
hipError_t dev_malloc(void** p, size_t bytes);

}  // namespace rsort
