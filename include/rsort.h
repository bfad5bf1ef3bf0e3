/*
 * rsort.h -- C ABI of the MI355X (gfx950) integer-sorting library.
 *
 * The library sorts n integer keys, optionally carrying a 32-bit payload, on
 * one AMD Instinct GPU.  It implements the data-parallel sorts studied in
 * Gerbessiotis, "A study of integer sorting on multicores" (arXiv 1808.10292):
 *
 *   RSORT_LSD_R8          PR4: LSD radix sort with radix r = 2^8, one stable
 *                         count-sort round per 8-bit digit (Section 3.2, PR4,
 *                         equations Tp and Tp4);
 *   RSORT_LSD_R16         PR2: the same with r = 2^16 (Section 3.2, eq. Tp2);
 *   RSORT_SAMPLE_REGULAR  GSD: local sort of p blocks, regular oversampling,
 *                         splitter selection, split by binary search,
 *                         routing to p buckets and a stable sort of every
 *                         bucket (Section 3.3, Algorithm 1).
 *
 * Every algorithm returns the same, unique result: the stable sort.  Keys come
 * out nondecreasing (as unsigned integers), equal keys keep their input order,
 * and each payload moves with its key.
 *
 * Conventions shared by every entry point
 *   - Return value: RSORT_OK (0) or a negative rsort_status.  No entry point
 *     aborts or throws.  Argument errors are detected before anything is
 *     enqueued.  Device-side failures are reported by rsort_synchronize.
 *   - Data pointers are HIP device pointers owned by the caller; the library
 *     never frees them.  Host pointers are rejected with RSORT_EINVAL.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is enqueued asynchronously on it and is stream-ordered; the call returns
 *     before the GPU finishes.
 *   - An rsort_ctx is used by one host thread at a time.
 *   - n < 2^30 (RSORT_EUNSUPPORTED otherwise).
 */
#ifndef RSORT_H
#define RSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rsort_ctx rsort_ctx;

enum rsort_status {
    RSORT_OK = 0,
    RSORT_EINVAL = -1,        /* bad argument (NULL, host pointer, overlap, range) */
    RSORT_ENOMEM = -2,        /* device allocation failed                          */
    RSORT_EDEVICE = -3,       /* a HIP call or a kernel failed                     */
    RSORT_EBUSY = -4,         /* resource in use                                   */
    RSORT_EUNSUPPORTED = -5   /* valid request outside the library's limits        */
};

enum rsort_key_type {
    RSORT_U32 = 0, RSORT_U64 = 1,   /* unsigned integers: every entry point */
    /* rsort_sort and rsort_workspace_bytes only (whole keys, radix sorts):
     * two's complement integers, and IEEE 754 binary32 / binary64 ordered by
     * totalOrder (-NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN) */
    RSORT_I32 = 2, RSORT_F32 = 3, RSORT_I64 = 4, RSORT_F64 = 5
};

enum rsort_algo {
    RSORT_AUTO = 0,            /* currently RSORT_LSD_R8                           */
    RSORT_LSD_R8 = 1,          /* PR4                                              */
    RSORT_LSD_R16 = 2,         /* PR2                                              */
    RSORT_SAMPLE_REGULAR = 3   /* GSD skeleton (uint32 keys)                        */
};

/* Create a context bound to HIP device `hip_device`.  The context owns a
 * growable cached workspace and small device-side state (error word, the
 * statistics of the last sample sort).  *out receives the handle. */
int rsort_create(int hip_device, rsort_ctx** out);

/* Release the context and everything it allocated.  Waits for the device. */
int rsort_destroy(rsort_ctx* ctx);

/* Static description of a status code. */
const char* rsort_status_string(int status);

/* Detail message for the last failure seen on ctx ("" if none).  The pointer
 * stays valid until the next call on ctx. */
const char* rsort_last_error(const rsort_ctx* ctx);

/* Bytes of workspace rsort_sort needs for this request (algo as in rsort_sort;
 * for RSORT_SAMPLE_REGULAR the default p and r).  Monotone in n. */
int rsort_workspace_bytes(rsort_ctx* ctx, int key_type, int has_vals, size_t n,
                          int algo, size_t* bytes);

/*
 * Stable sort of n keys on the key bits [begin_bit, end_bit).
 *
 *   key_type   RSORT_U32 (keys are uint32_t) or RSORT_U64 (uint64_t); also
 *              RSORT_I32 / RSORT_I64 (signed) and RSORT_F32 / RSORT_F64 (IEEE
 *              totalOrder), whole keys with RSORT_AUTO / _LSD_R8 / _LSD_R16:
 *              mapped by an order-preserving bijection into a workspace copy,
 *              sorted as unsigned keys and mapped back (two extra passes).
 *   keys_in    device array of n keys; read only unless it equals keys_out.
 *   keys_out   device array of n keys receiving the sorted keys.  keys_in ==
 *              keys_out sorts in place; any other overlap is RSORT_EINVAL.
 *   vals_in, vals_out
 *              both NULL (keys only) or both device arrays of n uint32_t
 *              payloads; vals_out[i] is the payload of the key now at i.
 *              Same aliasing rule as the keys.
 *   begin_bit, end_bit
 *              0 <= begin_bit <= end_bit <= key width.  Only these bits are
 *              compared; (0, 32) or (0, 64) sorts whole keys.  Sorting on
 *              [0, 8(d+1)) reproduces the array after round d of PR4.
 *   algo       an rsort_algo.  RSORT_SAMPLE_REGULAR requires whole uint32 keys
 *              and uses p = 256 buckets and oversampling factor r = 32 (see
 *              rsort_sample_sort for other values).
 *   workspace, ws_bytes
 *              NULL and 0 to use the context's cached workspace (grown with
 *              hipMalloc when needed), or a device buffer of at least
 *              rsort_workspace_bytes() bytes that stays untouched by others
 *              until the sort completes on `stream`.
 */
int rsort_sort(rsort_ctx* ctx, int key_type,
               const void* keys_in, void* keys_out,
               const uint32_t* vals_in, uint32_t* vals_out,
               size_t n, int begin_bit, int end_bit, int algo,
               void* workspace, size_t ws_bytes, void* stream);

/*
 * rsort_sort with RSORT_LSD_R8 for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine) and uses as its workspace a scratch array of 64 MiB that
 * the library's code object holds on each GPU from its load until the process
 * ends.  Arguments, result and errors as in rsort_sort (algo RSORT_LSD_R8, no
 * workspace argument).  Requests whose workspace (rsort_workspace_bytes with
 * RSORT_LSD_R8) exceeds 64 MiB return RSORT_EUNSUPPORTED without enqueuing
 * anything: about 15 million uint32 keys, or 7.8 million uint32 key-value
 * pairs or uint64 keys, fit.  Every call on a GPU shares that GPU's scratch
 * array (each call initialises what it needs; nothing carries over), so calls
 * whose execution overlaps on one GPU -- other streams, other threads, other
 * contexts of the same device -- race and give wrong results: order them on
 * one stream or synchronise between them.  Kernel timing (rsort_profile_*) is
 * not recorded for this call.
 */
int rsort_sort_noalloc(rsort_ctx* ctx, int key_type,
                       const void* keys_in, void* keys_out,
                       const uint32_t* vals_in, uint32_t* vals_out,
                       size_t n, int begin_bit, int end_bit, void* stream);

/*
 * How RSORT_LSD_R8 (and RSORT_AUTO) carries out each count-sort round of
 * Section 3.2 (count the digits of each block, exchange the p x r counts so
 * that every block knows where its keys of each digit go, route the keys):
 *
 *   RSORT_PR4_COUNTED      (default) per round three kernels: per-tile digit
 *                          counts (one read of the keys), a scan of the counts
 *                          over tiles, and the routing kernel (a second read
 *                          and one write).
 *   RSORT_PR4_SINGLE_READ  32-bit keys, at most four rounds: one counting pass
 *                          before the first round (per-chunk digit counts and
 *                          the joint counts of each digit with the top bits of
 *                          the digit below it), then per round one kernel that
 *                          counts a tile, learns the keys of each digit in the
 *                          earlier tiles of its chain by a look-back over
 *                          counts the other tiles publish, and routes (one read
 *                          and one write per round).  Other requests fall back
 *                          to the counted rounds.
 *
 * Both give the same, stable result.  The choice applies to later calls on
 * ctx (it changes rsort_workspace_bytes).  Returns RSORT_EINVAL for another
 * value.
 */
enum rsort_pr4_rounds { RSORT_PR4_COUNTED = 0, RSORT_PR4_SINGLE_READ = 1 };
int rsort_set_pr4_rounds(rsort_ctx* ctx, int kind);

/*
 * The counting step of every count-sort round, for all rounds at once
 * (Section 3.2: each round first counts digit occurrences): one read of the
 * keys produces, for every digit d of the key bits [begin_bit, end_bit) taken
 * digit_bits (8 or 16) at a time from the least significant end,
 *   hist_out[d * 2^digit_bits + v] = #{ i : digit d of keys[i] == v }.
 * hist_out is a device array of ceil((end_bit - begin_bit) / digit_bits) *
 * 2^digit_bits uint32_t that the call overwrites.
 */
int rsort_histogram(rsort_ctx* ctx, int key_type, const void* keys, size_t n,
                    int digit_bits, int begin_bit, int end_bit,
                    uint32_t* hist_out, void* stream);

/*
 * Batched segmented sort: num_segs independent arrays stored back to back,
 * segment s being elements [seg_offsets[s], seg_offsets[s+1]) of the key (and
 * payload) arrays, each sorted stably on its own (the paper's SR4 applied per
 * segment, Section 3.2).  seg_offsets is a HOST array of num_segs + 1
 * nondecreasing values; elements outside [seg_offsets[0], seg_offsets[num_segs])
 * are not touched.  Keys are whole (32 or 64 bits).  Segments of at most the
 * small/large split (rsort_segmented_set_split) are sorted inside one
 * workgroup's LDS; longer ones through the tiled round kernels.  Other
 * arguments as in rsort_sort; the call reads seg_offsets before returning.
 * The call may be captured into a HIP graph: make one identical call (same
 * offsets, key type, payload presence and workspace) outside the capture
 * first; it leaves the segment plan in the workspace, which the captured
 * kernels then read at every replay.  Use a caller-owned workspace for
 * captured calls (the context's cached one is reused by later calls).
 */
int rsort_segmented_sort(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
                         const uint32_t* vals_in, uint32_t* vals_out,
                         const uint64_t* seg_offsets, size_t num_segs,
                         void* workspace, size_t ws_bytes, void* stream);

/* Workspace rsort_segmented_sort needs for these segments (host offsets). */
int rsort_segmented_workspace_bytes(rsort_ctx* ctx, int key_type, int has_vals,
                                    const uint64_t* seg_offsets, size_t num_segs, size_t* bytes);

/*
 * The batched segmented sort with the segment offsets in DEVICE memory
 * (num_segs + 1 nondecreasing uint32_t, offsets[num_segs] <= total_n; the key
 * and payload arrays hold total_n elements).  Nothing is read back to the host:
 * one planning kernel classifies the segments on the device, so the call can
 * be captured in a HIP graph without a preceding eager call (with a
 * caller-owned workspace of rsort_segmented_device_workspace_bytes()).  Offsets
 * that decrease or end beyond total_n leave the arrays untouched and make the
 * next rsort_synchronize on ctx return RSORT_EDEVICE.  Other arguments as in
 * rsort_segmented_sort.
 */
int rsort_segmented_sort_device(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
                                const uint32_t* vals_in, uint32_t* vals_out,
                                const uint32_t* seg_offsets, size_t num_segs, size_t total_n,
                                void* workspace, size_t ws_bytes, void* stream);

/* Workspace rsort_segmented_sort_device needs (depends on the counts only). */
int rsort_segmented_device_workspace_bytes(rsort_ctx* ctx, int key_type, int has_vals,
                                           size_t num_segs, size_t total_n, size_t* bytes);

/* Tile of the large segments' tiled rounds: the workgroup size of the count
 * and scatter kernels, 256, 512 or 1024 threads (16 keys per thread for
 * 32-bit keys, 8 for 64-bit ones: tiles of 4096 / 8192 / 16384 or 2048 /
 * 4096 / 8192 keys); 0 restores the default, 512.  Chosen by the tuner;
 * applies to later calls on ctx.  RSORT_EINVAL for other values. */
int rsort_segmented_set_tile(rsort_ctx* ctx, int tile_threads);

/*
 * How the segmented sort with host offsets (rsort_segmented_sort) is launched:
 *   RSORT_SEG_ROUNDS      the small segments' in-LDS sorts, then per round of
 *                         the large segments a count, a per-segment scan and
 *                         a scatter kernel (default);
 *   RSORT_SEG_PERSISTENT  one persistent launch (after a fill kernel that
 *                         clears its counters): a cooperative launch whose
 *                         resident grid goes through phases separated by
 *                         grid-wide barriers -- the whole small segments (at
 *                         most 8192 32-bit or 4096 64-bit keys, radix rounds)
 *                         beside round 0's tile counts of the large segments,
 *                         then per round the tile counts, the per-segment
 *                         output starts (and, first, the per-segment round
 *                         plans) and the tiles' stable counting rounds.  Every
 *                         barrier wait is bounded (a wait that gives up is
 *                         reported by rsort_synchronize as RSORT_EDEVICE).  It
 *                         is not captured into a graph (RSORT_EUNSUPPORTED
 *                         inside a capture).
 * Same result either way (Section 3.2's SR4 on every segment).  Chosen by the
 * tuner; applies to later calls on ctx.  RSORT_EINVAL for other values.
 */
enum rsort_seg_launch { RSORT_SEG_ROUNDS = 0, RSORT_SEG_PERSISTENT = 1 };
int rsort_segmented_set_launch(rsort_ctx* ctx, int launch);

/* The segmented sort's current configuration on ctx: the small/large split,
 * the small-segment sorter, the tile workgroup size of the large path, the
 * radix width in bits of every count-sort round (8: the rounds of the
 * segmented sort are the paper's radix-2^8 rounds; a wider radix has no tile
 * that fits LDS with per-group ranking slots) and the launch mode
 * (rsort_seg_launch; the persistent launch always reports the radix sorter
 * and 512-thread tiles).  Any output may be NULL. */
int rsort_segmented_get_config(rsort_ctx* ctx, uint32_t* small_max, int* small_sort,
                               int* tile_threads, int* radix_bits, int* launch);

/* Largest segment sorted whole in LDS (<= 8192; 0 sends every segment through
 * the tiled path).  Chosen by the tuner; applies to later calls on ctx. */
int rsort_segmented_set_split(rsort_ctx* ctx, uint32_t small_max);

/*
 * Sorter of the segments sorted whole in LDS by the segmented sorts on ctx
 * (both entry points):
 *   RSORT_SMALL_RADIX  one stable count-sort round per byte in LDS (default);
 *   RSORT_SMALL_BTN    the paper's BTN (Section 2): each of P threads sorts a
 *                      run of R (key, position) composites, then the runs are
 *                      ordered by the lg P (lg P + 1) / 2 stages of a bitonic
 *                      sorter whose comparisons merge two runs and split them
 *                      into the lower and upper half;
 *   RSORT_SMALL_OET    the paper's OET: the same runs ordered by P rounds of
 *                      odd-even transposition with the same merge-split.
 * All three give the stable sort.  BTN and OET apply to 32-bit keys in
 * segments of up to 4096 keys (P x R = 256 x 4 or 512 x 8); other small
 * segments use the radix rounds.  RSORT_EINVAL for another value.
 */
enum rsort_small_sort { RSORT_SMALL_RADIX = 0, RSORT_SMALL_BTN = 1, RSORT_SMALL_OET = 2 };
int rsort_segmented_set_small_sort(rsort_ctx* ctx, int small_sort);
int rsort_segmented_get_small_sort(rsort_ctx* ctx, int* small_sort);

/* Tuner for the segmented sort: sorts the given batch (into keys_out /
 * vals_out) reps times with each candidate split (0, 1024, 4096, 8192 keys),
 * each small-segment sorter and each tile workgroup of the large path (256,
 * 512, 1024 threads), and the persistent launch at each split, keeps the
 * fastest combination on ctx and returns its split (the rest:
 * rsort_segmented_get_config), with its time per sort in ms.
 * Synchronises the stream. */
int rsort_segmented_tune(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
                         const uint32_t* vals_in, uint32_t* vals_out,
                         const uint64_t* seg_offsets, size_t num_segs, int reps, void* stream,
                         uint32_t* best_split, double* best_ms);

/*
 * Tune cache of ctx: a text file (path copied; NULL or "" for none) of one
 * JSON object per line, each a choice of rsort_segmented_tune keyed by the GPU
 * architecture (e.g. gfx950), the key type, whether payloads move and the
 * batch's size class (ceil(log2) of its total keys and of its segment count).
 * With a cache set, rsort_segmented_tune first looks the batch's key up: on a
 * hit (the last line with that key wins) it applies that choice, sorts the
 * batch once with it and returns the stored split and time instead of tuning;
 * otherwise it tunes and appends the choice.  Lines that do not parse, or
 * choices this library version cannot apply, are ignored, and a file that cannot be
 * written is not an error: tuning simply happens again.  A new context takes
 * the path in the environment variable RSORT_TUNE_CACHE, if set.
 */
int rsort_set_tune_cache(rsort_ctx* ctx, const char* path);

/*
 * Test hook for the out-of-memory paths: the k-th device allocation the
 * library makes from now on (workspaces, error words, descriptor buffers; any
 * context or server in the process) fails as out of memory, and the call that
 * needed it returns RSORT_ENOMEM; k = 0 disarms the hook.  RSORT_FAULT_ALLOC=k
 * in the environment arms it when the library first allocates.  RSORT_EINVAL
 * for k < 0.
 */
int rsort_debug_fail_alloc(int k);

/*
 * Deterministic regular-oversampling sample sort, GSD (Section 3.3,
 * Algorithm 1), of n uint32 keys (key_type must be RSORT_U32), stable, with
 * an optional payload.
 *
 *   p   number of blocks and of buckets, 1 <= p <= 1024 (clamped to n).  The
 *       keys are cut into blocks k = [floor(kn/p), floor((k+1)n/p)), each
 *       block is stable-sorted, and s = r p keys at positions
 *       ceil(j N_k / s) - 1 (j = 1..s, N_k the block length) form its regular
 *       sample.  The p s sample keys, ordered as composites (key, input index),
 *       give the splitters S_i = sample element i s - 1 (i = 1..p-1); block k
 *       is split at bnd[k][i] = #{q in block k : (key_q, index_q) <= S_i} and
 *       bucket j collects the runs [bnd[k][j], bnd[k][j+1]) of all blocks in
 *       block order.  Buckets are then stable-sorted, which yields the same
 *       array as the paper's p-way merge of each bucket.
 *   r   oversampling factor, r >= 1, with r p^2 <= 2^26.
 * Comparing composites makes the bucket bound of Lemma 1,
 * |bucket| <= (1 + 1/r) n/p + r p, hold for any keys, duplicates included.
 * Other arguments as in rsort_sort (whole keys only).  The split of the last
 * run is kept on the context for rsort_sample_sort_stats.  No host traffic
 * is enqueued, so the call can be captured in a HIP graph once an eager call
 * on the same context has run (it allocates the statistics area).
 */
int rsort_sample_sort(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
                      const uint32_t* vals_in, uint32_t* vals_out, size_t n, int p, int r,
                      void* workspace, size_t ws_bytes, void* stream);

/* Workspace rsort_sample_sort needs for (n, p, r, payload). */
int rsort_sample_sort_workspace_bytes(rsort_ctx* ctx, int key_type, int has_vals, size_t n,
                                      int p, int r, size_t* bytes);

/*
 * Random-oversampling sample sort, GER (Section 3.3, Algorithm 2): the GSD
 * skeleton above with a different step 2.  The sample is s p - 1 keys drawn
 * uniformly at random, with replacement, from the locally sorted blocks: draw i
 * is position ((SplitMix64 value i of stream `seed`) >> 32) * n >> 32 of the
 * concatenated blocks, SplitMix64 being the counter-based generator of Steele,
 * Lea and Flood (value i = mix(seed + (i + 1) * 0x9E3779B97F4A7C15)).  The
 * sample is ordered by (key, position) and splitter i is its (i s)-th smallest
 * element; split, route and the stable finish are as in GSD, so the result is
 * again the stable sort.  s = 0 selects s = 2 w^2 lg n with w = ceil(lg lg n)
 * (the paper's s = 2 w_n^2 lg n); s p <= 2^26.  Bucket sizes are bounded with
 * high probability (Lemma 2), not deterministically.  The statistics call
 * reports the split of the last sample sort of any kind.
 */
int rsort_sample_sort_random(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
                             const uint32_t* vals_in, uint32_t* vals_out, size_t n, int p, int s,
                             uint64_t seed, void* workspace, size_t ws_bytes, void* stream);

/* Workspace rsort_sample_sort_random needs for (n, p, s, payload). */
int rsort_sample_sort_random_workspace_bytes(rsort_ctx* ctx, int key_type, int has_vals, size_t n,
                                             int p, int s, size_t* bytes);

/*
 * Random-oversampling sample sort that samples before sorting, GVR (Section
 * 3.3, Algorithm 3).  The input is cut into p blocks as in GSD but not sorted
 * first.  s p - 1 positions of the INPUT are drawn exactly as in GER (same
 * generator, same seed semantics, here indexing the input), the keys there are
 * ordered by (key, input index) and splitter i is the (i s)-th smallest of
 * them.  Every element goes to the bucket counted by the splitters below its
 * (key, input index) -- a binary search over the splitters -- and is moved
 * there by a stable count sort on the bucket index, so bucket j is X_{0,j}
 * ... X_{p-1,j} with each X_{k,j} in input order; then every bucket is
 * stable-sorted.  The result is the stable sort.  s = 0 selects s = 2 w^2 lg n
 * as for GER; 1 <= p <= 256 (one 8-bit routing digit), s p <= 2^26.  The
 * statistics call reports cnt[k][j] for the input blocks k.  Same pointer,
 * overlap, workspace, stream and error rules as rsort_sort.
 */
int rsort_sample_sort_gvr(rsort_ctx* ctx, int key_type, const void* keys_in, void* keys_out,
                          const uint32_t* vals_in, uint32_t* vals_out, size_t n, int p, int s,
                          uint64_t seed, void* workspace, size_t ws_bytes, void* stream);

/* Workspace rsort_sample_sort_gvr needs for (n, p, s, payload). */
int rsort_sample_sort_gvr_workspace_bytes(rsort_ctx* ctx, int key_type, int has_vals, size_t n,
                                          int p, int s, size_t* bytes);

/*
 * Split statistics of the last sample sort on ctx (waits for the device).
 * *p_used receives the number of buckets; each non-NULL HOST array must hold
 * p_cap >= *p_used (or p_cap^2 for cnt) entries:
 *   cnt[k * p_used + j]  |X_{k,j}|, keys of block k routed to bucket j;
 *   bucket[j]            |Y_j|, the size of bucket j;
 *   split_key[i - 1], split_index[i - 1]
 *                        the splitter S_i as (key, input index), i = 1..p_used-1.
 * RSORT_EINVAL if no sample sort has run on ctx or p_cap is too small.
 */
int rsort_sample_sort_stats(rsort_ctx* ctx, int p_cap, int* p_used, uint32_t* cnt,
                            uint32_t* bucket, uint32_t* split_key, uint32_t* split_index);

/*
 * Sort server: a request loop with continuous batching over the sorts above.
 * Requests are device-resident key arrays (keys only, uint32 or uint64, whole
 * keys); each is sorted stably from keys_in into keys_out (equal pointers sort
 * in place).  A scheduling thread owned by the server admits requests in
 * arrival order onto num_streams streams while the summed HBM footprint of
 * the requests in flight (their key buffers plus workspace) stays within
 * hbm_cap_bytes; requests arriving while others run are admitted as streams
 * and memory free up, so they overlap on the device.  Small requests (at most
 * 8192 keys) of one key type that are waiting together are sorted by one
 * launch, one workgroup each, whole in LDS; larger ones run alone through the
 * radix-2^8 sort.  Each result equals the stable sort of that request's keys
 * regardless of what else is in flight; a request whose sort hits a device-side
 * failure completes with RSORT_EDEVICE.  The caller keeps the buffers alive and
 * untouched until the request completes.
 */
typedef struct rsort_server rsort_server;

/* Create a server on HIP device hip_device with 1..64 streams.  Starts its
 * scheduling thread. */
int rsort_server_create(int hip_device, size_t hbm_cap_bytes, int num_streams,
                        rsort_server** out);

/* Queue one sort (thread-safe).  *ticket identifies it.  The sort starts only
 * after all work enqueued on `stream` (a hipStream_t of the server's device,
 * NULL = the null stream) before this call: the writes of keys_in and any
 * earlier use of keys_out may still be in flight there.  Work enqueued on
 * `stream` later is not ordered with the sort: wait for the ticket before
 * reading keys_out.  RSORT_ENOMEM if the request's footprint alone exceeds the
 * cap; RSORT_EINVAL for host pointers or partially overlapping buffers;
 * RSORT_EBUSY once destruction has begun; RSORT_EDEVICE if the stream point
 * cannot be recorded. */
int rsort_server_submit_async(rsort_server* sv, int key_type, const void* keys_in,
                              void* keys_out, size_t n, void* stream, uint64_t* ticket);

/* rsort_server_submit_async on the null stream. */
int rsort_server_submit(rsort_server* sv, int key_type, const void* keys_in, void* keys_out,
                        size_t n, uint64_t* ticket);

/* Allocate now, on the calling thread, the workspace that requests of up to
 * max_n keys of key_type need on every stream slot, so that the scheduling
 * thread allocates nothing for them (larger requests still grow a slot's
 * workspace when they start).  Call while no request is queued or running
 * (RSORT_EBUSY otherwise); RSORT_ENOMEM if the device memory is not there. */
int rsort_server_reserve(rsort_server* sv, int key_type, size_t max_n);

/* Test hook for the failure path: the next request that runs through the
 * radix path (more than 8192 keys) has its slot's device error word set after
 * its sort, exactly as a look-back wait that gave up would set it, so that it
 * completes with RSORT_EDEVICE (poll / wait return it).  No kernel faults. */
int rsort_server_fail_next(rsort_server* sv);

/* HBM accounting: the summed footprint of the requests in flight now, its
 * maximum since creation or the last rsort_server_reset_stats, and the device
 * memory the server itself holds (slot workspaces, descriptors).  Any output
 * pointer may be NULL. */
int rsort_server_memory(rsort_server* sv, size_t* in_flight, size_t* max_in_flight,
                        size_t* reserved);

/* *done = 1 once the result is in keys_out (then returns the request's
 * status), else 0 and RSORT_OK.  Thread-safe. */
int rsort_server_poll(rsort_server* sv, uint64_t ticket, int* done);

/* Block until the request completes; returns its status.  Thread-safe. */
int rsort_server_wait(rsort_server* sv, uint64_t ticket);

/* Submit-to-completion latency percentiles (nearest rank, microseconds) over
 * the requests completed since creation or the last reset, the number of
 * such requests, and their keys per second of wall time from the first
 * submission to the last completion.  Any output pointer may be NULL. */
int rsort_server_latency(rsort_server* sv, double* p50_us, double* p99_us, double* keys_per_s,
                         uint64_t* completed);

/* Forget the latency statistics and the tickets of completed requests. */
int rsort_server_reset_stats(rsort_server* sv);

/* Finish every queued and running request, stop the thread, free the server. */
int rsort_server_destroy(rsort_server* sv);

/* Wait for `stream`, then report any device-side failure recorded by this
 * context's kernels since the last call (RSORT_EDEVICE) and clear it. */
int rsort_synchronize(rsort_ctx* ctx, void* stream);

/* Kernel timing for measurement.  While enabled, every sort on ctx records a
 * HIP event on its stream immediately before and after each kernel of the
 * timed kinds below; enabling (or disabling) resets the totals.  enable: 0
 * disables, otherwise a bit mask of the kinds to time (bit 1 << kind; -1 times
 * every kind).  Each event pair delays the stream by a few microseconds, so
 * time only the kinds you read. */
enum rsort_kernel_kind {
    RSORT_KERNEL_ROUND = 0,     /* rank-and-scatter kernel of a count-sort round  */
    RSORT_KERNEL_HIST = 1,      /* all-rounds digit counting before the rounds    */
    RSORT_KERNEL_COUNT = 2,     /* per-tile digit counts of a round               */
    RSORT_KERNEL_TILESCAN = 3,  /* exclusive scan of the tile counts of a round
                                   (none in radix-2^8 sorts of at most 256 tiles,
                                   whose scatter sums the tile counts itself)   */
    RSORT_KERNEL_SMALL = 4,     /* whole-segment in-LDS sorts (segmented sort)    */
    RSORT_KERNEL_GROUP = 5      /* high-byte grouping pass of a radix-2^16 round  */
};
int rsort_profile_enable(rsort_ctx* ctx, int enable);

/* Waits for the recorded events and returns, for one rsort_kernel_kind, how
 * many launches were timed since profiling was enabled and their summed
 * durations in milliseconds. */
int rsort_profile_read(rsort_ctx* ctx, int kind, uint64_t* launches, double* total_ms);

/* Time only every `period`-th launch of each timed kind: launches 0, period,
 * 2 period, ... of that kind since profiling was enabled (period 1, the
 * default, times them all).  Fewer event pairs delay the stream less; a period
 * coprime with a sort's launches of the kind (5 against the 4 count-sort
 * rounds of 32-bit keys) still samples every round equally often.  Returns
 * RSORT_EINVAL when profiling is not enabled or period is 0; enabling again
 * resets the period to 1. */
int rsort_profile_set_period(rsort_ctx* ctx, uint32_t period);

#ifdef __cplusplus
}
#endif

#endif /* RSORT_H */
