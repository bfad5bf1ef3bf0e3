// Deterministic regular-oversampling sample sort (GSD, arXiv 1808.10292
// Section 3.3, Algorithm 1) for 32-bit keys with an optional 32-bit payload,
// and its random-oversampling sibling GER (Algorithm 2), which differs only in
// step 2: s p - 1 sample keys drawn uniformly at random (with replacement)
// from the locally sorted blocks, sorted by (key, position).
//
//   1. local sort     the n keys are cut into p near-equal blocks
//                     (block k = [floor(kn/p), floor((k+1)n/p))) and every block
//                     is stable-sorted: the device-planned segmented radix sort;
//   2. sample         s = r p keys per sorted block at positions ceil(j N_k/s)-1,
//                     j = 1..s (the last one is the block maximum), each kept as
//                     the composite (key, global index);
//   3. sort sample    the p s composites by key with the stable LSD sort; the
//                     sample is laid out in block order, so equal keys already
//                     sit in index order and the result is sorted by composite;
//   4. splitters      S_i = sorted sample element i s - 1, i = 1..p-1;
//   5. split          every block is split around the splitters by binary search:
//                     bnd[k][i] = #{q in block k : (X_q, index) <= S_i};
//   6. route          runs X_{k,j} = block k between bnd[k][j] and bnd[k][j+1]
//                     are copied to bucket j, buckets in order, runs of one
//                     bucket in block order;
//   7. finish         every bucket is stable-sorted (device-planned segmented
//                     sort).  Bucket j holds exactly the keys between S_j and
//                     S_{j+1} as composites, so the concatenation is the stable
//                     sort of the input; the paper merges the p sorted runs of
//                     a bucket, which gives the same array.
// With p <= 256, GSD replaces steps 5-7 by the merge of step 5 itself: the
// buckets are cut further at every g-th sorted sample element into pieces of
// about 2048 keys, and one workgroup merges the p sorted sub-runs of a piece
// straight from the sorted blocks into the output (see k_gsd_merge).
// Duplicate keys: comparing composites (key, index) instead of keys keeps the
// bucket bound of Lemma 1 for any key distribution, and the split of equal
// keys by index keeps the result stable.
//
// GVR (Algorithm 3) samples before any sorting: s p - 1 input positions drawn
// as in GER, the keys there ordered by (key, input index), splitters picked
// the same way.  Each input element then finds its bucket (the number of
// splitters below its composite) by binary search, and one stable count-sort
// round on the bucket index -- per-tile bucket counts, the device-wide tile
// scan of the radix rounds, a rank-and-scatter -- moves the unsorted input
// into bucket order (X_{k,j} for k = 0..p-1 concatenated is bucket j).  The
// finish sorts every bucket as above.  p <= 256: one 8-bit routing digit.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "lsd_kernels.h"
#include "tile_sort.h"

namespace rsort {
namespace {

constexpr uint32_t kRouteWG = 256;
constexpr uint32_t kRouteItems = 16;
constexpr uint32_t kRouteTile = kRouteWG * kRouteItems;   // keys per route workgroup
constexpr uint32_t kScanCols = 64;                        // bucket columns per scan workgroup
constexpr uint32_t kScanGroups = 16;                      // block groups per column

// dst[0 .. count) = value.
__global__ void k_fill_u32(uint32_t* dst, uint32_t count, uint32_t value)
{
    for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) dst[i] = value;
}

// lo[k] = floor(k n / p), k = 0..p.
__global__ void k_gsd_blocks(uint32_t* lo, uint32_t n, uint32_t p)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k <= p) lo[k] = (uint32_t)(((uint64_t)k * n) / p);
}

// Regular sample of the sorted blocks: element t = k s + j - 1.
// The merge's boundary sample: s per block as well, but block k's j-th
// element at position floor((j p - k - 1) N_k / (s p)), j = 1..s, i.e. the
// regular positions shifted back by (k + 1) / p of a sample interval.  With
// unshifted positions the j-th elements of all blocks sit at the same rank in
// their blocks and, for blocks of similar keys, cluster in value near both
// ends of the key range, leaving pieces of many block keys between clusters;
// shifted, they spread over the interval.  Written in block order, positions
// increasing, so a stable sort by key orders the composites.
__global__ void k_merge_sample(const uint32_t* __restrict__ X, const uint32_t* lo, uint32_t p,
                               uint32_t s, uint32_t* Tk, uint32_t* Tg)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)p * s) return;
    const uint32_t k = (uint32_t)(t / s);
    const uint64_t j = t - (size_t)k * s + 1;
    const uint32_t b = lo[k];
    const uint64_t nk = lo[k + 1] - b;
    const uint32_t q = (uint32_t)(((j * p - k - 1) * nk) / ((uint64_t)s * p));
    Tk[t] = X[b + q];
    Tg[t] = b + q;
}

__global__ void k_gsd_sample(const uint32_t* __restrict__ X, const uint32_t* lo, uint32_t p,
                             uint32_t s, uint32_t* Tk, uint32_t* Tg)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)p * s) return;
    const uint32_t k = (uint32_t)(t / s);
    const uint64_t j = t - (size_t)k * s + 1;
    const uint32_t b = lo[k];
    const uint64_t nk = lo[k + 1] - b;
    const uint32_t q = (uint32_t)((j * nk + s - 1) / s - 1);
    Tk[t] = X[b + q];
    Tg[t] = b + q;
}

// GER (Algorithm 2) step 2: draw i of the random sample is the position
// ((SplitMix64 value i of stream seed) >> 32) * n >> 32, uniform in [0, n)
// with replacement.  SplitMix64 (Steele, Lea, Flood 2014) used counter-based:
// value i = mix(seed + (i + 1) * golden gamma).
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_ger_draw(uint64_t seed, uint32_t n, size_t m, uint32_t* pos)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    pos[i] = (uint32_t)(((splitmix64_at(seed, i) >> 32) * (uint64_t)n) >> 32);
}

// Sample composites (key, position) in position order.
__global__ void k_ger_gather(const uint32_t* __restrict__ X, const uint32_t* pos_sorted, size_t m,
                             uint32_t* Tk, uint32_t* Tg)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint32_t q = pos_sorted[i];
    Tk[i] = X[q];
    Tg[i] = q;
}

// Composite order (key, index).
__device__ __forceinline__ bool comp_less(uint32_t ak, uint32_t ag, uint32_t bk, uint32_t bg)
{
    return ak < bk || (ak == bk && ag < bg);
}

// bnd[k][i] for k < p, i <= p; splitter copies for the statistics.
__global__ void k_gsd_split(const uint32_t* __restrict__ X, const uint32_t* lo, uint32_t p,
                            uint32_t s, const uint32_t* Sk, const uint32_t* Sg, uint32_t* bnd,
                            uint32_t* split_key, uint32_t* split_g)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p * (p + 1)) return;
    const uint32_t k = t / (p + 1), i = t - k * (p + 1);
    const uint32_t b = lo[k], nk = lo[k + 1] - b;
    uint32_t res;
    if (i == 0) {
        res = 0;
    } else if (i == p) {
        res = nk;
    } else {
        const uint32_t sk = Sk[(size_t)i * s - 1], sg = Sg[(size_t)i * s - 1];
        if (k == 0) {
            split_key[i - 1] = sk;
            split_g[i - 1] = sg;
        }
        uint32_t a = 0, e = nk;   // first q with S_i < (X_q, b + q)
        while (a < e) {
            const uint32_t mid = a + ((e - a) >> 1);
            if (comp_less(sk, sg, X[b + mid], b + mid))
                e = mid;
            else
                a = mid + 1;
        }
        res = a;
    }
    bnd[t] = res;
}

// Within-bucket offsets: off[k][j] = sum over k' < k of |X_{k',j}|, and the
// bucket sizes.  Workgroup c covers columns [64c, 64c+64); thread (g, col)
// sums the run lengths of its block group, the 16 group sums of a column are
// scanned in LDS, and each thread writes the offsets of its group.
__global__ __launch_bounds__(kScanCols * kScanGroups) void k_gsd_colscan(const uint32_t* bnd,
                                                                         uint32_t p, uint32_t* off,
                                                                         uint32_t* bsize)
{
    __shared__ uint32_t part[kScanGroups][kScanCols];
    const uint32_t col = threadIdx.x % kScanCols, g = threadIdx.x / kScanCols;
    const uint32_t j = blockIdx.x * kScanCols + col;
    const uint32_t per = (p + kScanGroups - 1) / kScanGroups;
    const uint32_t k0 = min(p, g * per), k1 = min(p, k0 + per);
    uint32_t sum = 0;
    if (j < p)
        for (uint32_t k = k0; k < k1; ++k) {
            const uint32_t* row = bnd + (size_t)k * (p + 1);
            sum += row[j + 1] - row[j];
        }
    part[g][col] = sum;
    __syncthreads();
    uint32_t run = 0, total = 0;
    for (uint32_t h = 0; h < kScanGroups; ++h) {
        const uint32_t v = part[h][col];
        run += h < g ? v : 0u;
        total += v;
    }
    if (j >= p) return;
    if (g == 0) bsize[j] = total;
    for (uint32_t k = k0; k < k1; ++k) {
        const uint32_t* row = bnd + (size_t)k * (p + 1);
        off[(size_t)k * p + j] = run;
        run += row[j + 1] - row[j];
    }
}

// Bucket starts boff[j] = sum of bucket sizes before j, boff[p] = n.
__global__ __launch_bounds__(1024) void k_gsd_bucket_starts(const uint32_t* bsize, uint32_t p,
                                                            uint32_t* boff)
{
    __shared__ uint32_t wsum[16];
    __shared__ uint32_t carry;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (uint32_t c = 0; c < p; c += 1024) {
        const uint32_t j = c + tid;
        const uint32_t x = j < p ? bsize[j] : 0u;
        const uint32_t incl = wave_inclusive_sum(x);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t before = carry, all = 0;
        for (uint32_t w = 0; w < 16; ++w) {
            before += w < wave ? wsum[w] : 0u;
            all += wsum[w];
        }
        if (j < p) boff[j] = before + incl - x;
        __syncthreads();
        if (tid == 0) carry += all;
        __syncthreads();
    }
    if (tid == 0) boff[p] = carry;
}

// Route: workgroup (k, t) copies keys [t T, (t+1) T) of sorted block k.  The
// key at block offset u belongs to the run j with bnd[k][j] <= u < bnd[k][j+1]
// and lands at boff[j] + off[k][j] + u - bnd[k][j].  The runs met by the
// workgroup's range are found once, each key searches only among them.
template <bool KV>
__global__ __launch_bounds__(kRouteWG) void k_gsd_route(const uint32_t* __restrict__ X,
                                                        const uint32_t* __restrict__ XV,
                                                        const uint32_t* lo, uint32_t n,
                                                        uint32_t p, uint32_t tiles_per_block,
                                                        const uint32_t* bnd, const uint32_t* off,
                                                        const uint32_t* boff, uint32_t* Y,
                                                        uint32_t* YV)
{
    __shared__ uint32_t sb[1025];
    __shared__ uint32_t sd[1024];
    __shared__ uint32_t jr[2];
    const uint32_t k = blockIdx.x / tiles_per_block;
    const uint32_t t = blockIdx.x - k * tiles_per_block;
    const uint32_t b = lo[k], nk = lo[k + 1] - b;
    const uint32_t u0 = t * kRouteTile;
    if (u0 >= nk) return;
    const uint32_t u1 = min(nk, u0 + kRouteTile);
    const uint32_t* row = bnd + (size_t)k * (p + 1);
    // the run of the first and of the last key: last j with bnd[j] <= u
    if (threadIdx.x < 2) {
        const uint32_t u = threadIdx.x == 0 ? u0 : u1 - 1;
        uint32_t a = 0, e = p;   // search j in [0, p): bnd[0] = 0 <= u always
        while (e - a > 1) {
            const uint32_t mid = (a + e) >> 1;
            if (row[mid] <= u) a = mid; else e = mid;
        }
        jr[threadIdx.x] = a;
    }
    __syncthreads();
    const uint32_t j0 = jr[0], j1 = jr[1];
    for (uint32_t j = j0 + threadIdx.x; j <= j1 + 1; j += kRouteWG) sb[j - j0] = row[j];
    for (uint32_t j = j0 + threadIdx.x; j <= j1; j += kRouteWG)
        sd[j - j0] = boff[j] + off[(size_t)k * p + j] - row[j];
    __syncthreads();
    const uint32_t nr = j1 - j0 + 1;
    // the tile's keys (and payloads) loaded together, then each routed
    uint32_t kx[kRouteItems], vx[KV ? kRouteItems : 1];
#pragma unroll
    for (uint32_t i = 0; i < kRouteItems; ++i) {
        const uint32_t u = u0 + i * kRouteWG + threadIdx.x;
        kx[i] = u < u1 ? X[b + u] : 0u;
        if (KV) vx[i] = u < u1 ? XV[b + u] : 0u;
    }
#pragma unroll
    for (uint32_t i = 0; i < kRouteItems; ++i) {
        const uint32_t u = u0 + i * kRouteWG + threadIdx.x;
        if (u >= u1) break;
        uint32_t a = 0, e = nr;   // last local run with sb[a] <= u
        while (e - a > 1) {
            const uint32_t mid = (a + e) >> 1;
            if (sb[mid] <= u) a = mid; else e = mid;
        }
        const uint32_t d = sd[a] + u;
        if (d < n) {   // always true when the split is consistent
            Y[d] = kx[i];
            if (KV) YV[d] = vx[i];
        }
    }
}

// ---------------------------------------------------------------------------
// GVR route.  Route tile t covers keys [t' T, min(N_k, (t'+1) T)) of input
// block k = t / tpb (t' = t mod tpb); tiles past a block's end are empty.
constexpr uint32_t kGvrWG = 512;
constexpr uint32_t kGvrItems = 16;
constexpr uint32_t kGvrTile = kGvrWG * kGvrItems;
constexpr uint32_t kGvrGroups = kGvrWG / 32;   // ranking groups of 32 lanes
constexpr uint32_t kGvrTabBits = 12;            // bucket-search table over the top key bits
constexpr uint32_t kGvrTab = 1u << kGvrTabBits;

__device__ __forceinline__ uint2 gvr_tile(const uint32_t* lo, uint32_t tpb, uint32_t t)
{
    const uint32_t k = t / tpb, u0 = (t - k * tpb) * kGvrTile;
    const uint32_t b = lo[k], nk = lo[k + 1] - b;
    return make_uint2(b + u0, u0 < nk ? min(kGvrTile, nk - u0) : 0u);
}

// Round plan {exec = 1}, ticket and look-back words of the route's tile scan.
__global__ void k_gvr_init(RoundPlan* plan, uint32_t* ticket, uint32_t* state, size_t words)
{
    const size_t g = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) {
        *plan = RoundPlan{1, 0, 1, 1};
        *ticket = 0;
    }
    for (size_t i = g; i < words; i += (size_t)gridDim.x * blockDim.x) state[i] = 0;
}

// Search table: tab[c] = number of splitters whose key's top 12 bits are
// below c, c = 0..4096.  A key with top bits c has exactly tab[c] splitters
// with smaller keys and at least the splitters from tab[c + 1] on above it, so
// only splitters tab[c] .. tab[c+1]-1 need comparing (none, mostly, for
// spread-out keys).  One workgroup: a histogram of the splitters' top bits
// and its exclusive scan (values <= 255: p <= 256).
__global__ __launch_bounds__(1024) void k_gvr_table(const uint32_t* Sk, uint32_t p, uint32_t s,
                                                    uint8_t* tab)
{
    __shared__ uint32_t hc[kGvrTab];
    __shared__ uint32_t wsum[16];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (uint32_t c = tid; c < kGvrTab; c += 1024) hc[c] = 0;
    __syncthreads();
    if (tid + 1 < p) atomicAdd(&hc[Sk[(size_t)(tid + 1) * s - 1] >> (32 - kGvrTabBits)], 1u);
    __syncthreads();
    // thread tid owns entries 4 tid .. 4 tid + 3
    uint32_t c4[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        c4[q] = hc[4 * tid + q];
        sum += c4[q];
    }
    const uint32_t incl = wave_inclusive_sum(sum);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (uint32_t w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        tab[4 * tid + q] = (uint8_t)run;
        run += c4[q];
    }
    if (tid == 1023) tab[kGvrTab] = (uint8_t)run;
}

// Bucket of every key of the tile: the number of splitters S_i below its
// composite (key, input index), by binary search over the splitters in LDS;
// written as one byte per key, and counted per tile (counts[t][v], v < 256).
// Thread layout: key (q WG + tid) 4 + c, c < 4, so each group of 4 is one
// 16-byte load (aligned full tiles) and one 4-byte store of bucket bytes; the
// 16 searches of a thread advance together, one LDS probe each per step.
// The tile's key minimum and maximum go to tmm[t] and tmm[ntiles + t] (an
// empty tile writes 2^32 - 1 and 0).
__global__ __launch_bounds__(kGvrWG) void k_gvr_count(const uint32_t* __restrict__ X,
                                                      const uint32_t* lo, uint32_t p, uint32_t s,
                                                      uint32_t tpb, const uint32_t* Sk,
                                                      const uint32_t* Sg, const uint8_t* gtab,
                                                      uint8_t* bkt, uint32_t* counts,
                                                      uint32_t* tmm)
{
    constexpr int ITEMS = kGvrItems;
    __shared__ uint2 spl[kGvrMaxP];
    __shared__ uint2 wmm[kGvrWG / 64];
    __shared__ uint32_t h[R * 32];
    __shared__ uint32_t tabw[(kGvrTab + 4) / 4];
    uint8_t* tab = (uint8_t*)tabw;
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < R * 32 / 4; i += kGvrWG) ((uint4*)h)[i] = make_uint4(0, 0, 0, 0);
    if (tid + 1 < p) spl[tid] = make_uint2(Sk[(size_t)(tid + 1) * s - 1], Sg[(size_t)(tid + 1) * s - 1]);
    {
        // the table (4097 bytes, 4100 allocated) as words, all loads first
        constexpr uint32_t W = (kGvrTab + 4) / 4, PER = (W + kGvrWG - 1) / kGvrWG;
        const uint32_t* g4 = (const uint32_t*)gtab;
        uint32_t t4[PER];
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) t4[j] = j * kGvrWG + tid < W ? g4[j * kGvrWG + tid] : 0u;
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j)
            if (j * kGvrWG + tid < W) tabw[j * kGvrWG + tid] = t4[j];
    }
    const uint32_t t = xcd_tile(gridDim.x);
    const uint2 tr = gvr_tile(lo, tpb, t);
    const uint32_t base = tr.x, len = tr.y;
    const bool vec = len == kGvrTile && (base & 3) == 0 && ((uintptr_t)(X + base) & 15) == 0;
    uint32_t key[ITEMS];
    if (vec) {
        typedef uint32_t v4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int q = 0; q < ITEMS / 4; ++q) {
            const v4 x = __builtin_nontemporal_load((const v4*)(X + base) + q * kGvrWG + tid);
            key[4 * q] = x.x; key[4 * q + 1] = x.y; key[4 * q + 2] = x.z; key[4 * q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t u = ((i >> 2) * kGvrWG + tid) * 4 + (i & 3);
            key[i] = u < len ? X[base + u] : 0u;
        }
    }
    {
        uint32_t kmin = ~0u, kmax = 0u;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t u = ((i >> 2) * kGvrWG + tid) * 4 + (i & 3);
            if (u < len) {
                kmin = min(kmin, key[i]);
                kmax = max(kmax, key[i]);
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, o, 64));
            kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, o, 64));
        }
        if ((tid & 63) == 0) wmm[tid >> 6] = make_uint2(kmin, kmax);
    }
    __syncthreads();
    // b[i] = number of splitters below key i: binary search of the splitters
    // the table leaves open, [b, e); every open range shrinks each step, and
    // ranges hold at most 255 splitters, so 8 steps close all of them
    uint32_t b[ITEMS], e[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t c = key[i] >> (32 - kGvrTabBits);
        b[i] = tab[c];
        e[i] = tab[c + 1];
    }
    for (int step = 0; step < 8; ++step) {
        bool open = false;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (b[i] < e[i]) {
                const uint32_t g = base + ((i >> 2) * kGvrWG + tid) * 4 + (i & 3);
                const uint32_t mid = (b[i] + e[i]) >> 1;
                const uint2 sp = spl[mid];
                if (comp_less(sp.x, sp.y, key[i], g)) b[i] = mid + 1; else e[i] = mid;
                open |= b[i] < e[i];
            }
        }
        if (!__builtin_amdgcn_ballot_w64(open)) break;
    }
    const uint32_t col = tid & 31;
#pragma unroll
    for (int q = 0; q < ITEMS / 4; ++q) {
        const uint32_t u = (q * kGvrWG + tid) * 4;
        const uint32_t packed = b[4 * q] | (b[4 * q + 1] << 8) | (b[4 * q + 2] << 16) | (b[4 * q + 3] << 24);
        if (vec) {
            *(uint32_t*)(bkt + base + u) = packed;
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (u + c < len) bkt[base + u + c] = (uint8_t)b[4 * q + c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (u + c < len) atomicAdd(&h[b[4 * q + c] * 32 + col], 1u);
    }
    __syncthreads();
    if (tid == 0) {
        uint2 m = wmm[0];
#pragma unroll
        for (uint32_t w = 1; w < kGvrWG / 64; ++w) {
            m.x = min(m.x, wmm[w].x);
            m.y = max(m.y, wmm[w].y);
        }
        tmm[t] = m.x;
        tmm[gridDim.x + t] = m.y;
    }
    for (uint32_t v = tid; v < R; v += kGvrWG) {
        const uint4* r4 = (const uint4*)&h[v * 32];
        uint32_t sum = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint4 x = r4[(q + v) & 7];
            sum += x.x + x.y + x.z + x.w;
        }
        counts[(size_t)t * R + v] = sum;
    }
}

// Key offsets of the buckets: bucket j holds keys from lo_j (the key of
// splitter S_j; the smallest key for j = 0) to hi_j (the key of S_{j+1}; the
// largest key for j = p - 1), since its composites lie in (S_j, S_{j+1}].  The
// route stores key - lo_j, so the bucket sort only needs the low digits that
// cover the widest span hi_j - lo_j: rounds = ceil(bits / 8) of the largest
// span (0 when every bucket holds one key value).  When that still takes all
// four rounds the offsets are set to 0 (the route stores the keys as they are
// and nothing is added back).  The smallest and largest keys come from the
// route tiles' minima and maxima tmm.  One workgroup.
constexpr uint32_t kRangeWG = 1024;
__global__ __launch_bounds__(kRangeWG) void k_gvr_range(const uint32_t* Sk, uint32_t p,
                                                        uint32_t s, const uint32_t* tmm,
                                                        uint32_t ntiles, uint32_t* shift,
                                                        uint32_t* rounds)
{
    __shared__ uint2 wred[kRangeWG / 64];
    __shared__ uint32_t red[3];
    const uint32_t tid = threadIdx.x;
    uint32_t a = ~0u, b = 0u;
    for (uint32_t i = tid; i < ntiles; i += 8 * kRangeWG) {
        uint32_t x[8], y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t j = i + u * kRangeWG;
            x[u] = j < ntiles ? tmm[j] : ~0u;
            y[u] = j < ntiles ? tmm[ntiles + j] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a = min(a, x[u]);
            b = max(b, y[u]);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a = min(a, (uint32_t)__shfl_xor((int)a, o, 64));
        b = max(b, (uint32_t)__shfl_xor((int)b, o, 64));
    }
    if ((tid & 63) == 0) wred[tid >> 6] = make_uint2(a, b);
    __syncthreads();
    if (tid == 0) {
        for (uint32_t w = 1; w < kRangeWG / 64; ++w) {
            a = min(a, wred[w].x);
            b = max(b, wred[w].y);
        }
        red[0] = a;
        red[1] = b;
        red[2] = 0;
    }
    __syncthreads();
    uint32_t bits = 0, lo = 0;
    if (tid < p) {
        lo = tid ? Sk[(size_t)tid * s - 1] : red[0];
        const uint32_t hi = tid + 1 < p ? Sk[(size_t)(tid + 1) * s - 1] : red[1];
        const uint32_t span = hi - lo;
        bits = span ? 32u - (uint32_t)__clz(span) : 0u;
    }
    atomicMax(&red[2], bits);
    __syncthreads();
    const uint32_t nr = (red[2] + 7) / 8;
    if (tid < kGvrMaxP) shift[tid] = nr < 4 ? lo : 0u;
    if (tid == 0) *rounds = nr;
}

// Stable scatter of one route tile by bucket: counts[t][v] now holds the keys
// of bucket v in earlier tiles and bases[v] the start of bucket v, so the key
// of bucket v with tile rank q lands at bases[v] + counts[t][v] + q.  The rank
// among the tile's keys of one bucket, in input order, comes from 64-bit slots
// {lanes of the current row, keys of earlier rows} per 32-lane group (rows in
// order); the tile is staged in LDS in bucket order with its bucket bytes and
// written run by run, the payloads in a second staging pass.  A key of bucket
// v is stored as key - shift[v].  When no bucket needs a round (*rounds == 0:
// each bucket holds one key value) and the output is not the input
// (direct_ok), the route is the whole sort: keys and payloads go unchanged
// straight to out / vout instead of Y / YV.
template <bool KV>
__global__ __launch_bounds__(kGvrWG) void k_gvr_scatter(const uint32_t* __restrict__ X,
                                                        const uint32_t* __restrict__ XV,
                                                        const uint32_t* lo, uint32_t tpb,
                                                        const uint8_t* __restrict__ bkt,
                                                        const uint32_t* counts,
                                                        const uint32_t* bases,
                                                        const uint32_t* shift, uint32_t n,
                                                        uint32_t* Y, uint32_t* YV,
                                                        const uint32_t* rounds, uint32_t direct_ok,
                                                        uint32_t* out, uint32_t* vout)
{
    if (direct_ok && *rounds == 0) {
        Y = out;
        YV = vout;
        shift = nullptr;
    }
    constexpr int ITEMS = kGvrItems;
    constexpr uint32_t TILE = kGvrTile;
    struct Smem {
        union {
            uint2 slot[kGvrGroups][R];   // ranking
            struct {
                uint32_t keys[TILE];     // staging in bucket order (payloads second)
                uint8_t dig[TILE];       // bucket of each staged key
            } st;
        } u;
        uint32_t goff[R];
        uint32_t sub[R];
        uint32_t wsum[kGvrWG / 64];
    };
    __shared__ Smem sm;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t grp = tid >> 5, gl = tid & 31;
    const uint32_t hofs = grp * ITEMS * 32 + gl;   // row 0 position of this lane
    // every XCD takes a contiguous range of tiles (grid = tile count): tiles
    // whose bucket runs meet in one cache line write it through one L2
    const uint32_t t = xcd_tile(gridDim.x);
    const uint2 tr = gvr_tile(lo, tpb, t);
    const uint32_t base = tr.x, len = tr.y;
    if (len == 0) return;

    uint32_t k[ITEMS], v[ITEMS], d[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t o = hofs + i * 32;
        const bool ok = o < len;
        k[i] = ok ? X[base + o] : 0u;
        d[i] = ok ? bkt[base + o] : 0u;
        if (KV) v[i] = ok ? XV[base + o] : 0u;
    }
    for (uint32_t i = tid; i < kGvrGroups * R / 2; i += kGvrWG)
        ((uint4*)&sm.u.slot[0][0])[i] = make_uint4(0, 0, 0, 0);
    const uint32_t toff = tid < R ? counts[(size_t)t * R + tid] + bases[tid] : 0u;
    if (tid < R) sm.sub[tid] = shift ? shift[tid] : 0u;
    __syncthreads();

    // rank within the group, rows in order
    uint32_t pos[ITEMS];
    {
        uint2* sl = sm.u.slot[grp];
        const uint32_t bit = 1u << gl;
        const uint32_t lowsel = lane < 32 ? ~0u : 0u;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const bool ok = hofs + i * 32 < len;
            if (ok) __hip_atomic_fetch_or(&sl[d[i]].x, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            wave_lds_order();
            const uint64_t w = ok ? __hip_atomic_load((uint64_t*)&sl[d[i]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 0ull;
            const uint32_t m = (uint32_t)w, c = (uint32_t)(w >> 32);
            pos[i] = __builtin_amdgcn_mbcnt_hi(m, __builtin_amdgcn_mbcnt_lo(m & lowsel, c));
            wave_lds_order();
            if (ok)
                __hip_atomic_store((uint64_t*)&sl[d[i]], (uint64_t)(c + __builtin_popcount(m)) << 32,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            wave_lds_order();
        }
    }
    __syncthreads();
    // slot bases: bucket-major, groups in order within a bucket
    uint32_t run = 0;
    if (tid < R) {
        uint32_t total = 0;
#pragma unroll
        for (uint32_t g = 0; g < kGvrGroups; ++g) total += sm.u.slot[g][tid].y;
        const uint32_t incl = wave_inclusive_sum(total);
        if (lane == 63) sm.wsum[wave] = incl;
        run = incl - total;
    }
    __syncthreads();
    if (tid < R) {
        for (uint32_t w = 0; w < wave; ++w) run += sm.wsum[w];
        sm.goff[tid] = toff - run;
#pragma unroll
        for (uint32_t g = 0; g < kGvrGroups; ++g) {
            const uint32_t c = sm.u.slot[g][tid].y;
            sm.u.slot[g][tid].y = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) pos[i] += sm.u.slot[grp][d[i]].y;
    __syncthreads();
    // stage in bucket order, then write each bucket's run
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if (hofs + i * 32 < len) {
            sm.u.st.keys[pos[i]] = k[i] - sm.sub[d[i]];
            sm.u.st.dig[pos[i]] = (uint8_t)d[i];
        }
    __syncthreads();
    uint32_t outi[KV ? ITEMS : 1];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t q = i * kGvrWG + tid;
        uint32_t o = n;
        if (q < len) {
            o = sm.goff[sm.u.st.dig[q]] + q;
            if (o < n) Y[o] = sm.u.st.keys[q];   // always true unless a tile-scan wait was abandoned
        }
        if (KV) outi[i] = o;
    }
    if (KV) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            if (hofs + i * 32 < len) sm.u.st.keys[pos[i]] = v[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t q = i * kGvrWG + tid;
            if (q < len && outi[i] < n) YV[outi[i]] = sm.u.st.keys[q];
        }
    }
}

// After the route: bucket starts boff[j] (boff[p] = n), and the statistics --
// bnd[k][j] = keys of input block k in buckets below j (from the scanned tile
// counts: the keys of bucket j in block k are the difference of the exclusive
// tile prefixes at the first tiles of blocks k + 1 and k) and the splitters.
__global__ __launch_bounds__(R) void k_gvr_stats(const uint32_t* counts, const uint32_t* bases,
                                                 uint32_t n, uint32_t p, uint32_t s,
                                                 uint32_t tpb, const uint32_t* Sk,
                                                 const uint32_t* Sg, uint32_t* boff,
                                                 uint32_t* bnd, uint32_t* split_key,
                                                 uint32_t* split_g)
{
    __shared__ uint32_t wsum[4];
    const uint32_t k = blockIdx.x, j = threadIdx.x;
    const uint32_t start_j = bases[j];
    const uint32_t total_j = (j + 1 < R ? bases[j + 1] : n) - start_j;
    const uint32_t a = counts[(size_t)k * tpb * R + j];
    const uint32_t b = k + 1 < p ? counts[(size_t)(k + 1) * tpb * R + j] : total_j;
    const uint32_t c = j < p ? b - a : 0u;
    const uint32_t incl = block256_inclusive_sum(c, wsum);
    uint32_t* row = bnd + (size_t)k * (p + 1);
    if (j < p) row[j] = incl - c;
    if (j == p - 1) row[p] = incl;
    if (k == 0) {
        if (j < p) boff[j] = start_j;
        if (j == 0) boff[p] = n;
        if (j + 1 < p) {
            split_key[j] = Sk[(size_t)(j + 1) * s - 1];
            split_g[j] = Sg[(size_t)(j + 1) * s - 1];
        }
    }
}

// The bucket sort leaves key - shift[j] at the positions [boff[j], boff[j+1])
// of bucket j; this adds shift[j] back (nothing to do after all four rounds:
// the offsets were 0).  When it ran no round, the routed keys Y (and
// payloads YV) are already in order and are copied.  Thread
// groups of 4 consecutive keys (one 16-byte access where aligned), 4 groups
// per thread strided by the workgroup; the bucket of a thread's first key is
// found by binary search over the bucket starts, later keys walk forward.
constexpr uint32_t kUnshiftWG = 256;
constexpr uint32_t kUnshiftTile = kUnshiftWG * 16;
template <bool KV>
__global__ __launch_bounds__(kUnshiftWG) void k_gvr_unshift(uint32_t* keys_out, uint32_t* vals_out,
                                                            const uint32_t* Y, const uint32_t* YV,
                                                            const uint32_t* boff,
                                                            const uint32_t* shift,
                                                            const uint32_t* rounds, uint32_t p,
                                                            uint32_t n, uint32_t direct_ok)
{
    __shared__ uint32_t sb[kGvrMaxP + 1];
    __shared__ uint32_t sh[kGvrMaxP];
    const uint32_t nr = *rounds;
    if (nr >= 4 || (nr == 0 && direct_ok)) return;   // keys unchanged, or routed to the output
    const uint32_t tid = threadIdx.x;
    for (uint32_t j = tid; j <= p; j += kUnshiftWG) sb[j] = boff[j];
    if (tid < p) sh[tid] = shift[tid];
    const bool copy = nr == 0;
    const uint32_t* src = copy ? Y : keys_out;
    __syncthreads();
    const uint32_t base = blockIdx.x * kUnshiftTile;
    const uint32_t i0 = base + tid * 4;
    if (i0 >= n) return;
    uint32_t a = 0, b = p - 1;   // largest j < p with sb[j] <= i0 (sb[0] = 0)
    while (a < b) {
        const uint32_t mid = (a + b + 1) >> 1;
        if (sb[mid] <= i0) a = mid; else b = mid - 1;
    }
    uint32_t j = a;
    const bool vec = ((uintptr_t)keys_out & 15) == 0 && ((uintptr_t)src & 15) == 0 &&
                     (!KV || !copy || (((uintptr_t)vals_out & 15) == 0 && ((uintptr_t)YV & 15) == 0));
    typedef uint32_t v4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t i = base + (q * kUnshiftWG + tid) * 4;
        if (i >= n) break;
        uint32_t add[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            while (sb[j + 1] <= i + c && j + 1 < p) ++j;
            add[c] = sh[j];
        }
        if (vec && i + 4 <= n) {
            v4 x = *(const v4*)(src + i);
            x.x += add[0]; x.y += add[1]; x.z += add[2]; x.w += add[3];
            *(v4*)(keys_out + i) = x;
            if (KV && copy) *(v4*)(vals_out + i) = *(const v4*)(YV + i);
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (i + c < n) {
                    keys_out[i + c] = src[i + c] + add[c];
                    if (KV && copy) vals_out[i + c] = YV[i + c];
                }
        }
    }
}


// ---------------------------------------------------------------------------
// GSD step 5 as a merge of the p sorted runs of every bucket (also GER's).
// A sorted sample T of the sorted blocks, p intervals of sT elements, gives
// boundaries B_m = T[c(m) - 1], m = 1..M: each interval is cut into q
// near-equal parts (M = p q, c(m) = (m / q) sT + (m mod q) sT / q), so that
// B_{i q} = T[i sT - 1] ends interval i.  GSD uses its own regular sample
// (sT = s), whose splitters S_i = T[i s - 1] = B_{i q} are thus among the
// boundaries; GER the boundary sample of k_merge_sample (its own random
// sample gives unevenly sized pieces).
// Piece m (m = 0..M)
// holds the elements whose composite lies in (B_m, B_{m+1}] (B_0 = -inf,
// B_{M+1} = +inf): from every sorted block k the positions [F[k][m],
// F[k][m+1]), F[k][m] = #{q in block k : (X_q, index) <= B_m}.  The pieces
// cover the output in order, piece m from sum_k F[k][m] on, and a piece is the
// merge of its p sorted sub-runs; the buckets are unions of consecutive
// pieces' sub-runs, so merging piece by piece merges every bucket.  By Lemma
// 1's argument a piece holds at most (ceil(sT / q) + p - 1) x keys (x = block
// keys per sample); q is chosen so that the average is about 2560.
constexpr uint32_t kMergeWG = 256;
constexpr int kMergeItems = 16;
constexpr uint32_t kMergeCap = kMergeWG * kMergeItems;   // piece merged whole in LDS
constexpr uint32_t kMergeMaxP = 256;                     // one run per thread
constexpr uint32_t kMarkLen = kMergeCap / 16 * 24;       // padded run map (u16 entries)

// F[k][m] for m = 0..M+1, block-major (M + 2 per block).  Chunk c (8192 keys)
// of sorted block k handles the boundaries whose rank in the block falls in
// it: B_m with X[c0 - 1] <= B_m < X[c1 - 1] (first chunk: no lower
// condition; last: no upper one); every block key is read once.
constexpr uint32_t kFineChunk = 8192;

// Sample elements up to and including boundary m (1 <= m <= p q, q <= sT).
__device__ __forceinline__ size_t bound_count(uint32_t m, uint32_t sT, uint32_t q)
{
    return (size_t)(m / q) * sT + (size_t)(m % q) * sT / q;
}

// BK[m - 1] = B_m as one 64-bit composite (key << 32 | index), m = 1..M.
__global__ void k_gsd_bounds(const uint32_t* Sk, const uint32_t* Sg, uint32_t sT, uint32_t q,
                             uint32_t M, uint64_t* BK)
{
    const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (m <= M) {
        const size_t c = bound_count(m, sT, q) - 1;
        BK[m - 1] = ((uint64_t)Sk[c] << 32) | Sg[c];
    }
}

// Index (0..M) of the first boundary not below composite x: BK[i] >= x.
__device__ __forceinline__ uint32_t first_boundary_not_below(const uint64_t* __restrict__ BK,
                                                             uint32_t M, uint64_t x)
{
    uint32_t a = 0, e = M;
    while (a < e) {
        const uint32_t mid = (a + e) >> 1;
        if (BK[mid] < x) a = mid + 1; else e = mid;
    }
    return a;
}

// Boundary ranges of the fine split's chunks, all searched at once: for block
// k, R[k][c] (c = 1 .. nch - 1) = first boundary not below the key before
// chunk c; R[k][nch] / R[k][nch + 1] = first boundary not below the block's
// first / last key (0 and M for an empty block).
__global__ void k_gsd_chunk_ranges(const uint32_t* __restrict__ X, const uint32_t* lo, uint32_t p,
                                   uint32_t M, uint32_t nch, const uint64_t* __restrict__ BK,
                                   uint32_t* R)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t w = nch + 2;
    if (t >= p * w) return;
    const uint32_t k = t / w, c = t - k * w;
    const uint32_t b = lo[k], nk = lo[k + 1] - b;
    uint32_t q;   // block position of the key compared, or none
    uint32_t res;
    if (c == 0) {
        res = 0;
    } else if (c < nch) {
        q = c * kFineChunk - 1;
        res = q < nk ? first_boundary_not_below(BK, M, (uint64_t)X[b + q] << 32 | (b + q)) : M;
    } else if (nk == 0) {
        res = c == nch ? 0u : M;
    } else {
        q = c == nch ? 0u : nk - 1;
        res = first_boundary_not_below(BK, M, (uint64_t)X[b + q] << 32 | (b + q));
    }
    R[t] = res;
}

// Workgroup (c, k): chunk c of sorted block k in LDS; the boundaries whose
// rank in the block falls in the chunk, [R[k][c], R[k][c+1]) (last chunk: up
// to M), are ranked there by binary search in LDS.  Of those, the ones below
// the block's first key rank 0 and the ones at or above its last key rank N_k
// with no search: with presorted input most boundaries are of this kind and
// fall to the two end chunks of every block.
__global__ __launch_bounds__(256) void k_gsd_fine_split(const uint32_t* __restrict__ X,
                                                        const uint32_t* lo, uint32_t p, uint32_t M,
                                                        uint32_t nch, const uint64_t* __restrict__ BK,
                                                        const uint32_t* R, uint32_t* F)
{
    __shared__ uint32_t xs[kFineChunk];
    const uint32_t k = blockIdx.y, tid = threadIdx.x;
    const uint32_t b = lo[k], nk = lo[k + 1] - b;
    const uint32_t c0 = blockIdx.x * kFineChunk;
    if (blockIdx.x == 0) {   // rows 0 and M + 1
        if (tid == 0) F[(size_t)k * (M + 2)] = 0;
        if (tid == 1) F[(size_t)k * (M + 2) + M + 1] = nk;
    }
    if (c0 >= nk && c0 != 0) return;
    const uint32_t c1 = min(nk, c0 + kFineChunk);
    const bool last = c1 == nk;
    const uint32_t* r = R + (size_t)k * (nch + 2);
    const uint32_t r0 = r[blockIdx.x], r1 = last ? M : r[blockIdx.x + 1];
    const uint32_t in0 = blockIdx.x == 0 ? r[nch] : 0u, in1 = last ? r[nch + 1] : M;
    // the chunk into LDS: all of a thread's loads issued before the first
    // store (a loop of load -> store would wait out every load in turn)
    {
        constexpr int PER = kFineChunk / 256;
        const uint32_t len = c1 - c0;
        uint32_t v[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t i = j * 256 + tid;
            v[j] = i < len ? X[b + c0 + i] : 0u;
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t i = j * 256 + tid;
            if (i < len) xs[i] = v[j];
        }
    }
    __syncthreads();
    const uint32_t i0 = max(r0, in0), i1 = max(i0, min(r1, in1));
    for (uint32_t i = r0 + tid; i < i0; i += 256) F[(size_t)k * (M + 2) + i + 1] = 0;
    for (uint32_t i = i1 + tid; i < r1; i += 256) F[(size_t)k * (M + 2) + i + 1] = nk;
    // the next boundary is loaded while this one is searched
    uint64_t next = i0 + tid < i1 ? BK[i0 + tid] : 0ull;
    for (uint32_t i = i0 + tid; i < i1; i += 256) {
        const uint64_t bnd = next;
        if (i + 256 < i1) next = BK[i + 256];
        uint32_t a = 0, e = c1 - c0;   // first q in the chunk with B < (X_q, index)
        while (a < e) {
            const uint32_t mid = (a + e) >> 1;
            if (bnd < ((uint64_t)xs[mid] << 32 | (b + c0 + mid))) e = mid; else a = mid + 1;
        }
        F[(size_t)k * (M + 2) + i + 1] = c0 + a;
    }
}

// GSD: split bounds of the p buckets (bnd[k][i] = F[k][i q]: the splitters
// are boundaries) and the splitters, for the statistics.
__global__ void k_gsd_fine_bnd(const uint32_t* F, uint32_t p, uint32_t s, uint32_t q, uint32_t M,
                               const uint32_t* Sk, const uint32_t* Sg, uint32_t* bnd,
                               uint32_t* split_key, uint32_t* split_g)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p * (p + 1)) return;
    const uint32_t k = t / (p + 1), i = t - k * (p + 1);
    const uint32_t row = i == p ? M + 1 : i * q;
    bnd[t] = F[(size_t)k * (M + 2) + row];
    if (k == 0 && i > 0 && i < p) {
        split_key[i - 1] = Sk[(size_t)i * s - 1];
        split_g[i - 1] = Sg[(size_t)i * s - 1];
    }
}

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

// Run map index of piece position u: blocks of 16 u16 entries (8 dwords)
// padded to 12 dwords, so thread t's block (entries 16 t .. 16 t + 15) is two
// 16-byte vectors at byte 48 t, and the vectors of 16 consecutive threads
// cover the 64 LDS banks once.  The map must be 16-byte aligned.
__device__ __forceinline__ uint32_t mark_idx(uint32_t u) { return u + 8 * (u >> 4); }

// LDS of the piece merge outside the ranking tile.
struct MergeRuns {
    uint32_t src[kMergeMaxP];        // first element of run k in X
    uint32_t off[kMergeMaxP + 1];    // start of run k in the piece
};
struct MergeDigits {
    uint32_t st[R];                  // next output index of each digit
    uint32_t cs[R];                  // digit starts inside the chunk
    uint32_t cc[R];                  // digit counts of the chunk
};
union MergeAux {
    MergeRuns r;
    MergeDigits d;
};

// Registers <- piece positions [c0, c0 + nc) in the ranking layout with ni
// registers per half-wave (position c0 + hofs + 32 i in register i < ni).
// The run of every position is found through a map: run k + 1 is marked at
// its first position in the chunk, and a running maximum fills the positions
// after it.
template <bool KV>
__device__ __forceinline__ void merge_gather(const uint32_t* __restrict__ X,
                                             const uint32_t* __restrict__ XV, uint32_t p,
                                             const MergeRuns& runs, uint16_t* mark, uint32_t* wsc,
                                             uint32_t c0, uint32_t nc,
                                             uint32_t (&k)[kMergeItems], uint32_t (&v)[kMergeItems],
                                             uint32_t ni = kMergeItems)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t hofs = (tid >> 5) * ni * 32 + (tid & 31);
    static_assert(kMergeWG * 16 == kMergeCap && kMarkLen % 8 == 0, "16 map entries a thread");
    for (uint32_t j = tid; j < kMarkLen / 8; j += kMergeWG) ((uint4*)mark)[j] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    if (tid < p) {
        const uint32_t a = runs.off[tid], e = runs.off[tid + 1];
        const uint32_t s0 = max(a, c0), e0 = min(e, c0 + nc);
        if (s0 < e0) mark[mark_idx(s0 - c0)] = (uint16_t)(tid + 1);
    }
    __syncthreads();
    // this thread's 16 entries, two to a dword
    uint4* mb = (uint4*)(mark + mark_idx(16 * tid));
    const uint4 m0 = mb[0], m1 = mb[1];
    uint32_t w[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
    uint32_t run = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) run = max(run, max(w[q] & 0xFFFFu, w[q] >> 16));
    const uint32_t wmax = wave_inclusive_max(run);
    if ((tid & 63) == 63) wsc[tid >> 6] = wmax;
    __syncthreads();
    uint32_t cur = __shfl_up(wmax, 1, 64);
    if ((tid & 63) == 0) cur = 0;
    for (uint32_t w = 0; w < (tid >> 6); ++w) cur = max(cur, wsc[w]);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint32_t lo16 = max(cur, w[q] & 0xFFFFu);
        cur = max(lo16, w[q] >> 16);
        w[q] = lo16 | (cur << 16);
    }
    mb[0] = make_uint4(w[0], w[1], w[2], w[3]);
    mb[1] = make_uint4(w[4], w[5], w[6], w[7]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kMergeItems; ++i) {
        const uint32_t u = hofs + i * 32;
        k[i] = 0;
        v[i] = 0;
        if ((uint32_t)i < ni && u < nc) {
            const uint32_t r = mark[mark_idx(u)] - 1u;
            const uint32_t q = runs.src[r] + (c0 + u - runs.off[r]);
            k[i] = X[q];
            if (KV) v[i] = XV[q];
        }
    }
    __syncthreads();   // the map area is free again
}

// Piece m's runs: aux.r.src / aux.r.off from the bounds F (p <= 256, one run
// per thread); returns {keys in the piece, its output start}.
__device__ __forceinline__ uint2 merge_setup(const uint32_t* lo, uint32_t p, uint32_t M,
                                             const uint32_t* F, uint32_t m, MergeRuns& runs,
                                             uint32_t* wsc, uint32_t* tot)
{
    const uint32_t tid = threadIdx.x;
    uint32_t len = 0, before = 0;
    if (tid < p) {
        const uint32_t* f = F + (size_t)tid * (M + 2) + m;
        before = f[0];
        len = f[1] - before;
    }
    const uint32_t incl = block256_inclusive_sum(len, wsc);
    const uint32_t start = block256_inclusive_sum(before, wsc);
    if (tid < p) {
        runs.src[tid] = lo[tid] + before;
        runs.off[tid] = incl - len;
    }
    if (tid == kMergeWG - 1) {
        tot[0] = incl;    // keys in the piece
        tot[1] = start;   // keys before it: its output start
        runs.off[p] = incl;
    }
    __syncthreads();
    return make_uint2(tot[0], tot[1]);
}

// Key bounds of piece m: its keys lie between the keys of its two boundaries.
__device__ __forceinline__ uint2 merge_key_bounds(const uint32_t* Sk, uint32_t sT, uint32_t q,
                                                  uint32_t M, uint32_t m)
{
    return make_uint2(m == 0 ? 0u : Sk[bound_count(m, sT, q) - 1],
                      m == M ? 0xFFFFFFFFu : Sk[bound_count(m + 1, sT, q) - 1]);
}

// One workgroup per piece: the p sub-runs are read in run order (block order,
// which is input order on equal keys), combined by a stable sort in LDS --
// one tile_round per byte, rounds whose byte is the same for the whole piece
// skipped -- which is their merge, and written once at the piece's start.
// The piece is sorted as words key - lower bound (with payloads (key - lower
// bound) << 12 | position, the payloads following by position; that needs
// keys within 2^20 of the lower bound), keys only, on the bits the piece's
// key range spans.  Pieces beyond one LDS tile, and with
// payloads pieces of a wider key range, are only listed here (large[0] =
// count, large[1..] = pieces) for k_gsd_merge_large.
// The ranking slots share LDS with the key staging: with payloads about
// 35 KiB per workgroup, four 4-wave workgroups per CU.
template <bool KV>
__global__ __launch_bounds__(kMergeWG, 4) void k_gsd_merge(const uint32_t* __restrict__ X,
                                                           const uint32_t* __restrict__ XV,
                                                           const uint32_t* lo, uint32_t p,
                                                           uint32_t M, uint32_t sT, uint32_t q,
                                                           const uint32_t* Sk, const uint32_t* F,
                                                           uint32_t* out, uint32_t* vout,
                                                           uint32_t* large)
{
    constexpr int ITEMS = kMergeItems;
    constexpr uint32_t C = kMergeCap;
    static_assert(kMarkLen * 2 <= sizeof(uint2) * (kMergeWG / 32) * kTileRadix,
                  "the run map lives in the ranking slots");
    // LDS: the keys-only ranking tile, with payloads followed by the payloads
    // staged by piece position
    using SmK = TileSmem<uint32_t, false, kMergeWG, ITEMS, true>;
    struct Packed {
        SmK t;
        uint32_t vst[KV ? C : 1];
    };
    __shared__ alignas(16) Packed smu;
    __shared__ MergeRuns runs;
    __shared__ uint32_t wsc[4];
    __shared__ uint32_t tot[2];
    const uint32_t tid = threadIdx.x;
    // Piece of this workgroup.  The grid (a multiple of 8) is dealt to the 8
    // XCDs in turn; XCD x takes the x-th eighth of the pieces, so neighbouring
    // pieces, whose runs and outputs share cache lines, meet in one L2.
    const uint32_t per = gridDim.x >> 3, x = blockIdx.x & 7, j = blockIdx.x >> 3;
    const uint32_t m = x * per + j;
    if (m > M) return;
    const uint2 kb = merge_key_bounds(Sk, sT, q, M, m);
    const uint32_t klo = kb.x, khi = kb.y;
    const uint2 lb = merge_setup(lo, p, M, F, m, runs, wsc, tot);
    const uint32_t L = lb.x, base = lb.y;
    if (L == 0) return;
    if (L > C || (KV && khi - klo >= (1u << 20))) {
        if (tid == 0) large[1 + atomicAdd(&large[0], 1u)] = m;
        return;
    }
    // the piece spread over all half-waves: ni registers each
    constexpr uint32_t HW = kMergeWG / 32;
    const uint32_t ni = (L + 32 * HW - 1) / (32 * HW);
    const uint32_t hofs = (tid >> 5) * ni * 32 + (tid & 31);
    uint16_t* mark = (uint16_t*)&smu.t.slot[0][0];   // run map in the ranking slots
    uint32_t k[ITEMS], v[ITEMS];
    merge_gather<KV>(X, XV, p, runs, mark, wsc, 0, L, k, v, ni);
    // word = (key - klo) << 12 | position with payloads (range < 2^20), or
    // key - klo without; a keys-only stable sort on the range bits
    constexpr uint32_t low = KV ? 12u : 0u;
    const uint32_t range = khi - klo;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t u = hofs + i * 32;
        if (KV && (uint32_t)i < ni && u < L) smu.vst[u] = v[i];
        k[i] = ((k[i] - klo) << low) | (KV ? u : 0u);
    }
    const uint32_t nb = range ? 32u - __builtin_clz(range) : 0u;
#pragma unroll 1
    for (uint32_t sh = 0; sh < nb; sh += 8) {
        const uint32_t w = min(8u, nb - sh);
        tile_round<uint32_t, false, kMergeWG, ITEMS>(smu.t, k, v, L, low + sh, (1u << w) - 1u, ni);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t u = hofs + i * 32;
        if ((uint32_t)i < ni && u < L) {
            out[base + u] = klo + (k[i] >> low);
            if (KV) vout[base + u] = smu.vst[k[i] & 0xFFFu];
        }
    }
}

// The pieces k_gsd_merge listed (beyond one LDS tile, or with payloads a
// key range of 2^20 or more: mostly the two edge pieces), one workgroup each;
// the grid is an upper bound (every piece) and surplus workgroups exit.  The piece is gathered
// into tmp[base, base + L), then per byte stably count-sorted, chunk by
// chunk, between tmp and out[base, base + L) (both owned by this piece).
template <bool KV>
__global__ __launch_bounds__(kMergeWG) void k_gsd_merge_large(
    const uint32_t* __restrict__ X, const uint32_t* __restrict__ XV, const uint32_t* lo,
    uint32_t p, uint32_t M, uint32_t sT, uint32_t q, const uint32_t* Sk, const uint32_t* F, uint32_t* out,
    uint32_t* vout, uint32_t* tmp, uint32_t* vtmp, const uint32_t* large)
{
    constexpr int ITEMS = kMergeItems;
    constexpr uint32_t C = kMergeCap;
    __shared__ TileSmem<uint32_t, KV, kMergeWG, ITEMS> sm;
    __shared__ MergeAux aux;
    __shared__ uint32_t wsc[4];
    __shared__ uint32_t tot[2];
    if (blockIdx.x >= large[0]) return;
    const uint32_t m = large[1 + blockIdx.x];
    const uint32_t tid = threadIdx.x;
    const uint32_t hofs = (tid >> 5) * ITEMS * 32 + (tid & 31);
    const uint2 kb = merge_key_bounds(Sk, sT, q, M, m);
    const uint32_t varying = kb.x ^ kb.y;
    const uint2 lb = merge_setup(lo, p, M, F, m, aux.r, wsc, tot);
    const uint32_t L = lb.x, base = lb.y;
    // run map in the ranking slots, from their first 16-byte boundary
    static_assert(kMarkLen * 2 + 16 <= sizeof(sm.slot), "the run map fits the ranking slots");
    uint16_t* mark = (uint16_t*)(((uintptr_t)&sm.slot[0][0] + 15) & ~(uintptr_t)15);
    uint32_t k[ITEMS], v[ITEMS];
    for (uint32_t c0 = 0; c0 < L; c0 += C) {
        const uint32_t nc = min(C, L - c0);
        merge_gather<KV>(X, XV, p, aux.r, mark, wsc, c0, nc, k, v);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t u = hofs + i * 32;
            if (u < nc) {
                tmp[base + c0 + u] = k[i];
                if (KV) vtmp[base + c0 + u] = v[i];
            }
        }
    }
    __syncthreads();
    uint32_t* ck = tmp + base;      // current keys
    uint32_t* cv = KV ? vtmp + base : nullptr;
    uint32_t* ok = out + base;      // the other buffer
    uint32_t* ov = KV ? vout + base : nullptr;
    MergeDigits& dg = aux.d;
#pragma unroll 1
    for (uint32_t d = 0; d < 4 && (varying >> (8 * d)); ++d) {
        const uint32_t shift = 8u * d;
        dg.st[tid] = 0;
        __syncthreads();
        for (uint32_t j0 = 0; j0 < L; j0 += kMergeWG * 16) {   // 16 loads in flight per thread
            uint32_t x[16];
#pragma unroll
            for (uint32_t q = 0; q < 16; ++q) {
                const uint32_t j = j0 + q * kMergeWG + tid;
                x[q] = j < L ? ck[j] : 0u;
            }
#pragma unroll
            for (uint32_t q = 0; q < 16; ++q)
                if (j0 + q * kMergeWG + tid < L) atomicAdd(&dg.st[digit_of(x[q], shift, 0xFFu)], 1u);
        }
        __syncthreads();
        const uint32_t cnt = dg.st[tid];
        if (__syncthreads_or(cnt == L)) continue;   // one byte value everywhere: nothing moves
        const uint32_t ex = block256_inclusive_sum(cnt, wsc) - cnt;
        dg.st[tid] = ex;
        __syncthreads();
#pragma unroll 1
        for (uint32_t c0 = 0; c0 < L; c0 += C) {
            const uint32_t nc = min(C, L - c0);
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t u = hofs + i * 32;
                k[i] = u < nc ? ck[c0 + u] : 0u;
                v[i] = KV && u < nc ? cv[c0 + u] : 0u;
            }
            dg.cc[tid] = 0;
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; ++i)
                if (hofs + i * 32 < nc) atomicAdd(&dg.cc[digit_of(k[i], shift, 0xFFu)], 1u);
            __syncthreads();
            const uint32_t c = dg.cc[tid];
            dg.cs[tid] = block256_inclusive_sum(c, wsc) - c;
            __syncthreads();
            tile_round<uint32_t, KV, kMergeWG, ITEMS>(sm, k, v, nc, shift, 0xFFu);
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t u = hofs + i * 32;
                if (u < nc) {
                    const uint32_t dv = digit_of(k[i], shift, 0xFFu);
                    const uint32_t o = dg.st[dv] + u - dg.cs[dv];
                    ok[o] = k[i];
                    if (KV) ov[o] = v[i];
                }
            }
            __syncthreads();
            dg.st[tid] += c;
            __syncthreads();
        }
        uint32_t* t = ck; ck = ok; ok = t;
        if (KV) { t = cv; cv = ov; ov = t; }
    }
    if (ck != out + base) {
        for (uint32_t j0 = 0; j0 < L; j0 += kMergeWG * 8) {
            uint32_t x[8], y[8];
#pragma unroll
            for (uint32_t q = 0; q < 8; ++q) {
                const uint32_t j = j0 + q * kMergeWG + tid;
                x[q] = j < L ? ck[j] : 0u;
                y[q] = KV && j < L ? cv[j] : 0u;
            }
#pragma unroll
            for (uint32_t q = 0; q < 8; ++q) {
                const uint32_t j = j0 + q * kMergeWG + tid;
                if (j < L) {
                    out[base + j] = x[q];
                    if (KV) vout[base + j] = y[q];
                }
            }
        }
    }
}

}  // namespace

namespace {

GsdLayout skeleton_layout(bool has_vals, size_t n, uint32_t p, uint32_t s, size_t nT, int kind)
{
    GsdLayout L{};
    L.p = p;
    L.s = s;
    L.nT = nT;
    L.kind = kind;
    L.tiles_per_block = (uint32_t)((n / p + 1 + kRouteTile - 1) / kRouteTile);
    L.LT = lsd_r8_layout(4, true, L.nT, 0, 32);
    L.LTk = lsd_r8_layout(4, false, L.nT, 0, 32);
    L.LS = devseg_layout(4, has_vals, n, p);
    // the merge finish (GSD, GER with p <= 256) cuts its pieces at a sorted
    // sample of the sorted blocks: GSD's own; for GER a boundary sample
    // (k_merge_sample) of about one element per 128 block keys, its
    // splitters and statistics staying those of its random sample
    L.s2 = s;
    L.nT2 = L.nT;
    if (kind == kGER && n) {
        L.s2 = (uint32_t)std::min<size_t>(8192, std::max<size_t>(1, (n / p + 127) / 128));
        L.nT2 = (size_t)p * L.s2;
    }
    L.LT2 = lsd_r8_layout(4, true, L.nT2, 0, 32);
    const size_t nTmax = std::max(L.nT, L.nT2);
    size_t o = 0;
    L.off_lo = o;    o = align_up(o + (size_t)(p + 1) * 4);
    L.off_boff = o;  o = align_up(o + (size_t)(p + 1) * 4);
    L.off_bsize = o; o = align_up(o + (size_t)p * 4);
    L.off_coloff = o; o = align_up(o + (size_t)p * p * 4);
    L.off_Tk = o;    o = align_up(o + nTmax * 4);
    L.off_Tg = o;    o = align_up(o + nTmax * 4);
    L.off_Sk = o;    o = align_up(o + nTmax * 4);
    L.off_Sg = o;    o = align_up(o + nTmax * 4);
    L.off_lsd = o;   o = align_up(o + std::max(std::max(L.LT.bytes, L.LTk.bytes), L.LT2.bytes));
    L.off_Y = o;     o = align_up(o + n * 4);
    L.off_YV = o;    o = align_up(o + (has_vals ? n * 4 : 0));
    L.off_seg = o;   o = align_up(o + L.LS.bytes);
    if ((kind == kGSD || kind == kGER) && p <= kMergeMaxP && L.nT2 && n <= L.nT2 * 4096) {
        // the merge finish: each interval of s2 sample elements cut into q
        // parts (1 <= q <= s2) of about 2560 keys; at 2^28 pairs GER's merge
        // measured fastest with pieces of 2304 to 2816 keys (4 % below 2048;
        // 3072 slower again, more pieces above one tile)
        L.merge = true;
        // sample elements per piece for about 2560 keys, then parts per interval
        const double per_piece = std::max(1.0, 2560.0 * (double)L.nT2 / (double)n);
        const double parts = std::floor((double)L.s2 / per_piece + 0.5);
        L.q = (uint32_t)std::min<double>(L.s2, std::max(1.0, parts));
        L.M = p * L.q;
        L.off_F = o;       o = align_up(o + ((size_t)L.M + 2) * p * 4);
        L.off_BK = o;      o = align_up(o + (size_t)L.M * 8);
        L.off_large = o;   o = align_up(o + ((size_t)L.M + 2) * 4);
        const size_t nch = std::max<size_t>(1, ((n + p - 1) / p + kFineChunk - 1) / kFineChunk);
        L.off_R = o;       o = align_up(o + (size_t)p * (nch + 2) * 4);
    }
    if (kind == kGVR) {
        L.route_tpb = (uint32_t)(((n + p - 1) / p + kGvrTile - 1) / kGvrTile);
        L.route_ntiles = p * L.route_tpb;
        const size_t nblocks = (L.route_ntiles + kScanBlock - 1) / kScanBlock;
        L.off_rcounts = o; o = align_up(o + (size_t)L.route_ntiles * R * 4);
        L.off_rstate = o;  o = align_up(o + nblocks * R * 4);
        L.off_rplan = o;   o = align_up(o + sizeof(RoundPlan) + 4);
        L.off_rbases = o;  o = align_up(o + R * 4);
        L.off_bkt = o;     o = align_up(o + n);
        L.off_rtab = o;    o = align_up(o + kGvrTab + 4);
        L.off_rshift = o;  o = align_up(o + (kGvrMaxP + 1) * 4);
        L.off_rmm = o;     o = align_up(o + (size_t)L.route_ntiles * 8);
    }
    L.bytes = o;
    return L;
}

}  // namespace

GsdLayout gsd_layout(bool has_vals, size_t n, uint32_t p_req, uint32_t r)
{
    const uint32_t p = (uint32_t)std::min<size_t>(p_req, n ? n : 1);
    return skeleton_layout(has_vals, n, p, r * p, (size_t)p * r * p, kGSD);
}

GsdLayout ger_layout(bool has_vals, size_t n, uint32_t p_req, uint32_t s)
{
    const uint32_t p = (uint32_t)std::min<size_t>(p_req, n ? n : 1);
    return skeleton_layout(has_vals, n, p, s, (size_t)s * p - 1, kGER);
}

GsdLayout gvr_layout(bool has_vals, size_t n, uint32_t p_req, uint32_t s)
{
    const uint32_t p = (uint32_t)std::min<size_t>(p_req, n ? n : 1);
    return skeleton_layout(has_vals, n, p, s, (size_t)s * p - 1, kGVR);
}

size_t gsd_stats_words(uint32_t p) { return (size_t)p * (p + 1) + 2 * (size_t)p; }

namespace {

// The sample of GER and GVR: s p - 1 drawn positions, put in position order,
// their keys gathered from src, then ordered by key (ties stay in position
// order) into Sk / Sg.
hipError_t random_sample(const uint32_t* src, size_t n, const GsdLayout& L, uint64_t seed,
                         uint8_t* w, uint32_t* Tk, uint32_t* Tg, uint32_t* Sk, uint32_t* Sg,
                         uint32_t* dev_err, hipStream_t stream)
{
    if (!L.nT) return hipSuccess;
    const dim3 sg((uint32_t)((L.nT + 255) / 256));
    hipLaunchKernelGGL(k_ger_draw, sg, dim3(256), 0, stream, seed, (uint32_t)n, L.nT, Tg);
    hipError_t e = lsd_r8_sort(4, Tg, Sg, nullptr, nullptr, L.nT, 0, 32, w + L.off_lsd, L.LTk,
                               dev_err, stream, nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ger_gather, sg, dim3(256), 0, stream, src, Sg, L.nT, Tk, Tg);
    return lsd_r8_sort(4, Tk, Sk, Tg, Sg, L.nT, 0, 32, w + L.off_lsd, L.LT, dev_err, stream,
                       nullptr);
}

// GVR (Algorithm 3): sample the input, route it by bucket, sort the buckets.
hipError_t gvr_sort(const uint32_t* keys_in, uint32_t* keys_out, const uint32_t* vals_in,
                    uint32_t* vals_out, size_t n, const GsdLayout& L, uint64_t seed, uint8_t* w,
                    const uint32_t* lo, uint32_t* Tk, uint32_t* Tg, uint32_t* Sk, uint32_t* Sg,
                    uint32_t* Y, uint32_t* YV, uint32_t* bnd, uint32_t* split_key,
                    uint32_t* split_g, uint32_t* boff, uint32_t* dev_err, hipStream_t stream,
                    Profiler* prof)
{
    const uint32_t p = L.p, s = L.s, tpb = L.route_tpb, nt = L.route_ntiles;
    uint32_t* counts = (uint32_t*)(w + L.off_rcounts);
    uint32_t* state = (uint32_t*)(w + L.off_rstate);
    RoundPlan* plan = (RoundPlan*)(w + L.off_rplan);
    uint32_t* ticket = (uint32_t*)(w + L.off_rplan + sizeof(RoundPlan));
    uint32_t* bases = (uint32_t*)(w + L.off_rbases);
    uint8_t* bkt = w + L.off_bkt;
    uint32_t* shift = (uint32_t*)(w + L.off_rshift);
    uint32_t* rounds = shift + kGvrMaxP;
    uint32_t* tmm = (uint32_t*)(w + L.off_rmm);
    const size_t nblocks = (nt + kScanBlock - 1) / kScanBlock;
    // 1-2. sample of the input and splitters
    hipError_t e = random_sample(keys_in, n, L, seed, w, Tk, Tg, Sk, Sg, dev_err, stream);
    if (e != hipSuccess) return e;
    // 3. bucket of every key, the tile counts, their scan, the stable route
    hipLaunchKernelGGL(k_gvr_init, dim3((uint32_t)std::min<size_t>(1024, (nblocks * R + 255) / 256)),
                       dim3(256), 0, stream, plan, ticket, state, nblocks * R);
    uint8_t* tab = w + L.off_rtab;
    hipLaunchKernelGGL(k_gvr_table, dim3(1), dim3(1024), 0, stream, Sk, p, s, tab);
    hipLaunchKernelGGL(k_gvr_count, dim3(nt), dim3(kGvrWG), 0, stream, keys_in, lo, p, s, tpb, Sk,
                       Sg, tab, bkt, counts, tmm);
    hipLaunchKernelGGL(k_gvr_range, dim3(1), dim3(kRangeWG), 0, stream, Sk, p, s, tmm, nt, shift,
                       rounds);
    RoundArgs a{};
    a.n = (uint32_t)n;
    a.ntiles = nt;
    a.bases = bases;
    a.plan = plan;
    a.counts = counts;
    a.blk_state = state;
    a.tickets = ticket;
    a.err = dev_err;
    hipLaunchKernelGGL(k_tilescan, dim3((uint32_t)nblocks), dim3(R), 0, stream, a);
    // with no round to run the route may write the output itself, unless it
    // would overwrite keys or payloads other workgroups have yet to read
    const uint32_t direct_ok = (const void*)keys_out != (const void*)keys_in &&
                               (!vals_in || (const void*)vals_out != (const void*)vals_in);
    if (vals_in)
        hipLaunchKernelGGL(k_gvr_scatter<true>, dim3(nt), dim3(kGvrWG), 0, stream, keys_in,
                           vals_in, lo, tpb, bkt, counts, bases, shift, (uint32_t)n, Y, YV,
                           (const uint32_t*)rounds, direct_ok, keys_out, vals_out);
    else
        hipLaunchKernelGGL(k_gvr_scatter<false>, dim3(nt), dim3(kGvrWG), 0, stream, keys_in,
                           nullptr, lo, tpb, bkt, counts, bases, shift, (uint32_t)n, Y, nullptr,
                           (const uint32_t*)rounds, direct_ok, keys_out, nullptr);
    hipLaunchKernelGGL(k_gvr_stats, dim3(p), dim3(R), 0, stream, counts, bases, (uint32_t)n, p, s,
                       tpb, Sk, Sg, boff, bnd, split_key, split_g);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // 4. every bucket stable-sorted into the output by the digits its keys
    // span, then the bucket offsets added back
    e = devseg_sort(4, Y, keys_out, YV, vals_out, n, boff, p, kSmallMaxDefault, w + L.off_seg,
                    L.LS, dev_err, stream, prof, 0, rounds);
    if (e != hipSuccess) return e;
    const dim3 ug((uint32_t)((n + kUnshiftTile - 1) / kUnshiftTile));
    if (vals_in)
        hipLaunchKernelGGL(k_gvr_unshift<true>, ug, dim3(kUnshiftWG), 0, stream, keys_out,
                           vals_out, Y, YV, boff, shift, rounds, p, (uint32_t)n, direct_ok);
    else
        hipLaunchKernelGGL(k_gvr_unshift<false>, ug, dim3(kUnshiftWG), 0, stream, keys_out,
                           nullptr, Y, nullptr, boff, shift, rounds, p, (uint32_t)n, direct_ok);
    return hipGetLastError();
}

// GSD / GER with the merge finish: local sort into Y, the sample (regular or
// random) and splitters, fine split, and the piece merge from Y into the output.
hipError_t gsd_merge_sort(const uint32_t* keys_in, uint32_t* keys_out, const uint32_t* vals_in,
                          uint32_t* vals_out, size_t n, const GsdLayout& L, uint64_t seed,
                          uint8_t* w,
                          const uint32_t* lo, uint32_t* Tk, uint32_t* Tg, uint32_t* Sk,
                          uint32_t* Sg, uint32_t* Y, uint32_t* YV, uint32_t* bnd,
                          uint32_t* split_key, uint32_t* split_g, uint32_t* dev_err,
                          hipStream_t stream, Profiler* prof)
{
    const uint32_t p = L.p, s = L.s, sT = L.s2, q = L.q, M = L.M;
    uint32_t* F = (uint32_t*)(w + L.off_F);
    uint8_t* seg_ws = w + L.off_seg;
    uint32_t* tmp = (uint32_t*)(seg_ws + L.LS.off_tmp_keys);
    uint32_t* vtmp = vals_in ? (uint32_t*)(seg_ws + L.LS.off_tmp_vals) : nullptr;
    // 1. local sort of the blocks into Y
    hipError_t e = devseg_sort(4, keys_in, Y, vals_in, YV, n, lo, p, kSmallMaxDefault, seg_ws,
                               L.LS, dev_err, stream, prof);
    if (e != hipSuccess) return e;
    // 2-3. the sample of the sorted blocks, sorted by composite
    const uint32_t nb = p * (p + 1);
    if (L.kind == kGSD) {
        hipLaunchKernelGGL(k_gsd_sample, dim3((uint32_t)((L.nT + 255) / 256)), dim3(256), 0, stream,
                           Y, lo, p, s, Tk, Tg);
        e = lsd_r8_sort(4, Tk, Sk, Tg, Sg, L.nT, 0, 32, w + L.off_lsd, L.LT, dev_err, stream,
                        nullptr);
    } else {
        // GER: the random sample's splitters and the split bounds of the
        // statistics (binary search of each splitter in each sorted block),
        // then the boundary sample for the merge in the same buffers
        e = random_sample(Y, n, L, seed, w, Tk, Tg, Sk, Sg, dev_err, stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_gsd_split, dim3((nb + 255) / 256), dim3(256), 0, stream, Y, lo, p, s,
                           Sk, Sg, bnd, split_key, split_g);
        hipLaunchKernelGGL(k_merge_sample, dim3((uint32_t)((L.nT2 + 255) / 256)), dim3(256), 0,
                           stream, Y, lo, p, L.s2, Tk, Tg);
        e = lsd_r8_sort(4, Tk, Sk, Tg, Sg, L.nT2, 0, 32, w + L.off_lsd, L.LT2, dev_err, stream,
                        nullptr);
    }
    if (e != hipSuccess) return e;
    // 4. splitters, the fine split, the buckets' split bounds
    uint64_t* BK = (uint64_t*)(w + L.off_BK);
    hipLaunchKernelGGL(k_gsd_bounds, dim3((M + 255) / 256), dim3(256), 0, stream, Sk, Sg, sT, q, M, BK);
    const uint32_t chunks = (uint32_t)std::max<size_t>(1, ((n + p - 1) / p + kFineChunk - 1) / kFineChunk);
    uint32_t* R = (uint32_t*)(w + L.off_R);
    const uint32_t nr = p * (chunks + 2);
    hipLaunchKernelGGL(k_gsd_chunk_ranges, dim3((nr + 255) / 256), dim3(256), 0, stream, Y, lo, p, M,
                       chunks, BK, R);
    hipLaunchKernelGGL(k_gsd_fine_split, dim3(chunks, p), dim3(256), 0, stream, Y, lo, p, M, chunks,
                       BK, R, F);
    if (L.kind == kGSD)
        hipLaunchKernelGGL(k_gsd_fine_bnd, dim3((nb + 255) / 256), dim3(256), 0, stream, F, p, s, q,
                           M, Sk, Sg, bnd, split_key, split_g);
    // 5. merge every piece into the output
    uint32_t* large = (uint32_t*)(w + L.off_large);
    const uint32_t max_large = M + 1;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, stream, large, 1u, 0u);
    const dim3 mg((M + 1 + 7) & ~7u);
    if (vals_in) {
        hipLaunchKernelGGL(k_gsd_merge<true>, mg, dim3(kMergeWG), 0, stream, Y, YV, lo, p, M, sT, q, Sk,
                           F, keys_out, vals_out, large);
        hipLaunchKernelGGL(k_gsd_merge_large<true>, dim3(max_large), dim3(kMergeWG), 0, stream, Y,
                           YV, lo, p, M, sT, q, Sk, F, keys_out, vals_out, tmp, vtmp, large);
    } else {
        hipLaunchKernelGGL(k_gsd_merge<false>, mg, dim3(kMergeWG), 0, stream, Y, nullptr, lo, p, M,
                           sT, q, Sk, F, keys_out, nullptr, large);
        hipLaunchKernelGGL(k_gsd_merge_large<false>, dim3(max_large), dim3(kMergeWG), 0, stream, Y,
                           nullptr, lo, p, M, sT, q, Sk, F, keys_out, nullptr, tmp, nullptr, large);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t gsd_sort(const uint32_t* keys_in, uint32_t* keys_out, const uint32_t* vals_in,
                    uint32_t* vals_out, size_t n, const GsdLayout& L, uint64_t seed, void* ws,
                    uint32_t* stats, uint32_t* dev_err, hipStream_t stream, Profiler* prof)
{
    if (!n) return hipSuccess;
    const uint32_t p = L.p, s = L.s;
    uint8_t* w = (uint8_t*)ws;
    uint32_t* lo = (uint32_t*)(w + L.off_lo);
    uint32_t* boff = (uint32_t*)(w + L.off_boff);
    uint32_t* bsize = (uint32_t*)(w + L.off_bsize);
    uint32_t* coloff = (uint32_t*)(w + L.off_coloff);
    uint32_t* Tk = (uint32_t*)(w + L.off_Tk);
    uint32_t* Tg = (uint32_t*)(w + L.off_Tg);
    uint32_t* Sk = (uint32_t*)(w + L.off_Sk);
    uint32_t* Sg = (uint32_t*)(w + L.off_Sg);
    uint32_t* Y = (uint32_t*)(w + L.off_Y);
    uint32_t* YV = vals_in ? (uint32_t*)(w + L.off_YV) : nullptr;
    void* seg_ws = w + L.off_seg;
    uint32_t* bnd = stats;                                   // p x (p+1)
    uint32_t* split_key = stats + (size_t)p * (p + 1);       // p - 1
    uint32_t* split_g = split_key + p;                       // p - 1
    const uint32_t small_max = kSmallMaxDefault;

    hipLaunchKernelGGL(k_gsd_blocks, dim3((p + 256) / 256), dim3(256), 0, stream, lo, (uint32_t)n, p);
    if (L.kind == kGVR)
        return gvr_sort(keys_in, keys_out, vals_in, vals_out, n, L, seed, w, lo, Tk, Tg, Sk, Sg, Y,
                        YV, bnd, split_key, split_g, boff, dev_err, stream, prof);
    if (L.merge) return gsd_merge_sort(keys_in, keys_out, vals_in, vals_out, n, L, seed, w, lo, Tk,
                                       Tg, Sk, Sg, Y, YV, bnd, split_key, split_g, dev_err, stream,
                                       prof);
    // 1. local sort of the blocks into the output arrays
    hipError_t e = devseg_sort(4, keys_in, keys_out, vals_in, vals_out, n, lo, p, small_max,
                               seg_ws, L.LS, dev_err, stream, prof);
    if (e != hipSuccess) return e;
    // 2-3. the sample, sorted by composite (key, position)
    if (L.kind == kGSD) {
        // GSD: regular sample, built in position order; stable by key, so
        // ties stay in position order
        const dim3 sg((uint32_t)((L.nT + 255) / 256));
        hipLaunchKernelGGL(k_gsd_sample, sg, dim3(256), 0, stream, keys_out, lo, p, s, Tk, Tg);
        e = lsd_r8_sort(4, Tk, Sk, Tg, Sg, L.nT, 0, 32, w + L.off_lsd, L.LT, dev_err, stream,
                        nullptr);
    } else {
        // GER: random positions into the sorted blocks
        e = random_sample(keys_out, n, L, seed, w, Tk, Tg, Sk, Sg, dev_err, stream);
    }
    if (e != hipSuccess) return e;
    // 4-5. splitters and split
    const uint32_t nb = p * (p + 1);
    hipLaunchKernelGGL(k_gsd_split, dim3((nb + 255) / 256), dim3(256), 0, stream, keys_out, lo, p,
                       s, Sk, Sg, bnd, split_key, split_g);
    // 6. route
    hipLaunchKernelGGL(k_gsd_colscan, dim3((p + kScanCols - 1) / kScanCols),
                       dim3(kScanCols * kScanGroups), 0, stream, bnd, p, coloff, bsize);
    hipLaunchKernelGGL(k_gsd_bucket_starts, dim3(1), dim3(1024), 0, stream, bsize, p, boff);
    const dim3 rg(p * L.tiles_per_block);
    if (vals_in)
        hipLaunchKernelGGL(k_gsd_route<true>, rg, dim3(kRouteWG), 0, stream, keys_out, vals_out,
                           lo, (uint32_t)n, p, L.tiles_per_block, bnd, coloff, boff, Y, YV);
    else
        hipLaunchKernelGGL(k_gsd_route<false>, rg, dim3(kRouteWG), 0, stream, keys_out, nullptr,
                           lo, (uint32_t)n, p, L.tiles_per_block, bnd, coloff, boff, Y, nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // 7. finish: every bucket stable-sorted into the output
    return devseg_sort(4, Y, keys_out, YV, vals_out, n, boff, p, small_max, seg_ws, L.LS, dev_err,
                       stream, prof);
}

}  // namespace rsort
