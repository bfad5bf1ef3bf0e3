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

#include "lsd_kernels.h"

namespace rsort {
namespace {

constexpr uint32_t kRouteWG = 256;
constexpr uint32_t kRouteItems = 16;
constexpr uint32_t kRouteTile = kRouteWG * kRouteItems;   // keys per route workgroup
constexpr uint32_t kScanCols = 64;                        // bucket columns per scan workgroup
constexpr uint32_t kScanGroups = 16;                      // block groups per column

// lo[k] = floor(k n / p), k = 0..p.
__global__ void k_gsd_blocks(uint32_t* lo, uint32_t n, uint32_t p)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k <= p) lo[k] = (uint32_t)(((uint64_t)k * n) / p);
}

// Regular sample of the sorted blocks: element t = k s + j - 1.
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
#pragma unroll 4
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
            Y[d] = X[b + u];
            if (KV) YV[d] = XV[b + u];
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
__global__ __launch_bounds__(kGvrWG) void k_gvr_count(const uint32_t* __restrict__ X,
                                                      const uint32_t* lo, uint32_t p, uint32_t s,
                                                      uint32_t tpb, const uint32_t* Sk,
                                                      const uint32_t* Sg, const uint8_t* gtab,
                                                      uint8_t* bkt, uint32_t* counts)
{
    constexpr int ITEMS = kGvrItems;
    __shared__ uint2 spl[kGvrMaxP];
    __shared__ uint32_t h[R * 32];
    __shared__ uint8_t tab[kGvrTab + 4];
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < R * 32 / 4; i += kGvrWG) ((uint4*)h)[i] = make_uint4(0, 0, 0, 0);
    if (tid + 1 < p) spl[tid] = make_uint2(Sk[(size_t)(tid + 1) * s - 1], Sg[(size_t)(tid + 1) * s - 1]);
    for (uint32_t c = tid; c <= kGvrTab; c += kGvrWG) tab[c] = gtab[c];
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

// Stable scatter of one route tile by bucket: counts[t][v] now holds the keys
// of bucket v in earlier tiles and bases[v] the start of bucket v, so the key
// of bucket v with tile rank q lands at bases[v] + counts[t][v] + q.  The rank
// among the tile's keys of one bucket, in input order, comes from 64-bit slots
// {lanes of the current row, keys of earlier rows} per 32-lane group (rows in
// order); the tile is staged in LDS in bucket order with its bucket bytes and
// written run by run, the payloads in a second staging pass.
template <bool KV>
__global__ __launch_bounds__(kGvrWG) void k_gvr_scatter(const uint32_t* __restrict__ X,
                                                        const uint32_t* __restrict__ XV,
                                                        const uint32_t* lo, uint32_t tpb,
                                                        const uint8_t* __restrict__ bkt,
                                                        const uint32_t* counts,
                                                        const uint32_t* bases, uint32_t n,
                                                        uint32_t* Y, uint32_t* YV)
{
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
            sm.u.st.keys[pos[i]] = k[i];
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
    size_t o = 0;
    L.off_lo = o;    o = align_up(o + (size_t)(p + 1) * 4);
    L.off_boff = o;  o = align_up(o + (size_t)(p + 1) * 4);
    L.off_bsize = o; o = align_up(o + (size_t)p * 4);
    L.off_coloff = o; o = align_up(o + (size_t)p * p * 4);
    L.off_Tk = o;    o = align_up(o + L.nT * 4);
    L.off_Tg = o;    o = align_up(o + L.nT * 4);
    L.off_Sk = o;    o = align_up(o + L.nT * 4);
    L.off_Sg = o;    o = align_up(o + L.nT * 4);
    L.off_lsd = o;   o = align_up(o + std::max(L.LT.bytes, L.LTk.bytes));
    L.off_Y = o;     o = align_up(o + n * 4);
    L.off_YV = o;    o = align_up(o + (has_vals ? n * 4 : 0));
    L.off_seg = o;   o = align_up(o + L.LS.bytes);
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
                       Sg, tab, bkt, counts);
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
    if (vals_in)
        hipLaunchKernelGGL(k_gvr_scatter<true>, dim3(nt), dim3(kGvrWG), 0, stream, keys_in,
                           vals_in, lo, tpb, bkt, counts, bases, (uint32_t)n, Y, YV);
    else
        hipLaunchKernelGGL(k_gvr_scatter<false>, dim3(nt), dim3(kGvrWG), 0, stream, keys_in,
                           nullptr, lo, tpb, bkt, counts, bases, (uint32_t)n, Y, nullptr);
    hipLaunchKernelGGL(k_gvr_stats, dim3(p), dim3(R), 0, stream, counts, bases, (uint32_t)n, p, s,
                       tpb, Sk, Sg, boff, bnd, split_key, split_g);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // 4. every bucket stable-sorted into the output
    return devseg_sort(4, Y, keys_out, YV, vals_out, n, boff, p, kSmallMaxDefault, w + L.off_seg,
                       L.LS, dev_err, stream, prof);
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
