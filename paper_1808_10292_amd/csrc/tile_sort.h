// In-LDS stable counting round over a tile held by one workgroup: the count
// sort of arXiv 1808.10292 Section 3.2 (count, exclusive prefix, stable
// placement) on up to WG * ITEMS keys, with digits of at most 8 bits.
//
// Register layout ("ranking layout"): half-wave h (32 lanes) owns tile
// positions [h * NI * 32, (h + 1) * NI * 32); its lane l holds, in register
// i < NI, position h * NI * 32 + 32 i + l.  Positions >= len, and registers
// i >= NI, are empty.  NI (at most ITEMS) is ITEMS unless the caller spreads
// a short tile over every half-wave: NI = ceil(len / (32 * half-waves)).
//
// A round: every half-wave counts its digits into its own 256 slots, the
// slots are turned into the first output position of (half-wave, digit) in
// half-wave order, then each key gets its rank among the equal digits of its
// half-wave, rows in order (lane set bits of a 64-bit slot {lane mask, count}),
// keys and payloads are restaged in LDS at their new positions and read back
// in the ranking layout.  Stable because half-waves and rows are visited in
// position order.  A round in which one digit value holds every key moves
// nothing and is skipped.
#pragma once

#include "device_common.h"

namespace rsort {
namespace {

constexpr uint32_t kTileRadix = 256;

// SHARED: the slots and the key staging share their LDS (they are never live
// together; one more barrier separates the ranking from the restaging), so
// more workgroups fit a CU.  The keys of an identity round then do not stay
// in LDS.
template <typename K, bool KV, int WG, int ITEMS, bool SHARED = false>
struct TileSmem {
    static constexpr uint32_t TILE = (uint32_t)WG * ITEMS;
    static constexpr int HW = WG / 32;
    K keys[TILE];
    uint32_t vals[KV ? TILE : 1];
    uint2 slot[HW][kTileRadix];
    uint32_t wsum[4];
};
template <typename K, bool KV, int WG, int ITEMS>
struct TileSmem<K, KV, WG, ITEMS, true> {
    static constexpr uint32_t TILE = (uint32_t)WG * ITEMS;
    static constexpr int HW = WG / 32;
    union {
        K keys[TILE];
        uint2 slot[HW][kTileRadix];
    };
    uint32_t vals[KV ? TILE : 1];
    uint32_t wsum[4];
};

// Returns false if the round was the identity (nothing moved, LDS keys[]
// untouched); true if k / v now hold the new order and LDS keys[] / vals[]
// hold the tile in that order.  Every thread of the workgroup must call it.
template <typename K, bool KV, int WG, int ITEMS, bool SHARED>
__device__ __forceinline__ bool tile_round(TileSmem<K, KV, WG, ITEMS, SHARED>& sm, K (&k)[ITEMS], uint32_t (&v)[ITEMS],
                           uint32_t len, uint32_t shift, uint32_t mask, uint32_t ni = ITEMS)
{
    constexpr int HW = WG / 32;
    constexpr uint32_t R = kTileRadix;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    const uint32_t wave = tid >> 6;
    const uint32_t hw = tid >> 5;
    const uint32_t hl = tid & 31;
    const uint32_t hofs = hw * ni * 32 + hl;

    for (uint32_t i = tid; i < HW * R / 2; i += WG)
        ((uint4*)&sm.slot[0][0])[i] = make_uint4(0, 0, 0, 0);
    __syncthreads();
    // count
    uint2* sl = sm.slot[hw];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if ((uint32_t)i >= ni) continue;   // ni is uniform over the workgroup
        const bool ok = hofs + i * 32 < len;
        const uint32_t d = digit_of(k[i], shift, mask);
        if (wave_one_digit(ok, d)) {   // whole wave one digit: one add per half-wave
            if (hl == 0) atomicAdd(&sl[d].y, 32u);
            continue;
        }
        if (ok) atomicAdd(&sl[d].y, 1u);
    }
    __syncthreads();
    // bases
    uint32_t run = 0, total = 0;
    if (tid < R) {
#pragma unroll
        for (int h = 0; h < HW; ++h) total += sm.slot[h][tid].y;
        const uint32_t incl = wave_inclusive_sum(total);
        if (lane == 63) sm.wsum[wave] = incl;
        run = incl - total;
    }
    // barrier + "some digit value holds every key": the round is the identity
    if (__syncthreads_or(tid < R && total == len)) return false;
    if (tid < R) {
        for (uint32_t w = 0; w < wave; ++w) run += sm.wsum[w];
#pragma unroll
        for (int h = 0; h < HW; ++h) {
            const uint32_t c = sm.slot[h][tid].y;
            sm.slot[h][tid].y = run;
            run += c;
        }
    }
    __syncthreads();
    // rank
    uint32_t pos[ITEMS];
    {
        const uint32_t bit = 1u << hl;
        const uint32_t lowsel = lane < 32 ? ~0u : 0u;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if ((uint32_t)i >= ni) continue;
            const bool ok = hofs + i * 32 < len;
            const uint32_t d = digit_of(k[i], shift, mask);
            if (wave_one_digit(ok, d)) {   // whole wave one digit: ranks in lane order
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
    // restage in the new order and reload in the ranking layout
    if constexpr (SHARED) __syncthreads();   // every slot read before keys overwrite them
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if ((uint32_t)i < ni && hofs + i * 32 < len) {
            sm.keys[pos[i]] = k[i];
            if (KV) sm.vals[pos[i]] = v[i];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t o = hofs + i * 32;
        if ((uint32_t)i < ni && o < len) {
            k[i] = sm.keys[o];
            if (KV) v[i] = sm.vals[o];
        }
    }
    __syncthreads();
    return true;
}

}  // namespace
}  // namespace rsort
