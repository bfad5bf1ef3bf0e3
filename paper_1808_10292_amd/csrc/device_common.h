// Device helpers shared by the gfx950 kernels of the library (wave64 CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsort {

// Packed decoupled look-back word: 2-bit flag | 30-bit count (n < 2^30).
constexpr uint32_t kFlagShift = 30;
constexpr uint32_t kFlagAggregate = 1u << kFlagShift;   // tile's own count only
constexpr uint32_t kFlagPrefix = 2u << kFlagShift;      // inclusive prefix up to the tile
constexpr uint32_t kCountMask = (1u << kFlagShift) - 1;

// A look-back poll gives up after this many sleeps (each tens of ns plus a
// memory round trip) and records kErrLookbackTimeout instead of hanging.
constexpr uint32_t kSpinLimit = 1u << 20;

enum DeviceError : uint32_t {
    kErrNone = 0,
    kErrLookbackTimeout = 1u << 0,
    kErrBadPlan = 1u << 1,
};

__device__ __forceinline__ uint32_t lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of the 64-bit lane mask below this lane, plus `add`.
__device__ __forceinline__ uint32_t mbcnt64(uint64_t mask, uint32_t add)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, add));
}

// Keeps the compiler from moving LDS accesses across this point; the hardware
// already executes one wave's LDS instructions in order.
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T ld_agent(const T* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x)
{
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    return x;
}

// True (for the whole wave) when every lane of the wave is valid and holds
// the same digit d: then the lanes of a 32-lane group rank in lane order.
__device__ __forceinline__ bool wave_one_digit(bool valid, uint32_t d)
{
    const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d);
    return __builtin_amdgcn_ballot_w64(valid && d == d0) == ~0ull;
}

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, uint32_t shift, uint32_t mask)
{
    return (uint32_t)(key >> shift) & mask;
}

}  // namespace rsort
