// Signed and IEEE-754 floating-point keys sorted by the unsigned radix rounds:
// an order-preserving bijection maps each key to an unsigned integer of the
// same width, the unsigned sort runs, and the inverse restores the keys.
//   signed   flip the sign bit (two's complement order = offset order);
//   float    negative (sign bit set): complement every bit; otherwise flip the
//            sign bit.  The result orders keys by IEEE 754 totalOrder:
//            -NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN.
#include <algorithm>

#include "device_common.h"
#include "rsort_internal.h"

namespace rsort {
namespace {

template <typename U>
__device__ __forceinline__ U to_ordered(U x, int kind)
{
    constexpr U sign = U(1) << (sizeof(U) * 8 - 1);
    if (kind == kKeySigned) return x ^ sign;
    return (x & sign) ? U(~x) : U(x ^ sign);
}

template <typename U>
__device__ __forceinline__ U from_ordered(U y, int kind)
{
    constexpr U sign = U(1) << (sizeof(U) * 8 - 1);
    if (kind == kKeySigned) return y ^ sign;
    return (y & sign) ? U(y ^ sign) : U(~y);
}

constexpr int kMapItems = 8;

template <typename U, bool INVERSE>
__global__ void k_map_keys(const U* __restrict__ in, U* out, size_t n, int kind)
{
    // kMapItems keys per thread, all loaded before the first store
    const size_t base = (size_t)blockIdx.x * blockDim.x * kMapItems + threadIdx.x;
    U x[kMapItems];
#pragma unroll
    for (int j = 0; j < kMapItems; ++j) {
        const size_t i = base + (size_t)j * blockDim.x;
        x[j] = i < n ? in[i] : U(0);
    }
#pragma unroll
    for (int j = 0; j < kMapItems; ++j) {
        const size_t i = base + (size_t)j * blockDim.x;
        if (i < n) out[i] = INVERSE ? from_ordered<U>(x[j], kind) : to_ordered<U>(x[j], kind);
    }
}

}  // namespace

hipError_t map_keys(int key_bytes, int kind, bool inverse, const void* in, void* out, size_t n,
                    hipStream_t stream)
{
    if (!n) return hipSuccess;
    const dim3 grid((uint32_t)((n + 256 * kMapItems - 1) / (256 * kMapItems))), block(256);
    if (key_bytes == 4) {
        if (inverse)
            hipLaunchKernelGGL((k_map_keys<uint32_t, true>), grid, block, 0, stream,
                               (const uint32_t*)in, (uint32_t*)out, n, kind);
        else
            hipLaunchKernelGGL((k_map_keys<uint32_t, false>), grid, block, 0, stream,
                               (const uint32_t*)in, (uint32_t*)out, n, kind);
    } else {
        if (inverse)
            hipLaunchKernelGGL((k_map_keys<uint64_t, true>), grid, block, 0, stream,
                               (const uint64_t*)in, (uint64_t*)out, n, kind);
        else
            hipLaunchKernelGGL((k_map_keys<uint64_t, false>), grid, block, 0, stream,
                               (const uint64_t*)in, (uint64_t*)out, n, kind);
    }
    return hipGetLastError();
}

}  // namespace rsort
