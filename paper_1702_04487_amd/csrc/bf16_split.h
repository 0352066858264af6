// bf16_split.h -- a double value stored as a float plus the bfloat16 of its
// remainder (about 40 significant bits in 6 bytes).  Used for the rest
// order-parameter population g_0, which carries +-phi* and whose float
// rounding alone would quantise phi (the zeroth moment of Eq. 9).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ij_bf16 {

__device__ __forceinline__ float bf16_to_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// round-to-nearest-even to bfloat16 (finite inputs)
__device__ __forceinline__ uint16_t float_to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// v = hi + lo with hi = float(v) and lo the bfloat16 of v - hi
__device__ __forceinline__ void split(double v, float& hi, uint16_t& lo)
{
    hi = (float)v;
    lo = float_to_bf16((float)(v - (double)hi));
}

}  // namespace ij_bf16
