// Device helpers of librbsog: the counter-based generator and the phase
// functions, written for gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rbsog {

// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 64x64->128 multiplies with the published multipliers, Weyl-sequence key
// schedule (golden-ratio and sqrt(3)-1 increments) applied between rounds.
__device__ inline void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1,
                                     uint64_t out[4])
{
    const uint64_t mA = 0xD2E7470EE14C6C93ull, mB = 0xCA5A826395121157ull;
    const uint64_t wA = 0x9E3779B97F4A7C15ull, wB = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hA = __umul64hi(mA, c0), lA = mA * c0;
        uint64_t hB = __umul64hi(mB, c2), lB = mB * c2;
        uint64_t n0 = hB ^ c1 ^ k0, n2 = hA ^ c3 ^ k1;
        c0 = n0;
        c1 = lB;
        c2 = n2;
        c3 = lA;
        k0 += wA;
        k1 += wB;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// sin and cos of 2 pi u for a phase u given in revolutions (FP64).  The
// integer part is removed exactly first (u - rint(u) is exact in FP64), so the
// accuracy does not depend on |u|.
__device__ inline void sincos_rev(double u, double *s, double *c)
{
    double r = u - rint(u);
    sincospi(2.0 * r, s, c);
}

// The same in FP32 after the FP64 reduction to [-1/2, 1/2] revolutions.
__device__ inline void sincos_rev_f32(double u, float *s, float *c)
{
    float r = (float)(u - rint(u));
    sincospif(2.0f * r, s, c);
}

}  // namespace rbsog
