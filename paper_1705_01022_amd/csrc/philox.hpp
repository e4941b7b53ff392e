// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11,
// "Parallel random numbers: as easy as 1, 2, 3"): ten rounds of
//   (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key advanced by the Weyl increments between rounds.
//
// The octahedron simulation draws every random number it needs from this
// generator, keyed by (seed, stream) with counters built from the MCS,
// device step, tile, cell and round, so results are independent of the
// launch configuration.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace okpz {

struct u32x4 {
    uint32_t x, y, z, w;
};

__host__ __device__ __forceinline__ void mul_hilo(uint32_t a, uint32_t b, uint32_t &hi, uint32_t &lo)
{
    const uint64_t prod = static_cast<uint64_t>(a) * static_cast<uint64_t>(b);
    hi = static_cast<uint32_t>(prod >> 32);
    lo = static_cast<uint32_t>(prod);
}

__host__ __device__ __forceinline__ u32x4 philox4x32_10(uint32_t k0, uint32_t k1, uint32_t c0,
                                                       uint32_t c1, uint32_t c2, uint32_t c3)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hiA, loA, hiB, loB;
        mul_hilo(kMulA, c0, hiA, loA);
        mul_hilo(kMulB, c2, hiB, loB);
        const uint32_t n0 = hiB ^ c1 ^ k0;
        const uint32_t n2 = hiA ^ c3 ^ k1;
        c0 = n0;
        c1 = loB;
        c2 = n2;
        c3 = loA;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return u32x4{c0, c1, c2, c3};
}

// The same generator for counters that differ between the lanes of a wave:
// each round's two three-way XORs are one gfx950 three-input bit operation
// each (truth table 0x96), four VALU instructions fewer per round.  Uniform
// counters keep philox4x32_10, which the compiler runs on the scalar unit.
__device__ __forceinline__ u32x4 philox4x32_10_lane(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                                                    uint32_t c3)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hiA, loA, hiB, loB;
        mul_hilo(kMulA, c0, hiA, loA);
        mul_hilo(kMulB, c2, hiB, loB);
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hiB, c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hiA, c3, k1, 0x96);
        c0 = n0;
        c1 = loB;
        c2 = n2;
        c3 = loA;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return u32x4{c0, c1, c2, c3};
}

}  // namespace okpz
