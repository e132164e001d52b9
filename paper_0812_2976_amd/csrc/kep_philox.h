// Counter-based random numbers for the population sampler: Philox-4x32-10
// (Salmon, Moraes, Dror and Shaw, SC'11).  Device-only helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kep {

struct U4 {
    uint32_t w0, w1, w2, w3;
};

// Ten rounds of two 32x32->64-bit products with the counter words permuted
// and xored with the key; the key advances by the Weyl increments
// (0x9E3779B9, 0xBB67AE85) before every round but the first.
__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                            uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo_a = 0xD2511F53u * c0, hi_a = __umulhi(0xD2511F53u, c0);
        const uint32_t lo_b = 0xCD9E8D57u * c2, hi_b = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi_b ^ c1 ^ k0, n2 = hi_a ^ c3 ^ k1;
        c0 = n0;
        c1 = lo_b;
        c2 = n2;
        c3 = lo_a;
    }
    return U4{c0, c1, c2, c3};
}

// (0, 1]: 53 random bits n from the top of two words, (n + 1) 2^-53.
__device__ __forceinline__ double unit53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 1.0) * 0x1p-53;
}

// [0, m): floor(w m / 2^32).
__device__ __forceinline__ uint32_t below(uint32_t w, uint32_t m)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)m) >> 32);
}

// Draw j of chain i of half h at generation g.
__device__ __forceinline__ U4 demc_draw(uint32_t key0, uint32_t key1, int h, uint32_t i, uint32_t j, uint64_t g)
{
    return philox4x32_10(i, j, (uint32_t)g, (uint32_t)(g >> 32) | ((uint32_t)h << 31), key0, key1);
}

}  // namespace kep
