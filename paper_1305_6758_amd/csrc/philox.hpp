// philox.hpp -- Philox4x32-10 counter-based generator for the gfx950 kernels (Salmon, Moraes,
// Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11). Device code only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mmc {
namespace {

constexpr uint32_t PHI_M0 = 0xD2511F53u, PHI_M1 = 0xCD9E8D57u;
constexpr uint32_t PHI_W0 = 0x9E3779B9u, PHI_W1 = 0xBB67AE85u;

struct Words { uint32_t w0, w1, w2, w3; };

__device__ __forceinline__ uint32_t hi32(uint64_t x) { return (uint32_t)(x >> 32); }

// a ^ b ^ c in one VALU instruction (gfx950 v_bitop3_b32, truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96); }

// Philox4x32-10. One round maps (w0, w1, w2, w3) to
// (hi(M1 w2) ^ w1 ^ k0, lo(M1 w2), hi(M0 w0) ^ w3 ^ k1, lo(M0 w0)); the key then moves along
// the Weyl sequence (k0, k1) += (W0, W1). Only c0 (the site) differs between the lanes of a
// wave, so the first two rounds are spelled out to keep their wave-uniform half (c1, c2, c3,
// key) on the scalar unit; later rounds use one three-way xor per output word.
__device__ __forceinline__ Words philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                               uint32_t k1)
{
    uint64_t p0 = (uint64_t)PHI_M0 * c0;
    uint64_t p1 = (uint64_t)PHI_M1 * c2;  // uniform
    const uint32_t a0 = hi32(p1) ^ c1 ^ k0;  // uniform
    const uint32_t a1 = (uint32_t)p1;        // uniform
    const uint32_t a2 = hi32(p0) ^ (c3 ^ k1);
    const uint32_t a3 = (uint32_t)p0;
    k0 += PHI_W0;
    k1 += PHI_W1;
    p0 = (uint64_t)PHI_M0 * a0;  // uniform
    p1 = (uint64_t)PHI_M1 * a2;
    const uint32_t b0 = hi32(p1) ^ (a1 ^ k0);
    const uint32_t b1 = (uint32_t)p1;
    const uint32_t b2 = a3 ^ (hi32(p0) ^ k1);
    const uint32_t b3 = (uint32_t)p0;  // uniform
    k0 += PHI_W0;
    k1 += PHI_W1;
    p0 = (uint64_t)PHI_M0 * b0;
    p1 = (uint64_t)PHI_M1 * b2;
    c0 = xor3(hi32(p1), b1, k0);
    c1 = (uint32_t)p1;
    c2 = hi32(p0) ^ (b3 ^ k1);
    c3 = (uint32_t)p0;
#pragma unroll
    for (int r = 3; r < 10; ++r) {
        k0 += PHI_W0;
        k1 += PHI_W1;
        p0 = (uint64_t)PHI_M0 * c0;
        p1 = (uint64_t)PHI_M1 * c2;
        const uint32_t n0 = xor3(hi32(p1), c1, k0);
        const uint32_t n2 = xor3(hi32(p0), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
    }
    return {c0, c1, c2, c3};
}

}  // namespace
}  // namespace mmc
