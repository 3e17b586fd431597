// qz_cube.hpp -- cube masks of the double checkerboard (Supplementary Methods
// I A, I B) on the 1-bit colour-separated layout: bit b of word w of a colour
// row lies at x = 64w + 2b + pi, i.e. in cube column (32w + b) >> (sB - 1)
// for cubes of side B = 2^sB.  gfx950 only.
#pragma once
#include "qz_device.hpp"

namespace qz {

// Each of the low 32 >> q bits of `bits` (bit k: the k-th cube a word
// crosses) becomes a run of 2^q bits: q doubling steps, each moving bit k to
// bit 2k (at most 16 significant bits going in) and copying it to bit 2k + 1.
// From q = 5 on one cube covers the whole word.
__device__ __forceinline__ uint32_t cube_bits_mask(uint32_t bits, uint32_t q)
{
    if (q >= 5)
        return (bits & 1u) ? 0xFFFFFFFFu : 0u;
    uint32_t x = q == 0 ? bits : bits & ((1u << (32u >> q)) - 1u);
    for (uint32_t s = 0; s < q; ++s) {
        x = (x | (x << 8)) & 0x00FF00FFu;
        x = (x | (x << 4)) & 0x0F0F0F0Fu;
        x = (x | (x << 2)) & 0x33333333u;
        x = (x | (x << 1)) & 0x55555555u;
        x |= x << 1;
    }
    return x;
}

// The sites of word w (row y, plane z) whose cube updates fine colour 1 first
// in sweep t of the mixed cycle: cube b = bx + nb (by + nb bz), nb = L / B,
// takes fine colour 1 first iff bit b of the Philox blocks (b / 128, t, 4, 0)
// is set (bit k of a block = bit k & 31 of its word k >> 5).  The cubes a word
// crosses never straddle two Philox words (L is a multiple of 64).
__device__ __forceinline__ uint32_t cube_order_mask(uint32_t w, uint32_t y, uint32_t z,
                                                    uint32_t L, uint32_t sB, uint32_t k0,
                                                    uint32_t k1, uint32_t t)
{
    const uint32_t q = sB - 1;
    const uint32_t nb = L >> sB;
    const uint64_t cb0 = (uint64_t)((32u * w) >> q) +
                         (uint64_t)nb * ((uint64_t)(y >> sB) + (uint64_t)nb * (z >> sB));
    const Words4 o = philox10((uint32_t)(cb0 >> 7), t, 4u, 0u, k0, k1);
    const uint32_t sub = (uint32_t)(cb0 >> 5) & 3u;
    const uint32_t word = (sub & 2u) ? ((sub & 1u) ? o.w[3] : o.w[2])
                                     : ((sub & 1u) ? o.w[1] : o.w[0]);
    return cube_bits_mask(word >> (uint32_t)(cb0 & 31u), q);
}

}  // namespace qz
