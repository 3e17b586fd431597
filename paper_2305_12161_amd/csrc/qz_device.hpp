// qz_device.hpp -- device-side building blocks shared by the quench kernels:
// the counter-based generator, three-input bitwise helpers and wavefront
// reductions.  gfx950 only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qz {

// ---------------------------------------------------------------------------
// Symmetric three-input bitwise functions as single gfx950 v_bitop3_b32
// instructions.  The truth tables below are symmetric in their three inputs,
// so they do not depend on how the hardware orders the inputs in the index.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}
__device__ __forceinline__ uint32_t and3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x80);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Each round multiplies
// counter words 0 and 2 by the two round multipliers (full 64-bit products),
// then mixes: (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)).
// The key advances by the two Weyl increments between rounds.  Ten rounds.
// ---------------------------------------------------------------------------
struct Words4 {
    uint32_t w[4];
};

__device__ __forceinline__ Words4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        const uint32_t n0 = xor3((uint32_t)(pb >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(pa >> 32), c3, k1);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    Words4 r;
    r.w[0] = c0; r.w[1] = c1; r.w[2] = c2; r.w[3] = c3;
    return r;
}


// acc + popcount(x) as one v_bcnt_u32_b32 (the compiler otherwise tends to
// pair popcounts through v_add3, costing an extra instruction per two).
__device__ __forceinline__ uint32_t popc_acc(uint32_t x, uint32_t acc)
{
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// Funnel shift: the low 32 bits of ((hi:lo) >> s), 0 <= s < 32.
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t s)
{
    return __builtin_amdgcn_alignbit(hi, lo, s);
}

// ---------------------------------------------------------------------------
// The zero-temperature rule on 32 sites of one colour at once (T -> 0 Glauber
// acceptance, Methods).  It is written through the number U of UP neighbours
// (0..6) among the six, which does not depend on the site's own spin.  With a
// the number of anti-aligned neighbours, a = U for a down spin and a = 6 - U
// for an up spin, and the energy change of a flip is 12 - 4a, so:
//   U >= 4           -> the site ends up (a >= 4 flips a down spin; an up
//                       spin has a <= 2 and stays),
//   U <= 2           -> the site ends down (symmetrically),
//   U == 3 (a == 3)  -> the spin flips iff the tie bit r is set: s ^ r.
// In bit planes (U = 4*u2 + 2*u1 + u0; U = 7 is impossible, so u1 & u0 alone
// means U == 3): new = u2 | (u1 & u0 & (s ^ r)).
// ---------------------------------------------------------------------------
struct UpCount {
    uint32_t u0, u1, u2;
};

__device__ __forceinline__ UpCount count_up(uint32_t n0, uint32_t n1, uint32_t n2, uint32_t n3,
                                            uint32_t n4, uint32_t n5)
{
    const uint32_t xa = xor3(n0, n1, n2), ma = maj3(n0, n1, n2);
    const uint32_t xb = xor3(n3, n4, n5), mb = maj3(n3, n4, n5);
    const uint32_t k = xa & xb;
    UpCount u;
    u.u0 = xa ^ xb;
    u.u1 = xor3(ma, mb, k);
    u.u2 = maj3(ma, mb, k);
    return u;
}

__device__ __forceinline__ uint32_t up_tie(const UpCount &u) { return u.u1 & u.u0; }

__device__ __forceinline__ uint32_t up_rule(uint32_t s, const UpCount &u, uint32_t r)
{
    return (up_tie(u) & (s ^ r)) | u.u2;
}

// Sum of the anti-aligned counts a over the 32 sites.  A down site has a = U,
// an up site a = 6 - U; bit-sliced, a = (a2 a1 a0) with a0 = u0 (U and 6 - U
// have the same parity), a1 = u1 ^ (s & ~u0) and a2 = u2 ^ (s & ~(u1 & u0))
// (6 - U = ~U - 1 on three bits), so sum a = popc(a0) + 2 popc(a1) + 4 popc(a2).
__device__ __forceinline__ int up_antialigned_sum(uint32_t s, const UpCount &u)
{
    const uint32_t a1 = u.u1 ^ (s & ~u.u0);
    const uint32_t a2 = u.u2 ^ (s & ~(u.u1 & u.u0));
    return (int)(__builtin_popcount(u.u0) + 2 * __builtin_popcount(a1) +
                 4 * __builtin_popcount(a2));
}

// ---------------------------------------------------------------------------
// Wavefront (64-lane) sum of a 64-bit value; lane 0 ends with the total.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

// Map a linear block id to a tile so that consecutive tiles stay on one XCD.
// Workgroups are dealt round-robin over the 8 XCDs; tile = xcd*(n/8) + k.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t bid, uint32_t nblocks)
{
    if ((nblocks & 7u) != 0u)
        return bid;
    return (bid & 7u) * (nblocks >> 3) + (bid >> 3);
}

}  // namespace qz
