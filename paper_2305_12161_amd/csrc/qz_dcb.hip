// qz_dcb.hip -- the double checkerboard (Supplementary Methods I A, I B) as
// in-place phases over the 1-bit colour-separated layout (plane c = words
// [z][y][W], W = L/64, bit b of word w = site x = 64w + 2b + pi).  A sweep of
// the 01 cycle can also run as one pass of the four-stage kernel (its DCB
// flag); the phases here serve the mixed cycle and one sweep per pass.
#include "qz_bitops.hpp"
#include "qz_cube.hpp"
#include "qz_device.hpp"
#include "qz_internal.hpp"

namespace qz {
namespace {

uint32_t grid_cap(uint64_t work, uint32_t cap)
{
    uint64_t g = (work + 255) / 256;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

// --------------------------------------------------------------------------
// Double checkerboard (Supplementary Methods I A): cubes of side B = 2^sB form
// a coarse checkerboard, coarse colour (x/B + y/B + z/B) & 1.  One phase
// updates, in place, the fine-colour-p sites of the coarse-colour-cc cubes;
// they read only fine colour 1-p, so threads never race.  Thread per word of
// plane p; the sites outside the phase are masked out.
//
// Mixed cycle (Supplementary Methods I B): the coarse colour updated first is
// drawn once per sweep (coarse colour 1 first iff bit 0 of word 0 of Philox
// block (0, t, 3, 0)), and each cube draws its fine order once per sweep (fine
// colour 1 first iff bit b of blocks (b / 128, t, 4, 0), b = bx + nb (by + nb
// bz) the cube index, nb = L / B).  Then `kc` is the position of the coarse
// colour in the sweep's order and `step` selects, per cube, the fine colour
// (first ^ step); a launch for plane p masks in the cubes whose fine colour
// of this step is p.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
    k_bit_phase(uint32_t L, uint32_t W, uint32_t sB, uint32_t kc, uint32_t p, uint32_t k0,
                uint32_t k1, uint32_t t, uint32_t *Pp, const uint32_t *Po, uint32_t mixed,
                uint32_t step, unsigned long long *flip_acc)
{
    uint32_t flips = 0;
    const uint64_t nwords = (uint64_t)L * L * W;
    const size_t plane = (size_t)L * W;
    const uint32_t cc = mixed ? (kc ^ (philox10(0u, t, 3u, 0u, k0, k1).w[0] & 1u)) : kc;
    // bit b of a word holds x = 64w + 2b + pi, so x / B = (32w + b) >> (sB - 1)
    const uint32_t q = sB - 1;
    const uint32_t pat = (q == 0) ? 0xAAAAAAAAu : (q == 1) ? 0xCCCCCCCCu : (q == 2) ? 0xF0F0F0F0u
                       : (q == 3) ? 0xFF00FF00u : (q == 4) ? 0xFFFF0000u : 0u;
    for (uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x; g < nwords;
         g += (uint64_t)gridDim.x * 256) {
        const uint32_t w = (uint32_t)(g % W);
        const uint64_t row = g / W;
        const uint32_t y = (uint32_t)(row % L), z = (uint32_t)(row / L);
        const uint32_t A = (((32u * w) >> q) + (y >> sB) + (z >> sB)) & 1u;
        uint32_t mask = ((A ^ cc) & 1u) ? pat : ~pat;
        if (mixed && mask != 0u) {
            // cubes whose fine colour in this step is p: first == p ^ step
            const uint32_t first1 = cube_order_mask(w, y, z, L, sB, k0, k1, t);
            mask &= ((p ^ step) & 1u) ? first1 : ~first1;
        }
        if (mask == 0u)
            continue;
        const uint32_t pi = (p + y + z) & 1u;
        const size_t rb = (size_t)row * W;
        const uint32_t own = Pp[g], same = Po[g];
        const uint32_t sh = pi ? funnel(Po[rb + (w + 1) % W], same, 1)
                               : funnel(same, Po[rb + (w + W - 1) % W], 31);
        const size_t zb = (size_t)z * plane;
        const UpCount u = count_up(same, sh, Po[zb + (size_t)((y + L - 1) % L) * W + w],
                                   Po[zb + (size_t)((y + 1) % L) * W + w],
                                   Po[(size_t)((z + L - 1) % L) * plane + (size_t)y * W + w],
                                   Po[(size_t)((z + 1) % L) * plane + (size_t)y * W + w]);
        uint32_t r = 0u;
        if ((up_tie(u) & mask) != 0u) {
            const Words4 rb4 = philox10((uint32_t)(g >> 2), t, p, 0u, k0, k1);
            const uint32_t sub = (uint32_t)(g & 3u);
            const uint32_t lo = (sub & 1u) ? rb4.w[1] : rb4.w[0];
            const uint32_t hi = (sub & 1u) ? rb4.w[3] : rb4.w[2];
            r = (sub & 2u) ? hi : lo;
        }
        const uint32_t nw = up_rule(own, u, r);
        Pp[g] = (own & ~mask) | (nw & mask);
        flips = popc_acc((own ^ nw) & mask, flips);
    }
    if (flip_acc != nullptr) {
        const unsigned long long ws = wave_sum_u64((unsigned long long)flips);
        if ((threadIdx.x & 63) == 0 && ws)
            atomicAdd(flip_acc, ws);
    }
}

// The same phase with four consecutive words per lane (W % 4 == 0): one
// Philox block covers the lane's tie bits (its first word index is a multiple
// of 4), the words move as 16-byte vectors, and the rows come from a 2D
// mapping instead of 64-bit divisions.  In the mixed cycle the cube-order
// bits of the four words come from at most two Philox blocks.

__global__ void __launch_bounds__(256)
    k_bit_phase4(uint32_t L, uint32_t W, uint32_t sB, uint32_t kc, uint32_t p, uint32_t k0,
                 uint32_t k1, uint32_t t, uint32_t *Pp, const uint32_t *Po, uint32_t mixed,
                 uint32_t step, unsigned long long *flip_acc)
{
    uint32_t flips = 0;
    const uint32_t R = W / 4;                       // lanes per row
    const uint32_t rpb = 256u / R;                  // rows per block
    const uint32_t lr = threadIdx.x / R;
    const uint32_t row = blockIdx.x * rpb + lr;     // z * L + y
    const bool act = lr < rpb && row < L * L;
    const uint32_t cc = mixed ? (kc ^ (philox10(0u, t, 3u, 0u, k0, k1).w[0] & 1u)) : kc;
    const uint32_t q = sB - 1;
    const uint32_t pat = (q == 0) ? 0xAAAAAAAAu : (q == 1) ? 0xCCCCCCCCu : (q == 2) ? 0xF0F0F0F0u
                       : (q == 3) ? 0xFF00FF00u : (q == 4) ? 0xFFFF0000u : 0u;
    if (act) {
        const uint32_t w0 = (threadIdx.x % R) * 4u;
        const uint32_t y = row % L, z = row / L;
        uint32_t mask[4], any = 0u;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const uint32_t w = w0 + (uint32_t)v;
            const uint32_t A = (((32u * w) >> q) + (y >> sB) + (z >> sB)) & 1u;
            mask[v] = ((A ^ cc) & 1u) ? pat : ~pat;
            any |= mask[v];
        }
        if (mixed && any != 0u) {
            // cubes whose fine colour in this step is p: first == p ^ step
            const uint32_t nb = L >> sB;
            const uint64_t cbase = (uint64_t)nb * ((uint64_t)(y >> sB) + (uint64_t)nb * (z >> sB));
            uint32_t blk = 0xFFFFFFFFu;
            Words4 o;
            any = 0u;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint64_t cb0 = (uint64_t)((32u * (w0 + (uint32_t)v)) >> q) + cbase;
                if ((uint32_t)(cb0 >> 7) != blk) {
                    blk = (uint32_t)(cb0 >> 7);
                    o = philox10(blk, t, 4u, 0u, k0, k1);
                }
                const uint32_t sub = (uint32_t)(cb0 >> 5) & 3u;
                const uint32_t word = (sub & 2u) ? ((sub & 1u) ? o.w[3] : o.w[2])
                                                 : ((sub & 1u) ? o.w[1] : o.w[0]);
                const uint32_t first1 = cube_bits_mask(word >> (uint32_t)(cb0 & 31u), q);
                mask[v] &= ((p ^ step) & 1u) ? first1 : ~first1;
                any |= mask[v];
            }
        }
        if (any != 0u) {
            const uint32_t pi = (p + y + z) & 1u;
            const size_t plane = (size_t)L * W;
            const size_t rb = (size_t)row * W;
            const size_t zb = (size_t)z * plane;
            uint32_t own[4], same[4], ym[4], yp[4], zm[4], zp[4];
            bitops::load_words<4>(Pp + rb + w0, own);
            bitops::load_words<4>(Po + rb + w0, same);
            bitops::load_words<4>(Po + zb + (size_t)((y + L - 1) % L) * W + w0, ym);
            bitops::load_words<4>(Po + zb + (size_t)((y + 1) % L) * W + w0, yp);
            bitops::load_words<4>(Po + (size_t)((z + L - 1) % L) * plane + (size_t)y * W + w0, zm);
            bitops::load_words<4>(Po + (size_t)((z + 1) % L) * plane + (size_t)y * W + w0, zp);
            const uint32_t adj = pi ? Po[rb + (w0 + 4u) % W] : Po[rb + (w0 + W - 1u) % W];
            UpCount u[4];
            uint32_t ties = 0u;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                u[v] = count_up(same[v], bitops::shifted_word<4>(same, adj, pi, v), ym[v], yp[v],
                                zm[v], zp[v]);
                ties |= up_tie(u[v]) & mask[v];
            }
            uint32_t r[4] = {0u, 0u, 0u, 0u};
            if (ties != 0u) {
                const Words4 rb4 = philox10((uint32_t)((rb + w0) >> 2), t, p, 0u, k0, k1);
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    r[v] = rb4.w[v];
            }
            uint32_t nw[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t n = up_rule(own[v], u[v], r[v]);
                nw[v] = (own[v] & ~mask[v]) | (n & mask[v]);
                flips = popc_acc(own[v] ^ nw[v], flips);
            }
            bitops::store_words<4>(Pp + rb + w0, nw);
        }
    }
    if (flip_acc != nullptr) {
        const unsigned long long ws = wave_sum_u64((unsigned long long)flips);
        if ((threadIdx.x & 63) == 0 && ws)
            atomicAdd(flip_acc, ws);
    }
}

// Mixed cycle, both fine colours of one step in one launch: in step `step`
// of coarse colour cc each cube updates the fine colour first ^ step, so the
// cubes updating colour 0 and those updating colour 1 are disjoint, and every
// neighbour an update reads lies in its own cube (whose other colour waits
// for the next step) or in a cube of the other coarse colour (not updated in
// this step).  A lane updates its words of both planes, each under its own
// mask; the bits another lane may be rewriting at the same time are never
// ones its masked updates read.
__device__ __forceinline__ void phase4_plane(uint32_t L, uint32_t W, uint32_t y, uint32_t z,
                                             uint32_t w0, uint32_t p, uint32_t k0, uint32_t k1,
                                             uint32_t t, uint32_t *Pp, const uint32_t *Po,
                                             const uint32_t (&mask)[4], uint32_t &flips)
{
    const uint32_t pi = (p + y + z) & 1u;
    const size_t plane = (size_t)L * W;
    const size_t rb = ((size_t)z * L + y) * W;
    const size_t zb = (size_t)z * plane;
    uint32_t own[4], same[4], ym[4], yp[4], zm[4], zp[4];
    bitops::load_words<4>(Pp + rb + w0, own);
    bitops::load_words<4>(Po + rb + w0, same);
    bitops::load_words<4>(Po + zb + (size_t)((y + L - 1) % L) * W + w0, ym);
    bitops::load_words<4>(Po + zb + (size_t)((y + 1) % L) * W + w0, yp);
    bitops::load_words<4>(Po + (size_t)((z + L - 1) % L) * plane + (size_t)y * W + w0, zm);
    bitops::load_words<4>(Po + (size_t)((z + 1) % L) * plane + (size_t)y * W + w0, zp);
    const uint32_t adj = pi ? Po[rb + (w0 + 4u) % W] : Po[rb + (w0 + W - 1u) % W];
    UpCount u[4];
    uint32_t ties = 0u;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        u[v] = count_up(same[v], bitops::shifted_word<4>(same, adj, pi, v), ym[v], yp[v], zm[v],
                        zp[v]);
        ties |= up_tie(u[v]) & mask[v];
    }
    uint32_t r[4] = {0u, 0u, 0u, 0u};
    if (ties != 0u) {
        const Words4 rb4 = philox10((uint32_t)((rb + w0) >> 2), t, p, 0u, k0, k1);
#pragma unroll
        for (int v = 0; v < 4; ++v)
            r[v] = rb4.w[v];
    }
    uint32_t nw[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const uint32_t n = up_rule(own[v], u[v], r[v]);
        nw[v] = (own[v] & ~mask[v]) | (n & mask[v]);
        flips = popc_acc(own[v] ^ nw[v], flips);
    }
    bitops::store_words<4>(Pp + rb + w0, nw);
}

__global__ void __launch_bounds__(256)
    k_bit_phase4_mixed(uint32_t L, uint32_t W, uint32_t sB, uint32_t kc, uint32_t k0, uint32_t k1,
                       uint32_t t, uint32_t *P0, uint32_t *P1, uint32_t step,
                       unsigned long long *flip_acc)
{
    uint32_t flips = 0;
    const uint32_t R = W / 4;
    const uint32_t rpb = 256u / R;
    const uint32_t lr = threadIdx.x / R;
    const uint32_t row = blockIdx.x * rpb + lr;
    const bool act = lr < rpb && row < L * L;
    const uint32_t cc = kc ^ (philox10(0u, t, 3u, 0u, k0, k1).w[0] & 1u);
    const uint32_t q = sB - 1;
    const uint32_t pat = (q == 0) ? 0xAAAAAAAAu : (q == 1) ? 0xCCCCCCCCu : (q == 2) ? 0xF0F0F0F0u
                       : (q == 3) ? 0xFF00FF00u : (q == 4) ? 0xFFFF0000u : 0u;
    if (act) {
        const uint32_t w0 = (threadIdx.x % R) * 4u;
        const uint32_t y = row % L, z = row / L;
        // a word's bit b lies in cube column (32 w + b) >> (sB - 1) in both
        // planes, so the cube masks are shared
        uint32_t m0[4], m1[4], any0 = 0u, any1 = 0u;
        const uint32_t nb = L >> sB;
        const uint64_t cbase = (uint64_t)nb * ((uint64_t)(y >> sB) + (uint64_t)nb * (z >> sB));
        uint32_t blk = 0xFFFFFFFFu;
        Words4 o;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const uint32_t w = w0 + (uint32_t)v;
            const uint32_t A = (((32u * w) >> q) + (y >> sB) + (z >> sB)) & 1u;
            const uint32_t cm = ((A ^ cc) & 1u) ? pat : ~pat;
            const uint64_t cb0 = (uint64_t)((32u * w) >> q) + cbase;
            if ((uint32_t)(cb0 >> 7) != blk) {
                blk = (uint32_t)(cb0 >> 7);
                o = philox10(blk, t, 4u, 0u, k0, k1);
            }
            const uint32_t sub = (uint32_t)(cb0 >> 5) & 3u;
            const uint32_t word = (sub & 2u) ? ((sub & 1u) ? o.w[3] : o.w[2])
                                             : ((sub & 1u) ? o.w[1] : o.w[0]);
            const uint32_t first1 = cube_bits_mask(word >> (uint32_t)(cb0 & 31u), q);
            // fine colour p this step where first == p ^ step
            m0[v] = cm & ((step & 1u) ? first1 : ~first1);
            m1[v] = cm & ((step & 1u) ? ~first1 : first1);
            any0 |= m0[v];
            any1 |= m1[v];
        }
        if (any0 != 0u)
            phase4_plane(L, W, y, z, w0, 0u, k0, k1, t, P0, P1, m0, flips);
        if (any1 != 0u)
            phase4_plane(L, W, y, z, w0, 1u, k0, k1, t, P1, P0, m1, flips);
    }
    if (flip_acc != nullptr) {
        const unsigned long long ws = wave_sum_u64((unsigned long long)flips);
        if ((threadIdx.x & 63) == 0 && ws)
            atomicAdd(flip_acc, ws);
    }
}

}  // namespace

hipError_t bit_double_sweep(hipStream_t st, uint32_t L, uint32_t B, uint64_t seed, uint32_t t,
                            uint32_t *P0, uint32_t *P1, bool mixed, unsigned long long *flip_acc)
{
    uint32_t sB = 0;
    while ((1u << sB) < B)
        ++sB;
    if (B < 2 || (1u << sB) != B || L % (2 * B))
        return hipErrorInvalidValue;
    const uint32_t W = L / 64;
    const uint64_t nw = (uint64_t)L * L * W;
    // 01 cycle: (coarse, fine) = (0,0), (0,1), (1,0), (1,1).  Mixed cycle: for
    // each coarse colour in the drawn order, two steps, each one launch per plane.
    const uint32_t nsteps = mixed ? 2u : 1u;
    const bool quads = W % 4 == 0;
    const uint32_t rpb = quads ? 256u / (W / 4) : 1u;
    const dim3 grid4((uint32_t)(((uint64_t)L * L + rpb - 1) / rpb));
    if (quads && mixed) {
        // both fine colours of a step in one launch (cubes are independent)
        for (uint32_t kc = 0; kc < 2; ++kc)
            for (uint32_t step = 0; step < 2; ++step) {
                hipLaunchKernelGGL(k_bit_phase4_mixed, grid4, dim3(256), 0, st, L, W, sB, kc,
                                   (uint32_t)seed, (uint32_t)(seed >> 32), t, P0, P1, step,
                                   flip_acc);
                const hipError_t e = hipGetLastError();
                if (e != hipSuccess)
                    return e;
            }
        return hipSuccess;
    }
    for (uint32_t kc = 0; kc < 2; ++kc)
        for (uint32_t step = 0; step < nsteps; ++step)
            for (uint32_t p = 0; p < 2; ++p) {
                if (quads)
                    hipLaunchKernelGGL(k_bit_phase4, grid4, dim3(256), 0, st, L, W, sB, kc, p,
                                       (uint32_t)seed, (uint32_t)(seed >> 32), t, p ? P1 : P0,
                                       p ? P0 : P1, mixed ? 1u : 0u, step, flip_acc);
                else
                    hipLaunchKernelGGL(k_bit_phase, dim3(grid_cap(nw, 8192)), dim3(256), 0, st, L,
                                       W, sB, kc, p, (uint32_t)seed, (uint32_t)(seed >> 32), t,
                                       p ? P1 : P0, p ? P0 : P1, mixed ? 1u : 0u, step, flip_acc);
                const hipError_t e = hipGetLastError();
                if (e != hipSuccess)
                    return e;
            }
    return hipSuccess;
}

hipError_t bit_double_phase(hipStream_t st, uint32_t L, uint32_t B, uint64_t seed, uint32_t t,
                            uint32_t *P0, uint32_t *P1, uint32_t kc, uint32_t p, uint32_t step,
                            bool mixed, unsigned long long *flip_acc)
{
    uint32_t sB = 0;
    while ((1u << sB) < B)
        ++sB;
    if (B < 2 || (1u << sB) != B || L % (2 * B) || kc > 1 || p > 1 || step > 1)
        return hipErrorInvalidValue;
    const uint32_t W = L / 64;
    if (W % 4 == 0) {
        const uint32_t rpb = 256u / (W / 4);
        const dim3 grid4((uint32_t)(((uint64_t)L * L + rpb - 1) / rpb));
        hipLaunchKernelGGL(k_bit_phase4, grid4, dim3(256), 0, st, L, W, sB, kc, p,
                           (uint32_t)seed, (uint32_t)(seed >> 32), t, p ? P1 : P0, p ? P0 : P1,
                           mixed ? 1u : 0u, step, flip_acc);
    } else {
        const uint64_t nw = (uint64_t)L * L * W;
        hipLaunchKernelGGL(k_bit_phase, dim3(grid_cap(nw, 8192)), dim3(256), 0, st, L, W, sB, kc,
                           p, (uint32_t)seed, (uint32_t)(seed >> 32), t, p ? P1 : P0, p ? P0 : P1,
                           mixed ? 1u : 0u, step, flip_acc);
    }
    return hipGetLastError();
}

}  // namespace qz
