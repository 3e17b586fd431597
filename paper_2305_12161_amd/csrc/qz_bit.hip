// qz_bit.hip -- kernels for the 1-bit, colour-separated layout.
//
// Plane c (c = 0, 1) holds the colour-c sites as 32-bit words
//   P_c[(z*L + y)*W + w],  W = L/64,
// bit b of word w being the site x = 64w + 2b + pi with pi = (c + y + z) & 1
// (all colour-c sites of one row share the parity of x).  A colour-c site at
// x = 2k + pi has its two x-neighbours at colour indices k and k-1 (pi = 0) or
// k and k+1 (pi = 1) of the other colour's same row; its y- and z-neighbours
// are bit k of the other colour's rows (y+-1, z) and (y, z+-1).  The word index
// g = (z*L + y)*W + w equals j/32 for the colour index j of the contract, so the
// tie bits of word g are word (g & 3) of the Philox block g >> 2.
//
// The sweep (colour 0 then colour 1, Methods "Checkerboard update") is fused
// into ONE pass over memory that reads copy A and writes copy B: a workgroup
// owns a tile of Ty rows x all of x x Tz planes and streams it along z.  At
// plane step q it updates colour 0 of plane q (from old colour 1 of planes
// q-1, q, q+1) and then colour 1 of plane q-1 (from the new colour 0 of planes
// q-2, q-1, q), so each word is read once and written once per sweep.  The
// new colour 0 is recomputed for one halo row on each side and one halo plane
// at each end of the tile (from copy A, so tiles never race).  Rows are
// exchanged through LDS, one barrier per plane step.
#include "qz_bitops.hpp"
#include "qz_device.hpp"
#include "qz_internal.hpp"

namespace qz {
namespace {

using bitops::load_words;
using bitops::store_words;
using bitops::store_words_nt;
using bitops::rule_words;
using bitops::tie_words;
using bitops::update_words;

struct SweepArgs {
    const uint32_t *S0, *S1;   // read copy, colour planes 0 and 1
    uint32_t *D0, *D1;         // write copy
    unsigned long long *bond_acc;
    unsigned long long *flip_acc;   // accepted flips of this sweep (COUNT only, nullable)
    uint32_t L, W, R;          // R = W / V lanes per row
    uint32_t Ty, E, Tz, nty;   // E = rows held per tile (Ty + 4, or L for whole planes)
    uint32_t whole;            // 1 when a tile is a whole plane (no y halo)
    uint32_t k0, k1, t;
    uint32_t mixed;            // 1: mixed cycle (first colour drawn per sweep)
};

template <int V, bool COUNT>
__global__ void __launch_bounds__(1024) k_bit_sweep(SweepArgs A)
{
    extern __shared__ uint32_t lds[];
    const uint32_t L = A.L, W = A.W, E = A.E;
    const uint32_t tid = threadIdx.x;
    const uint32_t e = tid / A.R;               // held row
    const uint32_t w0 = (tid % A.R) * V;        // first word of this lane

    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t ty = tile % A.nty, tz = tile / A.nty;
    const uint32_t y0 = ty * A.Ty, z0 = tz * A.Tz;
    const uint32_t Tya = min(A.Ty, L - y0), Tza = min(A.Tz, L - z0);
    const uint32_t Ea = A.whole ? L : Tya + 4;

    const bool held = e < Ea;
    bool c0_row, owned;
    uint32_t y, em, ep;
    if (A.whole) {
        y = e;
        c0_row = held;
        owned = held;
        em = (e == 0) ? L - 1 : e - 1;
        ep = (e + 1 == L) ? 0 : e + 1;
    } else {
        y = (y0 + L - 2 + e) % L;
        c0_row = held && e >= 1 && e + 2 <= Ea;
        owned = held && e >= 2 && e + 3 <= Ea;
        em = e - 1;
        ep = e + 1;
    }
    const uint32_t wprev = (w0 + W - 1) % W, wnext = (w0 + V) % W;
    const size_t row_words = (size_t)W;
    const size_t plane_words = (size_t)L * W;

    uint32_t c1m[V], c1c[V], c1p[V], c0o[V], n0m2[V], n0m1[V], n0c[V], c1n[V];
    uint32_t pf1[V], pf0[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        c1m[v] = c1c[v] = c1p[v] = c0o[v] = n0m2[v] = n0m1[v] = n0c[v] = c1n[v] = 0u;
        pf1[v] = pf0[v] = 0u;
    }
    auto off = [&](uint32_t z) -> size_t { return (size_t)z * plane_words + (size_t)y * row_words + w0; };
    // Colour f is updated first: 0 in the 01 cycle; in the mixed cycle bit 0 of
    // Philox block (0, t, 2, 0) (Supplementary Methods I B: order drawn per sweep).
    // Below, "c0" names the first colour and "c1" the second.
    const uint32_t f = A.mixed ? (philox10(0u, A.t, 2u, 0u, A.k0, A.k1).w[0] & 1u) : 0u;
    const uint32_t *SF = f ? A.S1 : A.S0, *SS = f ? A.S0 : A.S1;
    uint32_t *DF = f ? A.D1 : A.D0, *DS = f ? A.D0 : A.D1;

    if (held) {
        load_words<V>(SS + off((z0 + L - 2) % L), c1m);
        load_words<V>(SS + off((z0 + L - 1) % L), c1c);
        load_words<V>(SS + off(z0 % L), c1p);
    }
    if (c0_row)
        load_words<V>(SF + off((z0 + L - 1) % L), c0o);

    int bonds = 0;       // sum of a over owned colour-0 sites (COUNT only)
    uint32_t flips = 0;  // accepted flips over owned sites (COUNT only)

    // The tie words depend only on the sites and the time, so each step's are
    // drawn one step ahead (unconditionally), off the chain from the first
    // colour's update to the second's.
    auto gword = [&](uint32_t z) -> uint32_t { return (uint32_t)(((size_t)z * L + y) * W + w0); };
    auto draw_step = [&](uint32_t z, uint32_t (&a)[V], uint32_t (&b)[V]) {
        const uint32_t ga = gword(z), gb = gword((z + L - 1) % L);
        tie_words<V>(A.k0, A.k1, ga, ga & 3u, A.t, f, a);
        tie_words<V>(A.k0, A.k1, gb, gb & 3u, A.t, 1u - f, b);
    };
    uint32_t sF[V], sS[V];   // tie words of the next step's two updates
    draw_step((z0 + L - 1) % L, sF, sS);

    for (int qi = -1; qi <= (int)Tza; ++qi) {
        const uint32_t zq = (z0 + L + qi) % L;            // plane of this step
        const uint32_t zm = (zq + L - 1) % L;             // plane of the colour-1 update
        // prefetch the next step's words
        if (qi < (int)Tza) {
            if (held)
                load_words<V>(SS + off((zq + 2) % L), pf1);
            if (c0_row)
                load_words<V>(SF + off((zq + 1) % L), pf0);
        }
        uint32_t *X1 = lds + (size_t)(qi & 1) * 2 * E * W;   // old colour 1 of plane q
        uint32_t *X0 = X1 + (size_t)E * W;                  // new colour 0 of plane q-1
        if (held) {
            store_words<V>(X1 + e * W + w0, c1c);   // aligned: W and w0 are multiples of V
            store_words<V>(X0 + e * W + w0, n0m1);
        }
        __syncthreads();

        uint32_t rF[V], rS[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            rF[v] = sF[v];
            rS[v] = sS[v];
        }
        draw_step((zq + 1) % L, sF, sS);
        const uint32_t pi = (f + y + zq) & 1u;   // x parity of the first colour at (y, zq), second at (y, zm)
        if (c0_row) {
            uint32_t ym[V], yp[V];
            load_words<V>(X1 + em * W + w0, ym);
            load_words<V>(X1 + ep * W + w0, yp);
            const uint32_t adj = X1[e * W + (pi == 0u ? wprev : wnext)];
            const bool mine = owned && qi >= 0 && qi < (int)Tza;
            int a_sum = 0;
            rule_words<V, COUNT>(c0o, c1c, adj, pi, ym, yp, c1m, c1p, rF, n0c, a_sum);
            if (mine) {
                if constexpr (COUNT) {
                    bonds += a_sum;
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        flips = popc_acc(c0o[v] ^ n0c[v], flips);
                }
                store_words_nt<V>(DF + off(zq), n0c);
            }
        }
        if (owned && qi >= 1) {
            uint32_t ym[V], yp[V];
            load_words<V>(X0 + em * W + w0, ym);
            load_words<V>(X0 + ep * W + w0, yp);
            const uint32_t adj = X0[e * W + (pi == 0u ? wprev : wnext)];
            int unused = 0;
            rule_words<V, false>(c1m, n0m1, adj, pi, ym, yp, n0m2, n0c, rS, c1n, unused);
            if constexpr (COUNT) {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    flips = popc_acc(c1m[v] ^ c1n[v], flips);
            }
            store_words_nt<V>(DS + off(zm), c1n);
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            c1m[v] = c1c[v];
            c1c[v] = c1p[v];
            c1p[v] = pf1[v];
            c0o[v] = pf0[v];
            n0m2[v] = n0m1[v];
            n0m1[v] = n0c[v];
        }
    }

    if constexpr (COUNT) {
        __shared__ unsigned long long part[2][16];
        const unsigned long long ws = wave_sum_u64((unsigned long long)bonds);
        const unsigned long long wf = wave_sum_u64((unsigned long long)flips);
        const uint32_t nw = (blockDim.x + 63) / 64;
        if ((tid & 63) == 0) {
            part[0][tid >> 6] = ws;
            part[1][tid >> 6] = wf;
        }
        __syncthreads();
        if (tid == 0) {
            unsigned long long tot = 0, ftot = 0;
            for (uint32_t k = 0; k < nw; ++k) {
                tot += part[0][k];
                ftot += part[1][k];
            }
            if (A.bond_acc != nullptr)
                atomicAdd(A.bond_acc, tot);
            if (A.flip_acc != nullptr)
                atomicAdd(A.flip_acc, ftot);
        }
    }
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
__device__ __forceinline__ uint32_t cube_order_mask(uint32_t w, uint32_t y, uint32_t z,
                                                    uint32_t L, uint32_t sB, uint32_t k0,
                                                    uint32_t k1, uint32_t t)
{
    // bit b of the word lies in cube column (32w + b) >> (sB - 1) along x
    const uint32_t q = sB - 1;
    const uint32_t nb = L >> sB;
    const uint64_t cb0 = (uint64_t)((32u * w) >> q) +
                         (uint64_t)nb * ((uint64_t)(y >> sB) + (uint64_t)nb * (z >> sB));
    const Words4 o = philox10((uint32_t)(cb0 >> 7), t, 4u, 0u, k0, k1);
    const uint32_t sub = (uint32_t)(cb0 >> 5) & 3u;
    const uint32_t word = (sub & 2u) ? ((sub & 1u) ? o.w[3] : o.w[2])
                                     : ((sub & 1u) ? o.w[1] : o.w[0]);
    const uint32_t bits = word >> (uint32_t)(cb0 & 31u);   // bit k: cube cb0 + k
    if (q >= 5)
        return (bits & 1u) ? 0xFFFFFFFFu : 0u;
    uint32_t m = 0u;
#pragma unroll
    for (uint32_t b = 0; b < 32; ++b)
        m |= ((bits >> (b >> q)) & 1u) << b;
    return m;
}

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
__device__ __forceinline__ uint32_t cube_bits_mask(uint32_t bits, uint32_t q)
{
    // bits: bit k = cube (first cube of the word) + k; word bit b lies in cube
    // column offset b >> q
    if (q >= 5)
        return (bits & 1u) ? 0xFFFFFFFFu : 0u;
    uint32_t m = 0u;
#pragma unroll
    for (uint32_t b = 0; b < 32; ++b)
        m |= ((bits >> (b >> q)) & 1u) << b;
    return m;
}

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

// --------------------------------------------------------------------------
// initial state: thread h covers lattice sites i = 64h .. 64h+63 (one row
// segment), i.e. one word of each colour.
// --------------------------------------------------------------------------
__device__ __forceinline__ uint32_t even_bits(uint64_t v)
{
    v &= 0x5555555555555555ull;
    v = (v | (v >> 1)) & 0x3333333333333333ull;
    v = (v | (v >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v >> 4)) & 0x00FF00FF00FF00FFull;
    v = (v | (v >> 8)) & 0x0000FFFF0000FFFFull;
    v = (v | (v >> 16)) & 0x00000000FFFFFFFFull;
    return (uint32_t)v;
}

__global__ void __launch_bounds__(256) k_bit_init(uint32_t L, uint32_t W, uint64_t nh, uint32_t k0,
                                                  uint32_t k1, uint32_t *P0, uint32_t *P1)
{
    const uint64_t h = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (h >= nh)
        return;
    const Words4 r = philox10((uint32_t)(h >> 1), 0u, 0u, 1u, k0, k1);
    const uint32_t q = (uint32_t)(h & 1u) * 2u;
    const uint64_t v = (uint64_t)r.w[q] | ((uint64_t)r.w[q + 1] << 32);
    const uint64_t row = h / W;
    const uint32_t y = (uint32_t)(row % L), z = (uint32_t)(row / L);
    const uint32_t ce = (y + z) & 1u;   // colour of the even-x sites of this row
    uint32_t *Pe = ce ? P1 : P0, *Po = ce ? P0 : P1;
    Pe[h] = even_bits(v);
    Po[h] = even_bits(v >> 1);
}

// --------------------------------------------------------------------------
// per-axis bond counts from the colour-0 sites (every bond has exactly one
// colour-0 end): thread per colour-0 word.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_bit_bonds(uint32_t L, uint32_t W, uint64_t nwords,
                                                   const uint32_t *P0, const uint32_t *P1,
                                                   unsigned long long *acc3, uint32_t total)
{
    unsigned long long bx = 0, by = 0, bz = 0;
    const size_t plane = (size_t)L * W;
    for (uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x; g < nwords;
         g += (uint64_t)gridDim.x * 256) {
        const uint32_t w = (uint32_t)(g % W);
        const uint64_t row = g / W;
        const uint32_t y = (uint32_t)(row % L), z = (uint32_t)(row / L);
        const uint32_t s = P0[g];
        const uint32_t same = P1[g];
        const uint32_t pi = (y + z) & 1u;
        const size_t rb = (size_t)row * W;
        uint32_t shifted;
        if (pi == 0u)
            shifted = funnel(same, P1[rb + (w + W - 1) % W], 31);
        else
            shifted = funnel(P1[rb + (w + 1) % W], same, 1);
        const size_t zb = (size_t)z * plane;
        const uint32_t ym = P1[zb + (size_t)((y + L - 1) % L) * W + w];
        const uint32_t yp = P1[zb + (size_t)((y + 1) % L) * W + w];
        const uint32_t zm = P1[(size_t)((z + L - 1) % L) * plane + (size_t)y * W + w];
        const uint32_t zp = P1[(size_t)((z + 1) % L) * plane + (size_t)y * W + w];
        bx += __builtin_popcount(s ^ same) + __builtin_popcount(s ^ shifted);
        by += __builtin_popcount(s ^ ym) + __builtin_popcount(s ^ yp);
        bz += __builtin_popcount(s ^ zm) + __builtin_popcount(s ^ zp);
    }
    __shared__ unsigned long long part[3][4];
    bx = wave_sum_u64(bx);
    by = wave_sum_u64(by);
    bz = wave_sum_u64(bz);
    if ((threadIdx.x & 63) == 0) {
        part[0][threadIdx.x >> 6] = bx;
        part[1][threadIdx.x >> 6] = by;
        part[2][threadIdx.x >> 6] = bz;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long tot = 0;
        for (int k = 0; k < 4; ++k)
            tot += part[threadIdx.x][k];
        atomicAdd(acc3 + (total ? 0 : threadIdx.x), tot);   // total: all axes into acc3[0]
    }
}

// --------------------------------------------------------------------------
// unpack / pack / window (checkpoint and test copies)
// --------------------------------------------------------------------------
__device__ __forceinline__ int8_t site_of(uint32_t L, uint32_t W, const uint32_t *P0,
                                          const uint32_t *P1, uint32_t x, uint32_t y, uint32_t z)
{
    const uint32_t c = (x + y + z) & 1u;
    const uint32_t word = (c ? P1 : P0)[((size_t)z * L + y) * W + (x >> 6)];
    return ((word >> ((x >> 1) & 31u)) & 1u) ? (int8_t)1 : (int8_t)-1;
}

__global__ void __launch_bounds__(256) k_bit_unpack(uint32_t L, uint32_t W, const uint32_t *P0,
                                                    const uint32_t *P1, uint32_t z0, uint64_t n,
                                                    int8_t *out)
{
    const uint64_t LL = (uint64_t)L * L;
    for (uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x; k < n;
         k += (uint64_t)gridDim.x * 256) {
        const uint32_t x = (uint32_t)(k % L), y = (uint32_t)((k / L) % L);
        const uint32_t z = z0 + (uint32_t)(k / LL);
        out[k] = site_of(L, W, P0, P1, x, y, z);
    }
}

__global__ void __launch_bounds__(256) k_bit_pack(uint32_t L, uint32_t W, uint32_t *P0,
                                                  uint32_t *P1, uint32_t z0, uint64_t nw,
                                                  const int8_t *in, unsigned long long *bad)
{
    // thread per (colour, word) of planes z0 .. z0+nz-1
    const uint64_t LL = (uint64_t)L * L;
    unsigned long long b = 0;
    for (uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x; k < nw;
         k += (uint64_t)gridDim.x * 256) {
        const uint32_t c = (uint32_t)(k & 1u);
        const uint64_t g = k >> 1;                  // word index relative to plane z0
        const uint32_t w = (uint32_t)(g % W);
        const uint64_t row = g / W;
        const uint32_t y = (uint32_t)(row % L), zl = (uint32_t)(row / L);
        const uint32_t pi = (c + y + z0 + zl) & 1u;
        const int8_t *src = in + (uint64_t)zl * LL + (uint64_t)y * L + 64u * w + pi;
        uint32_t word = 0;
        for (int bit = 0; bit < 32; ++bit) {
            const int8_t v = src[2 * bit];
            b += (v != 1 && v != -1);
            word |= (v == 1 ? 1u : 0u) << bit;
        }
        (c ? P1 : P0)[(size_t)z0 * L * W + g] = word;
    }
    __shared__ unsigned long long part[4];
    b = wave_sum_u64(b);
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long tot = part[0] + part[1] + part[2] + part[3];
        if (tot)
            atomicAdd(bad, tot);
    }
}

__global__ void __launch_bounds__(256) k_bit_window(uint32_t L, uint32_t W, const uint32_t *P0,
                                                    const uint32_t *P1, uint32_t ox, uint32_t oy,
                                                    uint32_t oz, uint32_t Wn, uint32_t lz0,
                                                    uint64_t n, int8_t *out)
{
    const uint64_t WW = (uint64_t)Wn * Wn;
    for (uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x; k < n;
         k += (uint64_t)gridDim.x * 256) {
        const uint32_t lx = (uint32_t)(k % Wn), ly = (uint32_t)((k / Wn) % Wn);
        const uint32_t lz = lz0 + (uint32_t)(k / WW);
        out[k] = site_of(L, W, P0, P1, (ox + lx) % L, (oy + ly) % L, (oz + lz) % L);
    }
}

uint32_t grid_cap(uint64_t work, uint32_t cap)
{
    uint64_t g = (work + 255) / 256;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

}  // namespace

// --------------------------------------------------------------------------
// tuning rules
// --------------------------------------------------------------------------
bool bit_tuning_valid(uint32_t L, const BitTuning &t)
{
    if (L < 64 || L % 64)
        return false;
    const uint32_t W = L / 64;
    if (t.V != 1 && t.V != 2 && t.V != 4)
        return false;
    if (W % (uint32_t)t.V)
        return false;
    if (t.Tz < 1 || (uint32_t)t.Tz > L || t.Ty < 1 || (uint32_t)t.Ty > L)
        return false;
    const uint32_t R = W / t.V;
    const uint32_t E = ((uint32_t)t.Ty == L) ? L : (uint32_t)t.Ty + 4;
    const uint32_t threads = ((E * R + 63) / 64) * 64;
    if (threads > 1024)
        return false;
    const size_t lds = (size_t)2 * 2 * E * W * 4;
    return lds <= 60 * 1024;   // stays inside the default dynamic LDS limit with the static part
}

BitTuning bit_tuning_default(uint32_t L)
{
    // Measured on MI355X: whole planes only pay off for L <= 128; above that,
    // tiles of E = 32 held rows (or fewer when a row needs many lanes) and
    // Tz = 8 planes give the most workgroups in flight and the best times
    // from L = 192 to L = 2048.
    const uint32_t W = L / 64;
    BitTuning t;
    t.V = (W % 4 == 0) ? 4 : (W % 2 == 0) ? 2 : 1;
    const uint32_t R = W / t.V;
    BitTuning whole = t;
    whole.Ty = (int)L;
    whole.Tz = (int)std::min<uint32_t>(8, L);
    if (L <= 128 && bit_tuning_valid(L, whole))
        return whole;
    uint32_t E = 8;
    while (E * 2 <= 32 && E * 2 * R <= 256 && E * 2 <= L)
        E *= 2;
    t.Ty = (int)(E - 4);
    t.Tz = (int)std::min<uint32_t>(8, L);
    return t;
}

hipError_t bit_init(hipStream_t st, uint32_t L, uint64_t seed, uint32_t *P0, uint32_t *P1)
{
    const uint32_t W = L / 64;
    const uint64_t nh = (uint64_t)L * L * W;
    hipLaunchKernelGGL(k_bit_init, dim3((uint32_t)((nh + 255) / 256)), dim3(256), 0, st, L, W, nh,
                       (uint32_t)seed, (uint32_t)(seed >> 32), P0, P1);
    return hipGetLastError();
}

hipError_t bit_sweep(hipStream_t st, uint32_t L, uint64_t seed, uint32_t t, const BitTuning &tu,
                     const uint32_t *S0, const uint32_t *S1, uint32_t *D0, uint32_t *D1,
                     unsigned long long *bond_acc, bool mixed, unsigned long long *flip_acc)
{
    if (!bit_tuning_valid(L, tu))
        return hipErrorInvalidValue;
    SweepArgs a;
    a.S0 = S0; a.S1 = S1; a.D0 = D0; a.D1 = D1;
    a.bond_acc = bond_acc;
    a.flip_acc = flip_acc;
    a.L = L;
    a.W = L / 64;
    a.R = a.W / tu.V;
    a.whole = ((uint32_t)tu.Ty == L) ? 1u : 0u;
    a.Ty = (uint32_t)tu.Ty;
    a.E = a.whole ? L : a.Ty + 4;
    a.Tz = (uint32_t)tu.Tz;
    a.nty = (L + a.Ty - 1) / a.Ty;
    const uint32_t ntz = (L + a.Tz - 1) / a.Tz;
    a.k0 = (uint32_t)seed;
    a.k1 = (uint32_t)(seed >> 32);
    a.t = t;
    a.mixed = mixed ? 1u : 0u;
    const uint32_t threads = ((a.E * a.R + 63) / 64) * 64;
    const size_t lds = (size_t)2 * 2 * a.E * a.W * 4;
    const dim3 grid(a.nty * ntz), block(threads);
    const bool count = bond_acc != nullptr || flip_acc != nullptr;
    switch (tu.V * 2 + (count ? 1 : 0)) {
    case 9: hipLaunchKernelGGL((k_bit_sweep<4, true>), grid, block, lds, st, a); break;
    case 8: hipLaunchKernelGGL((k_bit_sweep<4, false>), grid, block, lds, st, a); break;
    case 5: hipLaunchKernelGGL((k_bit_sweep<2, true>), grid, block, lds, st, a); break;
    case 4: hipLaunchKernelGGL((k_bit_sweep<2, false>), grid, block, lds, st, a); break;
    case 3: hipLaunchKernelGGL((k_bit_sweep<1, true>), grid, block, lds, st, a); break;
    default: hipLaunchKernelGGL((k_bit_sweep<1, false>), grid, block, lds, st, a); break;
    }
    return hipGetLastError();
}

hipError_t bit_bonds(hipStream_t st, uint32_t L, const uint32_t *P0, const uint32_t *P1,
                     unsigned long long *acc3)
{
    const uint32_t W = L / 64;
    const uint64_t nw = (uint64_t)L * L * W;
    hipLaunchKernelGGL(k_bit_bonds, dim3(grid_cap(nw, 4096)), dim3(256), 0, st, L, W, nw, P0, P1,
                       acc3, 0u);
    return hipGetLastError();
}

hipError_t bit_bonds_total(hipStream_t st, uint32_t L, const uint32_t *P0, const uint32_t *P1,
                           unsigned long long *acc)
{
    const uint32_t W = L / 64;
    const uint64_t nw = (uint64_t)L * L * W;
    hipLaunchKernelGGL(k_bit_bonds, dim3(grid_cap(nw, 4096)), dim3(256), 0, st, L, W, nw, P0, P1,
                       acc, 1u);
    return hipGetLastError();
}

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

hipError_t bit_unpack(hipStream_t st, uint32_t L, const uint32_t *P0, const uint32_t *P1,
                      uint32_t z0, uint32_t nz, int8_t *out)
{
    const uint64_t n = (uint64_t)L * L * nz;
    hipLaunchKernelGGL(k_bit_unpack, dim3(grid_cap(n, 8192)), dim3(256), 0, st, L, L / 64, P0, P1,
                       z0, n, out);
    return hipGetLastError();
}

hipError_t bit_pack(hipStream_t st, uint32_t L, uint32_t *P0, uint32_t *P1, uint32_t z0,
                    uint32_t nz, const int8_t *in, unsigned long long *bad)
{
    const uint32_t W = L / 64;
    const uint64_t nw = (uint64_t)L * W * nz * 2;
    hipLaunchKernelGGL(k_bit_pack, dim3(grid_cap(nw, 8192)), dim3(256), 0, st, L, W, P0, P1, z0,
                       nw, in, bad);
    return hipGetLastError();
}

hipError_t bit_window(hipStream_t st, uint32_t L, const uint32_t *P0, const uint32_t *P1,
                      uint32_t ox, uint32_t oy, uint32_t oz, uint32_t Wn, uint32_t lz0,
                      uint32_t nz, int8_t *out)
{
    const uint64_t n = (uint64_t)Wn * Wn * nz;
    hipLaunchKernelGGL(k_bit_window, dim3(grid_cap(n, 8192)), dim3(256), 0, st, L, L / 64, P0, P1,
                       ox, oy, oz, Wn, lz0, n, out);
    return hipGetLastError();
}

}  // namespace qz
