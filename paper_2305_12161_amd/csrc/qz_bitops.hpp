// qz_bitops.hpp -- word-level pieces of the 1-bit colour-separated sweeps,
// shared by the one-sweep and the two-sweep streaming kernels: vector loads
// and stores of V consecutive words, and the update of V words of one colour
// by the T = 0 rule (Methods, equ:glauberAcceptance) through the up-neighbour
// count.  gfx950 only.
#pragma once
#include "qz_device.hpp"

namespace qz {
namespace bitops {

// --------------------------------------------------------------------------
// vector load/store of V consecutive words
// --------------------------------------------------------------------------
template <int V> struct VecT;
template <> struct VecT<1> { using T = uint32_t; };
template <> struct VecT<2> { using T = uint2; };
template <> struct VecT<4> { using T = uint4; };

template <int V>
__device__ __forceinline__ void load_words(const uint32_t *p, uint32_t (&r)[V])
{
    if constexpr (V == 4) {
        const uint4 v = *reinterpret_cast<const uint4 *>(p);
        r[0] = v.x; r[1] = v.y; r[2] = v.z; r[3] = v.w;
    } else if constexpr (V == 2) {
        const uint2 v = *reinterpret_cast<const uint2 *>(p);
        r[0] = v.x; r[1] = v.y;
    } else {
        r[0] = *p;
    }
}

template <int V>
__device__ __forceinline__ void store_words(uint32_t *p, const uint32_t (&r)[V])
{
    if constexpr (V == 4) {
        *reinterpret_cast<uint4 *>(p) = make_uint4(r[0], r[1], r[2], r[3]);
    } else if constexpr (V == 2) {
        *reinterpret_cast<uint2 *>(p) = make_uint2(r[0], r[1]);
    } else {
        *p = r[0];
    }
}

// Store to HBM with the nontemporal hint: the written copy is not read again
// in this sweep, so it should not displace the read copy's rows from cache.
template <int V>
__device__ __forceinline__ void store_words_nt(uint32_t *p, const uint32_t (&r)[V])
{
#pragma unroll
    for (int v = 0; v < V; ++v)
        __builtin_nontemporal_store(r[v], p + v);
}

// The x-neighbour word on the side given by pi: pi = 0 takes site k-1 (bits
// move up by one, bit 0 from the word below), pi = 1 takes site k+1 (bits move
// down by one, bit 31 from the word above); adj is the word beyond the lane's V.
template <int V>
__device__ __forceinline__ uint32_t shifted_word(const uint32_t (&same)[V], uint32_t adj,
                                                 uint32_t pi, int v)
{
    if (pi == 0u) {
        const uint32_t lo = (v > 0) ? same[v > 0 ? v - 1 : 0] : adj;
        return funnel(same[v], lo, 31);
    }
    const uint32_t hi = (v < V - 1) ? same[v < V - 1 ? v + 1 : 0] : adj;
    return funnel(hi, same[v], 1);
}

// The tie words of this lane: word (sub + v) of Philox block ctr0 / 4 of
// (t, p), chosen without a dynamically indexed array (which would live in
// scratch memory).  With V = 4 the lane's words start a block (sub = 0); with
// V = 2, sub is 0 or 2.
template <int V>
__device__ __forceinline__ void tie_words(uint32_t k0, uint32_t k1, uint32_t ctr0, uint32_t sub,
                                          uint32_t t, uint32_t p, uint32_t (&r)[V])
{
    const Words4 rb = philox10(ctr0 >> 2, t, p, 0u, k0, k1);
    if constexpr (V == 4) {
#pragma unroll
        for (int v = 0; v < V; ++v)
            r[v] = rb.w[v];
    } else if constexpr (V == 2) {
        const bool hi = (sub & 2u) != 0u;
        r[0] = hi ? rb.w[2] : rb.w[0];
        r[1] = hi ? rb.w[3] : rb.w[1];
    } else {
        const uint32_t lo = (sub & 1u) ? rb.w[1] : rb.w[0];
        const uint32_t hi = (sub & 1u) ? rb.w[3] : rb.w[2];
        r[0] = (sub & 2u) ? hi : lo;
    }
}

// Update V words of one colour.  own = the words being updated; same = the
// other colour's same-row words (x-neighbour at the same index); adj = the
// word just outside the lane's range on the side given by pi; ym/yp/zm/zp the
// other colour's rows y-1, y+1 and planes z-1, z+1.
//
// Without counting, the rule runs as a majority of seven: with U the number
// of up neighbours and w = s ^ r, the new spin is up iff U + w >= 4 (U >= 4
// always up, U == 3 takes w, U <= 2 always down).  Split the neighbours into
// two triples with parities xa, xb and majorities ma, mb (U = xa + xb +
// 2(ma + mb)); then U + w >= 4 iff maj(ma, mb, maj(xa, xb, w)), and U == 3
// iff (xa ^ xb) & (ma ^ mb), which decides whether the lane needs its tie
// bits.  COUNT: the full three-bit count U instead, for the sum of a over the
// sites (added to acc).
template <int V, bool COUNT>
__device__ __forceinline__ void update_words(const uint32_t (&own)[V], const uint32_t (&same)[V],
                                             uint32_t adj, uint32_t pi, const uint32_t (&ym)[V],
                                             const uint32_t (&yp)[V], const uint32_t (&zm)[V],
                                             const uint32_t (&zp)[V], uint32_t k0, uint32_t k1,
                                             uint32_t ctr0, uint32_t sub, uint32_t t, uint32_t p,
                                             uint32_t (&out)[V], int &acc)
{
    uint32_t r[V];
#pragma unroll
    for (int v = 0; v < V; ++v)
        r[v] = 0u;
    if constexpr (COUNT) {
        UpCount c[V];
        uint32_t ties = 0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            c[v] = count_up(same[v], shifted_word<V>(same, adj, pi, v), ym[v], yp[v], zm[v], zp[v]);
            ties |= up_tie(c[v]);
        }
        if (ties != 0u)
            tie_words<V>(k0, k1, ctr0, sub, t, p, r);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            out[v] = up_rule(own[v], c[v], r[v]);
            acc += up_antialigned_sum(own[v], c[v]);
        }
    } else {
        uint32_t xa[V], ma[V], xb[V], mb[V];
        uint32_t ties = 0;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint32_t sh = shifted_word<V>(same, adj, pi, v);
            xa[v] = xor3(same[v], sh, ym[v]);
            ma[v] = maj3(same[v], sh, ym[v]);
            xb[v] = xor3(yp[v], zm[v], zp[v]);
            mb[v] = maj3(yp[v], zm[v], zp[v]);
            ties |= (xa[v] ^ xb[v]) & (ma[v] ^ mb[v]);
        }
        // w = own ^ r, formed only where some lane has a tie
        uint32_t w[V];
#pragma unroll
        for (int v = 0; v < V; ++v)
            w[v] = own[v];
        if (ties != 0u) {
            tie_words<V>(k0, k1, ctr0, sub, t, p, r);
#pragma unroll
            for (int v = 0; v < V; ++v)
                w[v] ^= r[v];
        }
#pragma unroll
        for (int v = 0; v < V; ++v)
            out[v] = maj3(ma[v], mb[v], maj3(xa[v], xb[v], w[v]));
        (void)acc;
    }
}

// The same rule with the tie words r already drawn: the new words with no
// branch on whether any lane ties.  The streaming kernels draw the tie words
// of their stages ahead, so that the Philox evaluations do not sit on the
// chain from one stage's result to the next.
//
// COUNT adds the sum of a over the sites, from the same two triples: with s
// the own spin, a = (xa ^ s) + (xb ^ s) + 2 ((ma ^ s) + (mb ^ s)) per site
// (a triple's parity and majority differ from s in exactly the ways that its
// anti-aligned count 0..3 requires), so four popcounts per word.
template <int V, bool COUNT>
__device__ __forceinline__ void rule_words(const uint32_t (&own)[V], const uint32_t (&same)[V],
                                           uint32_t adj, uint32_t pi, const uint32_t (&ym)[V],
                                           const uint32_t (&yp)[V], const uint32_t (&zm)[V],
                                           const uint32_t (&zp)[V], const uint32_t (&r)[V],
                                           uint32_t (&out)[V], int &acc)
{
    uint32_t ones = 0, twos = 0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const uint32_t sh = shifted_word<V>(same, adj, pi, v);
        const uint32_t xa = xor3(same[v], sh, ym[v]), ma = maj3(same[v], sh, ym[v]);
        const uint32_t xb = xor3(yp[v], zm[v], zp[v]), mb = maj3(yp[v], zm[v], zp[v]);
        out[v] = maj3(ma, mb, maj3(xa, xb, own[v] ^ r[v]));
        if constexpr (COUNT) {
            ones = popc_acc(xa ^ own[v], popc_acc(xb ^ own[v], ones));
            twos = popc_acc(ma ^ own[v], popc_acc(mb ^ own[v], twos));
        }
    }
    if constexpr (COUNT)
        acc += (int)(ones + 2u * twos);
    (void)acc;
}

}  // namespace bitops
}  // namespace qz
