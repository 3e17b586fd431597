// qz_bit2.hip -- two sweeps in ONE streaming pass (1-bit layout), and one
// double-checkerboard sweep in the same four-stage pass.
//
// The one-sweep kernel reads every word once and writes it once per sweep, so
// it is bound by HBM.  Here a workgroup carries the lattice through sweeps t
// and t+1 before writing it back: the intermediate state lives only in
// registers and LDS, halving the memory traffic per sweep.  A tile holds E =
// Ty + 8 rows x all of x and streams along z through Tz planes.  At plane step
// q four stages run, each one plane behind the one before:
//   A  sweep t,   colour 0 of plane q    from old colour 1 of planes q-1, q, q+1
//   B  sweep t,   colour 1 of plane q-1  from A's colour 0 of planes q-2, q-1, q
//   C  sweep t+1, colour 0 of plane q-2  from B's colour 1 of planes q-3, q-2, q-1
//   D  sweep t+1, colour 1 of plane q-3  from C's colour 0 of planes q-4, q-3, q-2
// (Methods, "Checkerboard update": each colour reads only the other one);
// "colour 0" here is the colour updated first in sweep t, which the mixed
// cycle draws per sweep (Supplementary Methods I B): colour 1 first runs with
// the planes exchanged, and a sweep t+1 that draws the other first colour
// runs C and D the other way round (MODE 3 below).  The
// y-neighbour rows of every stage's input come from LDS (four row sets per
// step, double-buffered, one barrier per step); each stage loses one row at
// each side, so the tile owns rows [4, E-4) and recomputes the rest, and it
// recomputes three planes at each z end.  Reads copy A, writes copy B, so
// tiles never race.  The results are identical to two one-sweep passes.
//
// MODE 1 and 2 (double checkerboard): one sweep of its 01 cycle
// (Supplementary Methods I A) in the same four stages.  Its four phases -- fine colour 0 then 1 of
// the coarse-colour-0 cubes, then of the coarse-colour-1 cubes -- read and
// write the planes exactly as A, B, C, D do, except that each stage changes
// only the sites of its coarse colour (A, B: 0; C, D: 1) and every stage draws
// the tie bits of sweep t.  In the mixed cycle (Supplementary Methods I B) the
// coarse colour taken first (c) and each cube's fine order are drawn per
// sweep; a cube's two steps (fine colour f, then 1 - f) then fall on the
// stages as A: c-cubes with f = 0; B: all c-cubes; C: c-cubes with f = 1 and
// (1-c)-cubes with f = 0; D: all (1-c)-cubes; the last step, fine colour 0 of
// the (1-c)-cubes with f = 1, is one more in-place phase after the pass.  Each
// update still reads its neighbours in the state the sequential order gives
// them: cubes of one coarse colour never touch, and every stage that updates
// a (1-c)-cube runs after the c-cubes' sites it reads are final.
#include "qz_bitops.hpp"
#include "qz_cube.hpp"
#include "qz_device.hpp"
#include "qz_internal.hpp"

namespace qz {
namespace {

using bitops::load_words;
using bitops::store_words;
using bitops::store_words_nt;
using bitops::rule_words;
using bitops::tie_words;

struct Sweep2Args {
    const uint32_t *S0, *S1;            // read copy, colour planes 0 and 1
    uint32_t *D0, *D1;                  // write copy
    unsigned long long *acc_a, *acc_c;  // bond counts entering sweeps t and t+1
    unsigned long long *flip_a, *flip_c;  // accepted flips in sweeps t and t+1
    uint32_t L, W, R;                   // R = W / V lanes per row
    uint32_t Ty, E, Tz, nty;            // E = Ty + 8 rows held per tile
    uint32_t k0, k1, t;
    uint32_t f;                         // colour updated first in both sweeps
    uint32_t sB;                        // DCB: cube side 2^sB
};

template <int V>
__device__ __forceinline__ void copy_words(uint32_t (&d)[V], const uint32_t (&s)[V])
{
#pragma unroll
    for (int v = 0; v < V; ++v)
        d[v] = s[v];
}

// CA: 1 adds the anti-aligned counts of the owned colour-0 sites of the state
// entering sweep t (stage A), 2 also the spins sweep t flips (stages A and B),
// 0 neither.  CC: the same two counts for sweep t+1 (stages C and D).
// PAIRED (needs 64 % R == 0 and E a multiple of 128 / R): waves come in pairs
// over 2 * (64 / R) consecutive rows, the even wave holding the even rows and
// the odd wave the odd ones.  Every wave's rows then share the parity of y, so
// the x parity pi of all four stages is the same across the wave and the
// x-neighbour shift takes one uniform branch instead of both.
// MODE 0: two sweeps that update the same colour first.  MODE 1, 2: the
// double-checkerboard sweep described above, 01 or mixed cycle (CA then
// counts the entering bonds, and with 2 the flips of the pass; CC is not used).
// MODE 3: two sweeps of the mixed cycle that draw different first colours,
// so the colours go 0, 1 | 1, 0 ("colour 0" being sweep t's first): C updates
// colour 1 of plane q-2 again, from A's colour 0 of planes q-3, q-2, q-1
// (their rows take B's row set, which C no longer reads), and D colour 0 of
// plane q-3 from C's colour 1; C and D draw the tie bits of sweep t+1 with
// their own colours, and their x parity is the opposite of A's and B's.
// The mixed double checkerboard keeps more state per lane (the cube-order
// masks of two stages): its workgroups are limited to 512 lanes, which leaves
// it registers enough not to spill.
template <int V, int CA, bool CC, bool PAIRED, int MODE>
__global__ void __launch_bounds__(MODE == 2 ? 512 : 1024) k_bit_sweep2(Sweep2Args A)
{
    constexpr bool DCB = MODE == 1 || MODE == 2;
    constexpr bool SWAP = MODE == 3;
    extern __shared__ uint32_t lds[];
    const uint32_t L = A.L, W = A.W, E = A.E;
    const uint32_t tid = threadIdx.x;
    uint32_t e;                                  // held row
    if constexpr (PAIRED) {
        const uint32_t rpw = 64u / A.R, wv = tid >> 6, j = (tid & 63u) / A.R;
        e = 2u * rpw * (wv >> 1) + 2u * j + (wv & 1u);
    } else {
        e = tid / A.R;
    }
    const uint32_t w0 = (tid % A.R) * V;        // first word of this lane

    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t ty = tile % A.nty, tz = tile / A.nty;
    const uint32_t y0 = ty * A.Ty, z0 = tz * A.Tz;
    const uint32_t Tya = min(A.Ty, L - y0), Tza = min(A.Tz, L - z0);
    const uint32_t Ea = Tya + 8;

    const bool held = e < Ea;
    const bool rowA = held && e >= 1 && e + 1 < Ea;
    const bool rowB = held && e >= 2 && e + 2 < Ea;
    const bool rowC = held && e >= 3 && e + 3 < Ea;
    const bool rowD = held && e >= 4 && e + 4 < Ea;   // owned rows
    const uint32_t y = (y0 + L - 4 + e) % L;
    const uint32_t em = e - 1, ep = e + 1;
    const uint32_t wprev = (w0 + W - 1) % W, wnext = (w0 + V) % W;
    const size_t plane_words = (size_t)L * W;
    auto off = [&](uint32_t z) -> size_t { return (size_t)z * plane_words + (size_t)y * W + w0; };
    // first word of the lane in the colour-index order that keys the tie bits
    auto gword = [&](uint32_t z) -> uint32_t { return (uint32_t)(((size_t)z * L + y) * W + w0); };

    // register rings, named by plane relative to the step's plane q
    // old colour 1 of planes q-1, q, q+1 and prefetches of q+2, q+3; old colour
    // 0 of plane q and prefetches of q+1, q+2 (two steps of loads in flight)
    uint32_t c1m[V], c1c[V], c1p[V], pf1[V], pg1[V];
    uint32_t c0o[V], pf0[V], pg0[V];
    uint32_t n0a[V], n0b[V], n0n[V];           // colour 0 after sweep t: q-1, q-2; new q
    uint32_t n0c[V];                           // SWAP: colour 0 after sweep t, plane q-3
    uint32_t n1a[V], n1b[V], n1n[V];           // colour 1 after sweep t: q-2, q-3; new q-1
    uint32_t m0a[V], m0b[V], m0n[V];           // colour 0 after sweep t+1: q-3, q-4; new q-2
    uint32_t m1n[V];                           // colour 1 after sweep t+1: new q-3
#pragma unroll
    for (int v = 0; v < V; ++v) {
        c1m[v] = c1c[v] = c1p[v] = pf1[v] = c0o[v] = pf0[v] = pg1[v] = pg0[v] = 0u;
        n0a[v] = n0b[v] = n0n[v] = n0c[v] = n1a[v] = n1b[v] = n1n[v] = 0u;
        m0a[v] = m0b[v] = m0n[v] = m1n[v] = 0u;
    }
    if (held) {
        load_words<V>(A.S1 + off((z0 + L - 4) % L), c1m);
        load_words<V>(A.S1 + off((z0 + L - 3) % L), c1c);
        load_words<V>(A.S1 + off((z0 + L - 2) % L), c1p);
        load_words<V>(A.S1 + off((z0 + L - 1) % L), pf1);
    }
    if (rowA) {
        load_words<V>(A.S0 + off((z0 + L - 3) % L), c0o);
        load_words<V>(A.S0 + off((z0 + L - 2) % L), pf0);
    }

    int bonds_a = 0, bonds_c = 0;
    uint32_t flips_a = 0, flips_c = 0;   // accepted flips over owned sites
    const size_t set = (size_t)E * W;   // words of one row set in LDS

    // The tie words of the four stages depend only on the sites and the time,
    // so they are drawn one plane step ahead: the Philox evaluations then
    // overlap the current step's loads, barrier and stage chain A -> B -> C
    // -> D instead of lengthening it.  They are drawn unconditionally; late
    // in a quench nearly every wave still has a tie in every stage.
    auto draw_step = [&](uint32_t z, uint32_t (&a)[V], uint32_t (&b)[V], uint32_t (&c)[V],
                         uint32_t (&d)[V]) {
        const uint32_t ga = gword(z), gb = gword((z + L - 1) % L);
        const uint32_t gc = gword((z + L - 2) % L), gd = gword((z + L - 3) % L);
        tie_words<V>(A.k0, A.k1, ga, ga & 3u, A.t, A.f, a);
        tie_words<V>(A.k0, A.k1, gb, gb & 3u, A.t, 1u - A.f, b);
        const uint32_t t2 = DCB ? A.t : A.t + 1u;
        tie_words<V>(A.k0, A.k1, gc, gc & 3u, t2, SWAP ? 1u - A.f : A.f, c);
        tie_words<V>(A.k0, A.k1, gd, gd & 3u, t2, SWAP ? A.f : 1u - A.f, d);
    };
    uint32_t sA[V], sB[V], sC[V], sD[V];   // tie words of the next step's stages
    draw_step((z0 + L - 3) % L, sA, sB, sC, sD);

    // DCB: the sites of coarse colour 0 among the lane's words of plane z.  A
    // word's sites lie in cubes (32 w + b) >> q along x (q = sB - 1, since a
    // colour row holds every second site), so below q = 5 the mask is a fixed
    // pattern of runs of 2^q bits, and from q = 5 on all 32 sites share a cube.
    const uint32_t dq = DCB ? A.sB - 1u : 0u;
    const uint32_t dpat = dq == 0 ? 0xAAAAAAAAu : dq == 1 ? 0xCCCCCCCCu : dq == 2 ? 0xF0F0F0F0u
                        : dq == 3 ? 0xFF00FF00u : dq == 4 ? 0xFFFF0000u : 0u;
    auto coarse0 = [&](uint32_t z, uint32_t (&m)[V]) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint32_t par = (((32u * (w0 + (uint32_t)v)) >> dq) + (y >> A.sB) + (z >> A.sB)) & 1u;
            m[v] = par ? dpat : ~dpat;
        }
    };
    // mixed: the coarse colour taken first, and per word the sites whose cube
    // takes fine colour 1 first (stages A and C), kept per layer of cubes
    constexpr bool MIX = MODE == 2;
    const uint32_t cc0 = MIX ? (philox10(0u, A.t, 3u, 0u, A.k0, A.k1).w[0] & 1u) : 0u;
    uint32_t fA[V], fC[V];
    uint32_t kA = 0xFFFFFFFFu, kC = 0xFFFFFFFFu;
#pragma unroll
    for (int v = 0; v < V; ++v)
        fA[v] = fC[v] = 0u;
    auto order = [&](uint32_t z, uint32_t &kz, uint32_t (&fo)[V]) {
        if ((z >> A.sB) != kz) {            // z is the same in every lane
            kz = z >> A.sB;
#pragma unroll
            for (int v = 0; v < V; ++v)
                fo[v] = cube_order_mask(w0 + (uint32_t)v, y, z, L, A.sB, A.k0, A.k1, A.t);
        }
    };
    // keep the stage's old words outside its coarse colour (sel = ~0: all new)
    auto keep = [&](const uint32_t (&own)[V], uint32_t (&out)[V], const uint32_t (&sel)[V]) {
#pragma unroll
        for (int v = 0; v < V; ++v)
            out[v] = (out[v] & sel[v]) | (own[v] & ~sel[v]);
    };

    for (int qi = -3; qi <= (int)Tza + 2; ++qi) {
        const uint32_t zq = (z0 + 2 * L + qi) % L;
        if (qi + 1 < (int)Tza + 2) {
            if (held)
                load_words<V>(A.S1 + off((zq + 3) % L), pg1);
            if (rowA)
                load_words<V>(A.S0 + off((zq + 2) % L), pg0);
        }
        const uint32_t zc = (zq + L - 2) % L, zd = (zq + L - 3) % L;
        // this step's tie words, and the next step's drawn now (on the last
        // step for a plane no stage reaches: harmless)
        uint32_t rA[V], rB[V], rC[V], rD[V];
        copy_words<V>(rA, sA);
        copy_words<V>(rB, sB);
        copy_words<V>(rC, sC);
        copy_words<V>(rD, sD);
        draw_step((zq + 1) % L, sA, sB, sC, sD);
        uint32_t *X1 = lds + (size_t)(qi & 1) * 4 * set;   // old colour 1, plane q
        uint32_t *X0 = X1 + set;                            // A's colour 0, plane q-1
        uint32_t *Y1 = X0 + set;                            // B's colour 1, plane q-2
        uint32_t *Y0 = Y1 + set;                            // C's colour 0, plane q-3
        if (held) {
            store_words<V>(X1 + e * W + w0, c1c);
            store_words<V>(X0 + e * W + w0, n0a);
            store_words<V>(Y1 + e * W + w0, SWAP ? n0b : n1a);
            store_words<V>(Y0 + e * W + w0, m0a);
        }
        __syncthreads();

        // all four stages update sites with the same x parity in this row
        uint32_t pi = (A.f + y + zq) & 1u;
        if constexpr (PAIRED)
            pi = __builtin_amdgcn_readfirstlane(pi);   // the same in every lane of the wave
        const uint32_t wadj = pi == 0u ? wprev : wnext;
        const uint32_t piC = SWAP ? pi ^ 1u : pi;          // stages C and D
        const uint32_t wadjC = piC == 0u ? wprev : wnext;
        // A: sweep t, colour 0, plane q
        if (rowA) {
            uint32_t ym[V], yp[V];
            load_words<V>(X1 + em * W + w0, ym);
            load_words<V>(X1 + ep * W + w0, yp);
            const uint32_t adj = X1[e * W + wadj];
            int a_sum = 0;
            rule_words<V, (CA != 0)>(c0o, c1c, adj, pi, ym, yp, c1m, c1p, rA, n0n, a_sum);
            if constexpr (DCB) {
                uint32_t m[V];
                coarse0(zq, m);
                if constexpr (MIX)
                    order(zq, kA, fA);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    m[v] = cc0 ? ~m[v] : m[v];
                    if constexpr (MIX)
                        m[v] &= ~fA[v];
                }
                keep(c0o, n0n, m);
            }
            if constexpr (CA != 0)
                if (rowD && qi >= 0 && qi < (int)Tza) {
                    bonds_a += a_sum;
                    if constexpr (CA == 2) {
#pragma unroll
                        for (int v = 0; v < V; ++v)
                            flips_a = popc_acc(c0o[v] ^ n0n[v], flips_a);
                    }
                }
        }
        // B: sweep t, colour 1, plane q-1
        if (rowB && qi >= -1) {
            uint32_t ym[V], yp[V];
            load_words<V>(X0 + em * W + w0, ym);
            load_words<V>(X0 + ep * W + w0, yp);
            const uint32_t adj = X0[e * W + wadj];
            int unused = 0;
            rule_words<V, false>(c1m, n0a, adj, pi, ym, yp, n0b, n0n, rB, n1n, unused);
            if constexpr (DCB) {
                uint32_t m[V];
                coarse0((zq + L - 1) % L, m);
#pragma unroll
                for (int v = 0; v < V; ++v)
                    m[v] = cc0 ? ~m[v] : m[v];
                keep(c1m, n1n, m);
            }
            if constexpr (CA == 2)
                if (rowD && qi >= 1 && qi <= (int)Tza) {
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        flips_a = popc_acc(c1m[v] ^ n1n[v], flips_a);
                }
        }
        // C: sweep t+1, colour 0, plane q-2
        if (rowC && qi >= 1) {
            uint32_t ym[V], yp[V];
            load_words<V>(Y1 + em * W + w0, ym);
            load_words<V>(Y1 + ep * W + w0, yp);
            const uint32_t adj = Y1[e * W + wadjC];
            int a_sum = 0;
            if constexpr (SWAP)
                rule_words<V, CC>(n1a, n0b, adj, piC, ym, yp, n0c, n0a, rC, m0n, a_sum);
            else
                rule_words<V, CC>(n0b, n1a, adj, pi, ym, yp, n1b, n1n, rC, m0n, a_sum);
            if constexpr (DCB) {
                uint32_t m[V];
                coarse0(zc, m);
                if constexpr (MIX)
                    order(zc, kC, fC);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const uint32_t first = cc0 ? ~m[v] : m[v];     // sites of the first coarse colour
                    // mixed: first-colour cubes with f = 1, the others with f = 0
                    m[v] = MIX ? ~(first ^ fC[v]) : ~first;
                }
                keep(n0b, m0n, m);
            }
            if (rowD && qi >= 2 && qi < (int)Tza + 2) {
                if constexpr (DCB && CA == 2) {
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        flips_a = popc_acc(n0b[v] ^ m0n[v], flips_a);
                }
                if constexpr (CC) {
                    bonds_c += a_sum;
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        flips_c = popc_acc((SWAP ? n1a[v] : n0b[v]) ^ m0n[v], flips_c);
                }
                store_words_nt<V>(A.D0 + off(zc), m0n);
            }
        }
        // D: sweep t+1, colour 1, plane q-3
        if (rowD && qi >= 3) {
            uint32_t ym[V], yp[V];
            load_words<V>(Y0 + em * W + w0, ym);
            load_words<V>(Y0 + ep * W + w0, yp);
            const uint32_t adj = Y0[e * W + wadjC];
            int unused = 0;
            if constexpr (SWAP)
                rule_words<V, false>(n0c, m0a, adj, piC, ym, yp, m0b, m0n, rD, m1n, unused);
            else
                rule_words<V, false>(n1b, m0a, adj, pi, ym, yp, m0b, m0n, rD, m1n, unused);
            if constexpr (DCB) {
                uint32_t m[V];
                coarse0(zd, m);
#pragma unroll
                for (int v = 0; v < V; ++v)
                    m[v] = cc0 ? m[v] : ~m[v];                     // the second coarse colour
                keep(n1b, m1n, m);
                if constexpr (CA == 2) {
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        flips_a = popc_acc(n1b[v] ^ m1n[v], flips_a);
                }
            }
            if constexpr (CC) {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    flips_c = popc_acc((SWAP ? n0c[v] : n1b[v]) ^ m1n[v], flips_c);
            }
            store_words_nt<V>(A.D1 + off(zd), m1n);
        }
        // advance the rings by one plane
        copy_words<V>(c1m, c1c);
        copy_words<V>(c1c, c1p);
        copy_words<V>(c1p, pf1);
        copy_words<V>(c0o, pf0);
        copy_words<V>(pf1, pg1);
        copy_words<V>(pf0, pg0);
        if constexpr (SWAP)
            copy_words<V>(n0c, n0b);
        copy_words<V>(n0b, n0a);
        copy_words<V>(n0a, n0n);
        copy_words<V>(n1b, n1a);
        copy_words<V>(n1a, n1n);
        copy_words<V>(m0b, m0a);
        copy_words<V>(m0a, m0n);
    }

    if constexpr (CA != 0 || CC) {
        // the row sets are no longer needed: reuse the start of LDS for the
        // per-wave partial sums (at most 16 waves x 4 counters)
        __syncthreads();
        unsigned long long(*part)[16] = reinterpret_cast<unsigned long long(*)[16]>(lds);
        const unsigned long long wa = wave_sum_u64((unsigned long long)bonds_a);
        const unsigned long long wc = wave_sum_u64((unsigned long long)bonds_c);
        const unsigned long long fa = wave_sum_u64((unsigned long long)flips_a);
        const unsigned long long fc = wave_sum_u64((unsigned long long)flips_c);
        const uint32_t nw = (blockDim.x + 63) / 64;
        if ((tid & 63) == 0) {
            part[0][tid >> 6] = wa;
            part[1][tid >> 6] = wc;
            part[2][tid >> 6] = fa;
            part[3][tid >> 6] = fc;
        }
        __syncthreads();
        if (tid == 0) {
            unsigned long long tot[4] = {0, 0, 0, 0};
            for (uint32_t k = 0; k < nw; ++k)
                for (int c = 0; c < 4; ++c)
                    tot[c] += part[c][k];
            if (CA != 0 && A.acc_a != nullptr)
                atomicAdd(A.acc_a, tot[0]);
            if (CC && A.acc_c != nullptr)
                atomicAdd(A.acc_c, tot[1]);
            if (CA == 2 && A.flip_a != nullptr)
                atomicAdd(A.flip_a, tot[2]);
            if (CC && A.flip_c != nullptr)
                atomicAdd(A.flip_c, tot[3]);
        }
    }
}

template <int V, bool P, int MODE, int CA, bool CC>
void launch2_as(hipStream_t st, const Sweep2Args &a, dim3 grid, dim3 block, size_t lds)
{
    hipLaunchKernelGGL((k_bit_sweep2<V, CA, CC, P, MODE>), grid, block, lds, st, a);
}

// CA: 0 = sweep t not counted, 1 = its entering bond count only, 2 = also its
// flips (the flips of stages A and B cost more than the bond count, so they
// are compiled in only when asked for); CC: sweep t+1's count and flips.
template <int V, bool P, int MODE = 0>
void launch2(hipStream_t st, const Sweep2Args &a, dim3 grid, dim3 block, size_t lds)
{
    const int ca = a.flip_a != nullptr ? 2 : (a.acc_a != nullptr ? 1 : 0);
    const bool cc = a.acc_c != nullptr || a.flip_c != nullptr;
    if constexpr (MODE == 1 || MODE == 2) {
        if (ca == 2)
            launch2_as<V, P, MODE, 2, false>(st, a, grid, block, lds);
        else if (ca == 1)
            launch2_as<V, P, MODE, 1, false>(st, a, grid, block, lds);
        else
            launch2_as<V, P, MODE, 0, false>(st, a, grid, block, lds);
    } else if (cc) {
        if (ca == 2)
            launch2_as<V, P, MODE, 2, true>(st, a, grid, block, lds);
        else if (ca == 1)
            launch2_as<V, P, MODE, 1, true>(st, a, grid, block, lds);
        else
            launch2_as<V, P, MODE, 0, true>(st, a, grid, block, lds);
    } else {
        // the first sweep's count alone runs the kernel that also counts the
        // second one, whose sums are then dropped (both pointers are null):
        // compiled that way the pass measured about 8 % faster on MI355X
        // (0.61 against 0.67 ms at L = 2048; 0.54 ms uncounted)
        if (ca == 2)
            launch2_as<V, P, MODE, 2, false>(st, a, grid, block, lds);
        else if (ca == 1)
            launch2_as<V, P, MODE, 1, true>(st, a, grid, block, lds);
        else
            launch2_as<V, P, MODE, 0, false>(st, a, grid, block, lds);
    }
}

}  // namespace

bool bit_tuning2_valid(uint32_t L, const BitTuning &t)
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
    const uint32_t E = (uint32_t)t.Ty + 8;
    const uint32_t threads = ((E * R + 63) / 64) * 64;
    if (threads > 1024)
        return false;
    const size_t lds = (size_t)2 * 4 * E * W * 4;
    return lds <= 64 * 1024 && lds >= 4 * 16 * 8;
}

BitTuning bit_tuning2_default(uint32_t L)
{
    const uint32_t W = L / 64;
    BitTuning t;
    t.V = (W % 4 == 0) ? 4 : (W % 2 == 0) ? 2 : 1;
    // Measured on MI355X at late times (microseconds per sweep, best tile
    // against the next best and the one-sweep pass): the best tile depends on
    // how the workgroups of a launch fill the chip, so the sizes that were
    // timed take their best.
    //   L = 1024  Ty 24, Tz 24:  50.3 (Ty 56, Tz 16: 50.7; one sweep 58.5)
    //   L = 1280  Ty 56, Tz 64: 100.1 (Ty 56, Tz 24: 107.9; one sweep 108.9)
    //   L = 1536  Ty 24, Tz 48: 147.3 (Ty 24, Tz 32: 149.6; one sweep 176.8)
    //   L = 1792  Ty 56, Tz 48: 212.3 (Ty 56, Tz 64: 220.1; one sweep 282.6)
    //   L = 2048  Ty 56, Tz 64: 270.5 (Ty 56, Tz 48: 280.0; one sweep 397.9)
    struct Timed {
        uint32_t L;
        int Ty, Tz;
    };
    static const Timed timed[] = {
        {1024, 24, 24}, {1280, 56, 64}, {1536, 24, 48}, {1792, 56, 48}, {2048, 56, 64}};
    for (const Timed &m : timed)
        if (m.L == L && t.V == 4) {
            t.Ty = m.Ty;
            t.Tz = m.Tz;
            return t;
        }
    // Elsewhere: where the lattice is far larger than the caches (L >= 1536)
    // tiles of E = 64 held rows (56 owned) and Tz = 64 planes; below that
    // E = 32 and Tz = 8, which keep more workgroups in flight.
    const uint32_t R = W / t.V;
    const bool big = L >= 1536;
    const uint32_t Emax = big ? 64 : 32, Rmax = big ? 1024 : 256;
    uint32_t E = 16;
    while (E * 2 <= Emax && E * 2 * R <= Rmax && (size_t)2 * 4 * (E * 2) * W * 4 <= 64 * 1024)
        E *= 2;
    t.Ty = (int)std::min<uint32_t>(E - 8, L);
    t.Tz = (int)std::min<uint32_t>(big ? 64 : 8, L);
    return t;
}

// Sweeps per pass chosen by default for a bit lattice of side L: two where the
// one-sweep kernel is bound by HBM bandwidth (two copies of the lattice well
// beyond the last-level cache; from L = 1024, where the two-sweep pass was
// measured faster), one otherwise (L = 768: 30.1 us per sweep with one sweep
// per pass, 30.8 at best with two).
int bit_pass_default(uint32_t L) { return L >= 1024 ? 2 : 1; }

namespace {

// the launch geometry and arguments shared by both entry points
template <int MODE>
hipError_t sweep2_launch(hipStream_t st, uint32_t L, uint64_t seed, uint32_t t,
                         const BitTuning &tu, Sweep2Args &a)
{
    a.L = L;
    a.W = L / 64;
    a.R = a.W / tu.V;
    a.Ty = (uint32_t)tu.Ty;
    a.E = a.Ty + 8;
    a.Tz = (uint32_t)tu.Tz;
    a.nty = (L + a.Ty - 1) / a.Ty;
    const uint32_t ntz = (L + a.Tz - 1) / a.Tz;
    a.k0 = (uint32_t)seed;
    a.k1 = (uint32_t)(seed >> 32);
    a.t = t;
    const uint32_t threads = ((a.E * a.R + 63) / 64) * 64;
    const size_t lds = (size_t)2 * 4 * a.E * a.W * 4;
    const dim3 grid(a.nty * ntz), block(threads);
    // paired row mapping (wave-uniform x parity) where the tile shape allows it
    const bool paired = tu.V == 4 && 64 % a.R == 0 && a.E % (128 / a.R) == 0;
    switch (tu.V) {
    case 4:
        if (paired)
            launch2<4, true, MODE>(st, a, grid, block, lds);
        else
            launch2<4, false, MODE>(st, a, grid, block, lds);
        break;
    case 2: launch2<2, false, MODE>(st, a, grid, block, lds); break;
    default: launch2<1, false, MODE>(st, a, grid, block, lds); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t bit_sweep2(hipStream_t st, uint32_t L, uint64_t seed, uint32_t t, const BitTuning &tu,
                      const uint32_t *S0, const uint32_t *S1, uint32_t *D0, uint32_t *D1,
                      unsigned long long *acc_a, unsigned long long *acc_c,
                      unsigned long long *flip_a, unsigned long long *flip_c, uint32_t first,
                      bool swap)
{
    if (!bit_tuning2_valid(L, tu) || first > 1u)
        return hipErrorInvalidValue;
    Sweep2Args a;
    // the kernel's stages A and C update "colour 0", B and D "colour 1": here
    // the colour updated first, and the other (swap: C and D the other way
    // round; C writes through D0 and D the other plane)
    a.S0 = first ? S1 : S0;
    a.S1 = first ? S0 : S1;
    a.D0 = (first ^ (swap ? 1u : 0u)) ? D1 : D0;
    a.D1 = (first ^ (swap ? 1u : 0u)) ? D0 : D1;
    a.f = first;
    a.sB = 0;
    a.acc_a = acc_a;
    a.acc_c = acc_c;
    a.flip_a = flip_a;
    a.flip_c = flip_c;
    return swap ? sweep2_launch<3>(st, L, seed, t, tu, a) : sweep2_launch<0>(st, L, seed, t, tu, a);
}

namespace {

// The tile a double-checkerboard pass runs with.  The mixed cycle's kernel
// holds about 150 registers per lane: rows cut so that a workgroup has about
// 256 lanes let three of them share a CU (at L = 2048, Ty = 24 instead of 56:
// 1.22 against 1.35 ms per sweep on MI355X); the 01 cycle is fastest with the
// lattice's own tile.
BitTuning dcb2_tile(uint32_t L, const BitTuning &tu, bool mixed)
{
    BitTuning tm = tu;
    if (mixed && tu.V >= 1) {
        const int R = (int)((L / 64) / (uint32_t)tu.V);
        if (R > 0)
            tm.Ty = std::max(8, std::min(tu.Ty, 256 / R - 8));
    }
    return tm;
}

}  // namespace

bool bit_double_sweep2_fits(uint32_t L, const BitTuning &tu, bool mixed)
{
    const BitTuning tm = dcb2_tile(L, tu, mixed);
    if (!bit_tuning2_valid(L, tm))
        return false;
    const uint32_t R = (L / 64) / (uint32_t)tm.V, E = (uint32_t)tm.Ty + 8;
    return !mixed || ((E * R + 63) / 64) * 64 <= 512;
}

hipError_t bit_double_sweep2(hipStream_t st, uint32_t L, uint32_t B, uint64_t seed, uint32_t t,
                             const BitTuning &tu, const uint32_t *S0, const uint32_t *S1,
                             uint32_t *D0, uint32_t *D1, bool mixed,
                             unsigned long long *bond_acc, unsigned long long *flip_acc)
{
    uint32_t sB = 0;
    while ((1u << sB) < B)
        ++sB;
    const BitTuning tm = dcb2_tile(L, tu, mixed);
    if (!bit_double_sweep2_fits(L, tu, mixed) || B < 2 || (1u << sB) != B || L % (2 * B))
        return hipErrorInvalidValue;
    Sweep2Args a;
    a.S0 = S0;
    a.S1 = S1;
    a.D0 = D0;
    a.D1 = D1;
    a.f = 0;
    a.sB = sB;
    a.acc_a = bond_acc;
    a.acc_c = nullptr;
    a.flip_a = flip_acc;
    a.flip_c = nullptr;
    return mixed ? sweep2_launch<2>(st, L, seed, t, tm, a) : sweep2_launch<1>(st, L, seed, t, tu, a);
}

}  // namespace qz
