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
