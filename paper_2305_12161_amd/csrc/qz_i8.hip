// qz_i8.hip -- kernels for the int8 layout: one signed byte (+1 / -1) per site,
// lattice index i = x + L*(y + L*z).  One launch per colour (the colour-p pass
// reads only colour 1-p, so it updates in place without races), the bond count
// of the state entering a sweep fused into its colour-0 pass.
#include <algorithm>

#include "qz_device.hpp"
#include "qz_internal.hpp"

namespace qz {
namespace {

constexpr int kThreads = 256;

// Sum a per-thread 64-bit value over the block and add it to *acc (one atomic).
__device__ __forceinline__ void block_add_u64(unsigned long long v, unsigned long long *acc)
{
    __shared__ unsigned long long part[kThreads / 64];
    __syncthreads();   // a previous call may still be reading part[]
    v = wave_sum_u64(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        part[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int k = 0; k < kThreads / 64; ++k)
            tot += part[k];
        if (tot)
            atomicAdd(acc, tot);
    }
}

__device__ __forceinline__ uint32_t wrap_up(uint32_t v, uint32_t L) { return v + 1 == L ? 0 : v + 1; }
__device__ __forceinline__ uint32_t wrap_dn(uint32_t v, uint32_t L) { return v == 0 ? L - 1 : v - 1; }

// Infinite-temperature start: thread b draws Philox block (b, 0, 0, 1) and
// writes the 128 sites i = 128b .. 128b+127 (+1 where the bit is set).
__global__ void __launch_bounds__(kThreads) k_i8_init(uint64_t N, uint32_t k0, uint32_t k1,
                                                      int8_t *s)
{
    const uint64_t b = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    const uint64_t base = b * 128;
    if (base >= N)
        return;
    const Words4 r = philox10((uint32_t)b, 0u, 0u, 1u, k0, k1);
    uint32_t *out = reinterpret_cast<uint32_t *>(s + base);
#pragma unroll
    for (int q = 0; q < 32; ++q) {          // 4 sites per 32-bit store; N % 8 == 0
        if (base + 4 * q >= N)
            break;
        const uint32_t bits = (r.w[q >> 3] >> ((q & 7) * 4)) & 0xFu;
        uint32_t v = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            v |= (((bits >> k) & 1u) ? 0x01u : 0xFFu) << (8 * k);
        out[q] = v;
    }
}

// The colour updated by half-sweep `which` (0 = first, 1 = second) of sweep
// t: p = which in the 01 cycle; in the mixed cycle the first colour is bit 0
// of Philox block (0, t, 2, 0) (Supplementary Methods I B: order drawn per
// sweep).
__device__ __forceinline__ uint32_t half_colour(uint32_t which, uint32_t mixed, uint32_t t,
                                                uint32_t k0, uint32_t k1)
{
    const uint32_t first = mixed ? (philox10(0u, t, 2u, 0u, k0, k1).w[0] & 1u) : 0u;
    return which ^ first;
}

// Half-sweep of any even L: thread per colour site of one plane (blockIdx.y =
// z), consecutive lanes at consecutive colour indices j, so a wave shares one
// Philox block and evaluates it once.
__global__ void __launch_bounds__(kThreads)
    k_i8_half(uint32_t L, uint32_t k0, uint32_t k1, uint32_t t, uint32_t which, uint32_t mixed,
              int8_t *s, unsigned long long *bond_acc, unsigned long long *flip_acc)
{
    const uint32_t p = half_colour(which, mixed, t, k0, k1);
    const uint32_t H = L >> 1, z = blockIdx.y;
    const uint32_t q = blockIdx.x * kThreads + threadIdx.x;   // colour site within the plane
    unsigned long long acc = 0, flips = 0;
    if (q < L * H) {
        const uint32_t xh = q % H, y = q / H;
        const uint32_t x = 2 * xh + ((p + y + z) & 1u);
        const uint64_t LL = (uint64_t)L * L;
        const uint64_t zo = (uint64_t)z * LL, yo = (uint64_t)y * L;
        const uint64_t i = zo + yo + x;
        const uint64_t j = (uint64_t)z * L * H + q;
        const int8_t me = s[i];
        uint32_t a = 0;
        a += s[zo + yo + wrap_up(x, L)] != me;
        a += s[zo + yo + wrap_dn(x, L)] != me;
        a += s[zo + (uint64_t)wrap_up(y, L) * L + x] != me;
        a += s[zo + (uint64_t)wrap_dn(y, L) * L + x] != me;
        a += s[(uint64_t)wrap_up(z, L) * LL + yo + x] != me;
        a += s[(uint64_t)wrap_dn(z, L) * LL + yo + x] != me;
        acc = a;
        bool flip = a >= 4;
        if (a == 3) {
            const Words4 r = philox10((uint32_t)(j >> 7), t, p, 0u, k0, k1);
            flip = (r.w[(j >> 5) & 3] >> (j & 31)) & 1u;
        }
        if (flip) {
            s[i] = (int8_t)-me;
            flips = 1;
        }
    }
    if (bond_acc != nullptr)
        block_add_u64(acc, bond_acc);
    if (flip_acc != nullptr)
        block_add_u64(flips, flip_acc);
}

// Sum of the four bytes of v (each at most 63).
__device__ __forceinline__ uint32_t byte_sum(uint32_t v) { return (v * 0x01010101u) >> 24; }

// One 16-byte chunk along x (sites x0 .. x0+15 of row (y, z), L % 16 == 0)
// of a colour-p half-sweep, in place.  A site's spin becomes a bit per byte
// (1 where it is -1); its six neighbour bits come from 16-byte loads of the
// rows y +- 1 and planes z +- 1, and for x from the chunk itself shifted by
// one byte, with one byte loaded at each end.  The anti-aligned count a
// (0..6) is then a bytewise sum of six XORs, four sites per 32-bit word; a >=
// 4 flips, a == 3 flips on the site's tie bit.  The chunk's 8 sites of colour
// p have consecutive colour indices j0 .. j0 + 7, i.e. one byte of one Philox
// output word.  The lattice is reached through `ld16(offset)`, `ld1(offset)`
// and `st16(offset, value)`, so that the same update runs on global memory and
// on a lattice held in LDS.  Adds the chunk's anti-aligned counts over the
// colour-p sites to asum and its flips to fsum.
template <class Off, class LD16, class LD1, class ST16>
__device__ __forceinline__ void i8_chunk(uint32_t L, uint32_t p, uint32_t y, uint32_t z,
                                         uint32_t x0, uint32_t t, uint32_t k0, uint32_t k1,
                                         LD16 ld16, LD1 ld1, ST16 st16, uint32_t &asum,
                                         uint32_t &fsum)
{
    const Off LL = (Off)L * L;
    const Off rb = (Off)z * LL + (Off)y * L;
    const uint4 vme = ld16(rb + x0);
    const uint4 vym = ld16((Off)z * LL + (Off)wrap_dn(y, L) * L + x0);
    const uint4 vyp = ld16((Off)z * LL + (Off)wrap_up(y, L) * L + x0);
    const uint4 vzm = ld16((Off)wrap_dn(z, L) * LL + (Off)y * L + x0);
    const uint4 vzp = ld16((Off)wrap_up(z, L) * LL + (Off)y * L + x0);
    const uint32_t lbit = ((uint32_t)(uint8_t)ld1(rb + (x0 == 0 ? L - 1 : x0 - 1)) >> 7) & 1u;
    const uint32_t rbit = ((uint32_t)(uint8_t)ld1(rb + (x0 + 16 == L ? 0 : x0 + 16)) >> 7) & 1u;
    constexpr uint32_t kOnes = 0x01010101u;
    const uint32_t me[4] = {vme.x, vme.y, vme.z, vme.w};
    const uint32_t ym[4] = {vym.x, vym.y, vym.z, vym.w};
    const uint32_t yp[4] = {vyp.x, vyp.y, vyp.z, vyp.w};
    const uint32_t zm[4] = {vzm.x, vzm.y, vzm.z, vzm.w};
    const uint32_t zp[4] = {vzp.x, vzp.y, vzp.z, vzp.w};
    uint32_t u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        u[k] = (me[k] >> 7) & kOnes;
    // bytes of colour p: those whose offset k in the chunk has the parity
    // (p + y + z) & 1 (x0 is even); as 0x01 flags per byte
    const uint32_t kpar = (p + y + z) & 1u;
    const uint32_t cm = kpar ? 0x01000100u : 0x00010001u;
    const Off j0 = (Off)z * L * (L >> 1) + (Off)y * (L >> 1) + (x0 >> 1);
    uint32_t ge4[4], eq3[4], ties = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t xl = (u[k] << 8) | (k == 0 ? lbit : u[k - 1] >> 24);
        const uint32_t xr = (u[k] >> 8) | ((k == 3 ? rbit : u[k + 1]) << 24);
        const uint32_t a = (u[k] ^ xl) + (u[k] ^ xr) + (u[k] ^ ((ym[k] >> 7) & kOnes)) +
                           (u[k] ^ ((yp[k] >> 7) & kOnes)) + (u[k] ^ ((zm[k] >> 7) & kOnes)) +
                           (u[k] ^ ((zp[k] >> 7) & kOnes));
        asum += byte_sum(a & (cm * 7u));
        ge4[k] = (a >> 2) & cm;                          // a <= 6: bit 2 set iff a >= 4
        eq3[k] = a & (a >> 1) & ~(a >> 2) & cm;          // a == 3
        ties |= eq3[k];
    }
    uint32_t r[4] = {0u, 0u, 0u, 0u};
    if (ties) {
        const Words4 w = philox10((uint32_t)(j0 >> 7), t, p, 0u, k0, k1);
        const uint32_t sel = (uint32_t)(j0 >> 5) & 3u;     // selected, not indexed (no scratch)
        const uint32_t word = sel == 0u ? w.w[0] : sel == 1u ? w.w[1] : sel == 2u ? w.w[2] : w.w[3];
        const uint32_t bits = (word >> (j0 & 31)) & 0xFFu;
        // site m (j0 + m) is byte 2m + kpar of the chunk
#pragma unroll
        for (int k = 0; k < 4; ++k)
            r[k] = (((bits >> (2 * k)) & 1u) << (8 * kpar)) |
                   (((bits >> (2 * k + 1)) & 1u) << (8 * (2 + kpar)));
    }
    uint32_t out[4], any = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t f = ge4[k] | (eq3[k] & r[k]);
        fsum += byte_sum(f);
        out[k] = me[k] ^ (f * 0xFEu);                    // +1 (0x01) <-> -1 (0xFF)
        any |= f;
    }
    if (any)
        st16(rb + x0, make_uint4(out[0], out[1], out[2], out[3]));
}

// Half-sweep for L % 16 == 0: thread per 16-byte chunk of one plane
// (blockIdx.y = z), global memory.
__global__ void __launch_bounds__(kThreads)
    k_i8_half16(uint32_t L, uint32_t k0, uint32_t k1, uint32_t t, uint32_t which, uint32_t mixed,
                int8_t *s, unsigned long long *bond_acc, unsigned long long *flip_acc)
{
    const uint32_t p = half_colour(which, mixed, t, k0, k1);
    const uint32_t C = L >> 4, z = blockIdx.y;
    const uint32_t q = blockIdx.x * kThreads + threadIdx.x;   // chunk within the plane
    uint32_t asum = 0, fsum = 0;
    if (q < L * C) {
        const uint32_t cx = q % C, y = q / C;
        i8_chunk<uint64_t>(
            L, p, y, z, cx << 4, t, k0, k1,
            [&](uint64_t o) { return *reinterpret_cast<const uint4 *>(s + o); },
            [&](uint64_t o) { return s[o]; },
            [&](uint64_t o, uint4 v) { *reinterpret_cast<uint4 *>(s + o) = v; }, asum, fsum);
    }
    if (bond_acc != nullptr)
        block_add_u64(asum, bond_acc);
    if (flip_acc != nullptr)
        block_add_u64(fsum, flip_acc);
}

// n sweeps of a small lattice (L = 16 or 32, at most 32 KiB) in one launch
// of one workgroup holding the whole lattice in LDS: per
// half-sweep every thread updates its chunks in place (a colour-p update
// reads only colour 1 - p), then a barrier; the lattice goes back to global
// memory at the end.  Sweep t0 + k with k % every == 0 (every > 0) adds its
// entering bond count to dev_B[k / every] and the spins it flips to
// dev_F[k / every] (either pointer may be null).
constexpr uint32_t kI8OnchipThreads = 1024;

__global__ void __launch_bounds__(kI8OnchipThreads)
    k_i8_onchip(uint32_t L, uint32_t k0, uint32_t k1, uint32_t t0, uint32_t n, uint32_t mixed,
                int8_t *s, uint32_t every, unsigned long long *dev_B, unsigned long long *dev_F)
{
    extern __shared__ uint4 i8o_sm[];
    __shared__ unsigned long long red[2][kI8OnchipThreads / 64];
    int8_t *lat = reinterpret_cast<int8_t *>(i8o_sm);
    const uint32_t N = L * L * L, tid = threadIdx.x;
    for (uint32_t i = tid; i < N / 16; i += kI8OnchipThreads)
        i8o_sm[i] = reinterpret_cast<const uint4 *>(s)[i];
    __syncthreads();
    const uint32_t C = L >> 4, nchunks = L * L * C;
    auto ld16 = [&](uint32_t o) { return *reinterpret_cast<const uint4 *>(lat + o); };
    auto ld1 = [&](uint32_t o) { return lat[o]; };
    auto st16 = [&](uint32_t o, uint4 v) { *reinterpret_cast<uint4 *>(lat + o) = v; };
    // L is 16 or 32: chunk q = cx + C (y + L z) by shifts
    const uint32_t lc = C == 1u ? 0u : 1u, ll = L == 16u ? 4u : 5u;
    for (uint32_t k = 0; k < n; ++k) {
        const uint32_t t = t0 + k;
        const bool traced = every != 0u && k % every == 0u;
        uint32_t asum = 0, fsum = 0;
        for (uint32_t which = 0; which < 2; ++which) {
            const uint32_t p = half_colour(which, mixed, t, k0, k1);
            uint32_t a = 0;
#pragma unroll 1
            for (uint32_t q = tid; q < nchunks; q += kI8OnchipThreads) {
                const uint32_t row = q >> lc;
                i8_chunk<uint32_t>(L, p, row & (L - 1u), row >> ll, (q & (C - 1u)) << 4, t, k0, k1,
                                   ld16, ld1, st16, a, fsum);
            }
            if (which == 0)
                asum = a;
            __syncthreads();
        }
        if (traced && (dev_B != nullptr || dev_F != nullptr)) {
            const unsigned long long wb = wave_sum_u64(asum), wf = wave_sum_u64(fsum);
            if ((tid & 63u) == 0u) {
                red[0][tid >> 6] = wb;
                red[1][tid >> 6] = wf;
            }
            __syncthreads();
            if (tid == 0) {
                unsigned long long b = 0, f = 0;
                for (uint32_t w = 0; w < kI8OnchipThreads / 64; ++w) {
                    b += red[0][w];
                    f += red[1][w];
                }
                if (dev_B != nullptr)
                    dev_B[k / every] += b;
                if (dev_F != nullptr)
                    dev_F[k / every] += f;
            }
            __syncthreads();
        }
    }
    for (uint32_t i = tid; i < N / 16; i += kI8OnchipThreads)
        reinterpret_cast<uint4 *>(s)[i] = i8o_sm[i];
}

// Per-axis unsatisfied bonds: [s_i != s_{i+e_x}], [.. e_y], [.. e_z]; thread
// per column (x, y), looping over z.
__global__ void __launch_bounds__(kThreads) k_i8_bonds(uint32_t L, const int8_t *s,
                                                       unsigned long long *acc3)
{
    unsigned long long bx = 0, by = 0, bz = 0;
    const uint32_t col = blockIdx.x * kThreads + threadIdx.x;
    if (col < L * L) {
        const uint32_t x = col % L, y = col / L;
        const uint64_t LL = (uint64_t)L * L;
        const uint64_t ox = (uint64_t)y * L + wrap_up(x, L), oy = (uint64_t)wrap_up(y, L) * L + x;
        int8_t nz = s[col];
        for (uint32_t z = 0; z < L; ++z) {
            const uint64_t zo = (uint64_t)z * LL;
            const int8_t me = nz;
            nz = s[(uint64_t)wrap_up(z, L) * LL + col];
            bx += s[zo + ox] != me;
            by += s[zo + oy] != me;
            bz += nz != me;
        }
    }
    block_add_u64(bx, acc3 + 0);
    block_add_u64(by, acc3 + 1);
    block_add_u64(bz, acc3 + 2);
}

// Correlation sums S_a(r) = sum_i s_i s_{i + r e_a}, r = 0..L/2, and
// M = sum_i s_i.  A workgroup takes X lines along axis a (line position u,
// transverse index v in [v0, v0 + X), the third coordinate o fixed) and
// stages them in LDS, each padded with its own first bytes again (circular
// continuation) so that a shifted read never wraps.  Work item (line, r-block
// of 8): for every aligned word k of the line (4 sites u = 4k .. 4k+3) the 8
// shifted words starting at byte 4k + r come from three words by byte
// alignment, and a signed 4-way byte dot product accumulates each
// separation: 8 dot products and 6 alignments per 32 products.  Per-block
// sums meet in LDS (32-bit: at most X L per entry) and go to the global
// 64-bit sums once per block.  Element (u, v, o) sits at
//   x lines: u + L v + L^2 o;  y lines: L u + v + L^2 o;  z lines: L^2 u + v + L o.
struct I8CorrGeom {
    uint32_t L, R, X, Lp, nrb, ntile;   // Lp: staged bytes per line (multiple of 4)
};

__global__ void __launch_bounds__(kThreads) k_i8_corr(I8CorrGeom g, const int8_t *s,
                                                      unsigned long long *S)
{
    extern __shared__ uint32_t i8c_sm[];
    const uint32_t L = g.L, R = g.R, X = g.X, Lp = g.Lp;
    int *sS = reinterpret_cast<int *>(i8c_sm);              // [R] this block's sums, then M
    int8_t *buf = reinterpret_cast<int8_t *>(i8c_sm + R + 1);   // [X][Lp]
    const uint32_t tile = blockIdx.x % g.ntile;
    const uint32_t o = (blockIdx.x / g.ntile) % L;
    const uint32_t a = blockIdx.x / (g.ntile * L);
    const uint32_t v0 = tile * X;
    const uint32_t nl = min(X, L - v0);                     // lines in this block
    for (uint32_t k = threadIdx.x; k <= R; k += kThreads)
        sS[k] = 0;
    const uint64_t LL = (uint64_t)L * L;
    // staging: the memory-contiguous coordinate runs fastest across threads
    const uint32_t nst = nl * Lp;
    for (uint32_t e = threadIdx.x; e < nst; e += kThreads) {
        uint32_t u, vl;
        if (a == 0) {
            vl = e / Lp;
            u = e % Lp;
        } else {
            u = e / nl;
            vl = e % nl;
        }
        const uint32_t uu = u % L, v = v0 + vl;
        const uint64_t off = a == 0 ? uu + (uint64_t)L * v + LL * o
                           : a == 1 ? (uint64_t)L * uu + v + LL * o
                                    : LL * uu + v + (uint64_t)L * o;
        buf[(size_t)vl * Lp + u] = s[off];
    }
    __syncthreads();
    const uint32_t nk = (L + 3) / 4;                        // words of a line's sites
    const uint32_t tail = L % 4;                            // sites in a partial last word
    const uint32_t last_mask = tail ? (1u << (8 * tail)) - 1u : 0xFFFFFFFFu;
    int m_acc = 0;
    for (uint32_t item = threadIdx.x; item < nl * g.nrb; item += kThreads) {
        const uint32_t vl = item / g.nrb, rb = item % g.nrb;
        const uint32_t r0 = 8u * rb;
        const uint32_t *lw = reinterpret_cast<const uint32_t *>(buf + (size_t)vl * Lp);
        int acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const uint32_t kb = r0 / 4;
        uint32_t w0 = lw[kb], w1 = lw[kb + 1], w2 = lw[kb + 2];
        for (uint32_t k = 0; k < nk; ++k) {
            uint32_t av = lw[k];
            if (k + 1 == nk)
                av &= last_mask;                            // sites past L contribute nothing
            const int ai = (int)av;
            acc[0] = __builtin_amdgcn_sdot4(ai, (int)w0, acc[0], false);
            acc[1] = __builtin_amdgcn_sdot4(ai, (int)__builtin_amdgcn_alignbyte(w1, w0, 1), acc[1], false);
            acc[2] = __builtin_amdgcn_sdot4(ai, (int)__builtin_amdgcn_alignbyte(w1, w0, 2), acc[2], false);
            acc[3] = __builtin_amdgcn_sdot4(ai, (int)__builtin_amdgcn_alignbyte(w1, w0, 3), acc[3], false);
            acc[4] = __builtin_amdgcn_sdot4(ai, (int)w1, acc[4], false);
            acc[5] = __builtin_amdgcn_sdot4(ai, (int)__builtin_amdgcn_alignbyte(w2, w1, 1), acc[5], false);
            acc[6] = __builtin_amdgcn_sdot4(ai, (int)__builtin_amdgcn_alignbyte(w2, w1, 2), acc[6], false);
            acc[7] = __builtin_amdgcn_sdot4(ai, (int)__builtin_amdgcn_alignbyte(w2, w1, 3), acc[7], false);
            w0 = w1;
            w1 = w2;
            w2 = lw[kb + k + 3];
            if (a == 0 && rb == 0)
                m_acc = __builtin_amdgcn_sdot4(ai, 0x01010101, m_acc, false);
        }
#pragma unroll
        for (int d = 0; d < 8; ++d)
            if (r0 + d < R)
                atomicAdd(sS + r0 + d, acc[d]);
    }
    if (a == 0 && m_acc != 0)
        atomicAdd(sS + R, m_acc);
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < R; k += kThreads)
        if (sS[k] != 0)
            atomicAdd(S + (size_t)a * R + k, (unsigned long long)(long long)sS[k]);
    if (a == 0 && threadIdx.x == 0 && sS[R] != 0)
        atomicAdd(S + 3 * (size_t)R, (unsigned long long)(long long)sS[R]);
}

__global__ void __launch_bounds__(kThreads) k_i8_check(uint64_t n, const int8_t *s,
                                                       unsigned long long *bad)
{
    unsigned long long b = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kThreads)
        b += (s[i] != 1 && s[i] != -1);
    block_add_u64(b, bad);
}

__global__ void __launch_bounds__(kThreads)
    k_i8_window(uint32_t L, const int8_t *s, uint32_t ox, uint32_t oy, uint32_t oz, uint32_t W,
                uint32_t lz0, uint64_t n, int8_t *out)
{
    const uint64_t WW = (uint64_t)W * W;
    for (uint64_t k = (uint64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
         k += (uint64_t)gridDim.x * kThreads) {
        const uint32_t lx = (uint32_t)(k % W), ly = (uint32_t)((k / W) % W);
        const uint32_t lz = lz0 + (uint32_t)(k / WW);
        const uint64_t x = (ox + lx) % L, y = (oy + ly) % L, z = (oz + lz) % L;
        out[k] = s[(z * L + y) * L + x];
    }
}

__global__ void __launch_bounds__(kThreads) k_fill_u64(unsigned long long *p, uint64_t n,
                                                       unsigned long long v)
{
    for (uint64_t k = (uint64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
         k += (uint64_t)gridDim.x * kThreads)
        p[k] = v;
}

uint32_t grid_for(uint64_t work, uint32_t cap)
{
    uint64_t g = (work + kThreads - 1) / kThreads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

}  // namespace

hipError_t i8_init(hipStream_t st, uint32_t L, uint64_t seed, int8_t *s)
{
    const uint64_t N = (uint64_t)L * L * L;
    const uint64_t blocks = (N + 128 - 1) / 128;
    const uint32_t g = (uint32_t)((blocks + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_i8_init, dim3(g), dim3(kThreads), 0, st, N, (uint32_t)seed,
                       (uint32_t)(seed >> 32), s);
    return hipGetLastError();
}

hipError_t i8_half_sweep(hipStream_t st, uint32_t L, uint64_t seed, uint32_t t, int which,
                         bool mixed, int8_t *s, unsigned long long *bond_acc,
                         unsigned long long *flip_acc)
{
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (L % 16 == 0) {
        const dim3 grid((L * (L / 16) + kThreads - 1) / kThreads, L);
        hipLaunchKernelGGL(k_i8_half16, grid, dim3(kThreads), 0, st, L, k0, k1, t,
                           (uint32_t)which, mixed ? 1u : 0u, s, bond_acc, flip_acc);
    } else {
        const dim3 grid((L * (L / 2) + kThreads - 1) / kThreads, L);
        hipLaunchKernelGGL(k_i8_half, grid, dim3(kThreads), 0, st, L, k0, k1, t, (uint32_t)which,
                           mixed ? 1u : 0u, s, bond_acc, flip_acc);
    }
    return hipGetLastError();
}

bool i8_onchip_ok(uint32_t L) { return L == 16 || L == 32; }

hipError_t i8_onchip_run(hipStream_t st, uint32_t L, uint64_t seed, uint32_t t0, uint32_t n,
                         bool mixed, int8_t *s, uint32_t every, unsigned long long *dev_B,
                         unsigned long long *dev_F)
{
    if (!i8_onchip_ok(L))
        return hipErrorInvalidValue;
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_i8_onchip, dim3(1), dim3(kI8OnchipThreads), (size_t)L * L * L, st, L,
                       (uint32_t)seed, (uint32_t)(seed >> 32), t0, n, mixed ? 1u : 0u, s, every,
                       dev_B, dev_F);
    return hipGetLastError();
}

hipError_t i8_bonds(hipStream_t st, uint32_t L, const int8_t *s, unsigned long long *acc3)
{
    hipLaunchKernelGGL(k_i8_bonds, dim3((L * L + kThreads - 1) / kThreads), dim3(kThreads), 0, st,
                       L, s, acc3);
    return hipGetLastError();
}

hipError_t i8_corr(hipStream_t st, uint32_t L, const int8_t *s, long long *S, long long *M)
{
    // S and M are contiguous: M sits at S[3*(L/2+1)].
    (void)M;
    I8CorrGeom g;
    g.L = L;
    g.R = L / 2 + 1;
    g.nrb = (g.R + 7) / 8;
    // staged bytes per line: the line, then its continuation far enough for
    // the largest r-block's three-word window to stay inside
    g.Lp = ((L + 8 * g.nrb + 16) + 3) / 4 * 4;
    uint32_t X = 40960 / g.Lp;
    X = std::max(1u, std::min({X, 64u, L}));
    g.X = X;
    g.ntile = (L + X - 1) / X;
    const size_t lds = (size_t)(g.R + 1) * 4 + (size_t)X * g.Lp;
    const uint64_t blocks = 3ull * L * g.ntile;
    if (blocks > 0x7FFFFFFFull)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_i8_corr, dim3((uint32_t)blocks), dim3(kThreads), lds, st, g, s,
                       reinterpret_cast<unsigned long long *>(S));
    return hipGetLastError();
}

hipError_t i8_check_pm1(hipStream_t st, size_t n, const int8_t *s, unsigned long long *bad)
{
    hipLaunchKernelGGL(k_i8_check, dim3(grid_for(n, 2048)), dim3(kThreads), 0, st, (uint64_t)n, s,
                       bad);
    return hipGetLastError();
}

hipError_t i8_window(hipStream_t st, uint32_t L, const int8_t *s, uint32_t ox, uint32_t oy,
                     uint32_t oz, uint32_t W, uint32_t lz0, uint32_t nz, int8_t *out)
{
    const uint64_t n = (uint64_t)W * W * nz;
    hipLaunchKernelGGL(k_i8_window, dim3(grid_for(n, 8192)), dim3(kThreads), 0, st, L, s, ox, oy,
                       oz, W, lz0, n, out);
    return hipGetLastError();
}

hipError_t fill_u64(hipStream_t st, unsigned long long *p, size_t n, unsigned long long v)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 1024)), dim3(kThreads), 0, st, p, (uint64_t)n,
                       v);
    return hipGetLastError();
}

}  // namespace qz
