// qz_corr.hip -- axis correlation sums of the 1-bit layout.
//
// S_a(r) = sum_i s_i s_{i + r e_a} = N - 2 * anti_a(r), where anti_a(r) counts
// the site pairs at separation r along axis a whose spins differ (the integer
// pieces of C(r,t), Results, eq:correlation function), for r = 0..L/2.  Where
// L is a multiple of 256 they come from Gram matrices on the matrix cores
// (k_corr_gram, further down); elsewhere the kernels below accumulate
// anti_a(r) with XOR + popcount on 32 sites at a time.
//
// Lines along y or z: for x-parity pi, word column w and fixed other
// coordinate o (z for the y axis, y for the z axis), the words
//   line[u] = P_{(pi + u + o) & 1}[row u][w],  u = 0..L-1,
// hold 32 parallel lines of sites along the axis (the colour alternates with
// u, the x-parity stays fixed).  anti(r) += popc(line[u] ^ line[u + r]).
//
// Rows along x: the even-x and odd-x sites of row (y, z) are the colour
// planes (y+z)&1 and its complement (rows E and O).  With
// rot(X, m)[k] = X[(k + m) mod L/2]:
//   r = 2m      pairs E[k]-E[k+m] and O[k]-O[k+m]
//   r = 2m + 1  pairs E[k]-O[k+m] and O[k]-E[k+m+1].
#include <algorithm>

#include "qz_device.hpp"
#include "qz_internal.hpp"

namespace qz {
namespace {

constexpr int kBlock = 256;
constexpr int kG = 8;             // separations per register block
constexpr int kItems = 2;         // work items per thread in k_corr_lines
constexpr int kFill = 8;          // loads in flight per thread while filling LDS
constexpr int kPipeA = 16;        // prefetched rows of region A per thread
constexpr int kPipeB = 32;        // prefetched rows of region B per thread
constexpr size_t kLineLds = 56 * 1024;

struct LineGeom {
    uint32_t L, W, R;             // R = L/2 + 1 separations
    uint32_t Cy;                  // rows of u per tile
    uint32_t Rr;                  // separations per block (multiple of kG)
    uint32_t nrc;                 // separation chunks
    uint32_t nsplit;              // blocks per separation chunk
};

__host__ __device__ inline size_t line_lds_bytes(uint32_t W, uint32_t Cy, uint32_t Rr)
{
    return (size_t)2 * W * ((Cy + 1) + (Cy + Rr + 1)) * 4;
}

// One block owns separations [r_base, r_base + Rr) and a strided share of the
// tiles (o, Y), Y a multiple of Cy.  LDS holds, column-major, rows [Y, Y+Cy)
// (region A) and [Y+r_base, Y+r_base+Cy+Rr) (region B) of both colour planes:
// column c*W + w is word w of colour plane c, one entry per row, padded to an
// odd length so that lanes (consecutive columns) hit distinct banks.  For line
// (pi, w) the colour alternates with the row, so even and odd rows come from
// two fixed columns and every read uses an immediate offset.  Threads keep
// their partial sums in registers over all tiles and add them to the global
// counts once.
template <int AX>
__global__ void __launch_bounds__(kBlock) k_corr_lines(LineGeom g, const uint32_t *P0,
                                                      const uint32_t *P1, unsigned long long *anti)
{
    extern __shared__ uint32_t sm[];
    const uint32_t L = g.L, W = g.W, W2 = 2 * g.W;
    const uint32_t nrc = g.nrc;
    // blocks on one XCD (bid % 8) share splits, so they read the same planes
    const uint32_t bid = blockIdx.x;
    const uint32_t rc = (bid / 8) % nrc;
    const uint32_t split = (bid % 8) + 8 * (bid / (8 * nrc));
    const uint32_t r_base = rc * g.Rr;
    const uint32_t r_end = min(r_base + g.Rr, g.R);
    const uint32_t ngr = (r_end - r_base + kG - 1) / kG;   // register blocks in this chunk
    const uint32_t nitems = ngr * W2;
    const uint32_t Cy = g.Cy, PA = g.Cy + 1, PB = g.Cy + g.Rr + 1;
    uint32_t *A = sm;
    uint32_t *B = sm + (size_t)W2 * PA;
    const size_t plane = (size_t)L * W;
    const uint32_t ytiles = L / Cy;
    const uint32_t ntiles = L * ytiles;
    // fill geometry: thread -> (column fcw = c*W + w, first row fs0), frows rows apart
    const uint32_t frows = kBlock / W2;           // >= 1 since W2 <= 128
    const uint32_t fcw = threadIdx.x % W2, fs0 = threadIdx.x / W2;
    const bool fill_active = fs0 < frows;
    const uint32_t *fP = ((fcw / W) ? P1 : P0) + (fcw % W);
    const size_t ustride = (AX == 1) ? (size_t)W : plane;   // words between consecutive rows u

    uint32_t acc[kItems][kG];
#pragma unroll
    for (int k = 0; k < kItems; ++k)
#pragma unroll
        for (int d = 0; d < kG; ++d)
            acc[k][d] = 0u;

    // The LDS fill of tile t+1 is loaded into registers while tile t is being
    // counted (kPipeA + kPipeB words per thread), so the loads' latency hides
    // behind the arithmetic; larger fills fall back to batched loads.
    const uint32_t nb = Cy + g.Rr;                       // rows of region B
    const uint32_t fr = frows % L;
    const uint32_t na = fill_active ? (Cy > fs0 ? (Cy - fs0 + frows - 1) / frows : 0u) : 0u;
    const uint32_t nbb = fill_active ? (nb > fs0 ? (nb - fs0 + frows - 1) / frows : 0u) : 0u;
    const bool pipelined = __syncthreads_and(na <= (uint32_t)kPipeA && nbb <= (uint32_t)kPipeB);
    uint32_t va[kPipeA], vb[kPipeB];
    auto fetch = [&](uint32_t tile) {
        const uint32_t o = tile / ytiles;
        const uint32_t Y = (tile % ytiles) * Cy;
        const uint32_t *col = fP + (AX == 1 ? (size_t)o * plane : (size_t)o * W);
#pragma unroll
        for (int j = 0; j < kPipeA; ++j)
            va[j] = (uint32_t)j < na ? col[(size_t)(Y + fs0 + j * frows) * ustride] : 0u;
        uint32_t u = (Y + r_base + fs0) % L;
#pragma unroll
        for (int j = 0; j < kPipeB; ++j) {
            vb[j] = (uint32_t)j < nbb ? col[(size_t)u * ustride] : 0u;
            u += fr;
            if (u >= L)
                u -= L;
        }
    };
    if (pipelined && split < ntiles)
        fetch(split);

    for (uint32_t tile = split; tile < ntiles; tile += g.nsplit) {
        const uint32_t o = tile / ytiles;
        const uint32_t Y = (tile % ytiles) * Cy;
        __syncthreads();
        if (pipelined) {
#pragma unroll
            for (int j = 0; j < kPipeA; ++j)
                if ((uint32_t)j < na)
                    A[fcw * PA + fs0 + j * frows] = va[j];
#pragma unroll
            for (int j = 0; j < kPipeB; ++j)
                if ((uint32_t)j < nbb)
                    B[fcw * PB + fs0 + j * frows] = vb[j];
            __syncthreads();
            if (tile + g.nsplit < ntiles)
                fetch(tile + g.nsplit);
        } else {
            // fill: this thread always loads column fcw; rows advance by frows,
            // in batches of kFill loads before any is stored
            if (fill_active) {
                const uint32_t *col = fP + (AX == 1 ? (size_t)o * plane : (size_t)o * W);
                for (uint32_t s = fs0; s < Cy; s += kFill * frows) {   // A: rows Y .. Y+Cy-1
                    uint32_t v[kFill];
#pragma unroll
                    for (int j = 0; j < kFill; ++j) {
                        const uint32_t sj = s + j * frows;
                        v[j] = sj < Cy ? col[(size_t)(Y + sj) * ustride] : 0u;
                    }
#pragma unroll
                    for (int j = 0; j < kFill; ++j) {
                        const uint32_t sj = s + j * frows;
                        if (sj < Cy)
                            A[fcw * PA + sj] = v[j];
                    }
                }
                for (uint32_t s = fs0; s < nb; s += kFill * frows) {   // B: from Y + r_base, wrapping
                    uint32_t v[kFill];
                    uint32_t u = (Y + r_base + s) % L;
#pragma unroll
                    for (int j = 0; j < kFill; ++j) {
                        const uint32_t sj = s + j * frows;
                        v[j] = sj < nb ? col[(size_t)u * ustride] : 0u;
                        u += fr;
                        if (u >= L)
                            u -= L;
                    }
#pragma unroll
                    for (int j = 0; j < kFill; ++j) {
                        const uint32_t sj = s + j * frows;
                        if (sj < nb)
                            B[fcw * PB + sj] = v[j];
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint32_t it = threadIdx.x + k * kBlock;
            if (it >= nitems)
                break;
            const uint32_t col = it % W2, gr = it / W2;
            const uint32_t pi = col / W, w = col % W;
            const uint32_t r0 = gr * kG;            // relative to r_base
            // colour of even rows of the line in A and in B
            const uint32_t cA = (pi + Y + o) & 1u, cB = (pi + Y + r_base + o) & 1u;
            const uint32_t *Ae = A + (cA * W + w) * PA, *Ao = A + ((1u - cA) * W + w) * PA;
            const uint32_t *Be = B + (cB * W + w) * PB + r0, *Bo = B + ((1u - cB) * W + w) * PB + r0;
            uint32_t b[2 * kG];
#pragma unroll
            for (int j = 0; j < kG; ++j)
                b[j] = (j & 1) ? Bo[j] : Be[j];
            for (uint32_t u = 0; u < Cy; u += kG) {
                uint32_t a[kG];
#pragma unroll
                for (int i = 0; i < kG; ++i) {
                    a[i] = (i & 1) ? Ao[u + i] : Ae[u + i];
                    b[kG + i] = (i & 1) ? Bo[u + kG + i] : Be[u + kG + i];
                }
#pragma unroll
                for (int i = 0; i < kG; ++i)
#pragma unroll
                    for (int d = 0; d < kG; ++d)
                        acc[k][d] = popc_acc(a[i] ^ b[i + d], acc[k][d]);
#pragma unroll
                for (int j = 0; j < kG; ++j)
                    b[j] = b[kG + j];
            }
        }
    }
    // flush: per-separation block sums in LDS, then one global atomic each
    __syncthreads();
    unsigned long long *bacc = reinterpret_cast<unsigned long long *>(sm);
    for (uint32_t r = threadIdx.x; r < g.Rr; r += kBlock)
        bacc[r] = 0ull;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint32_t it = threadIdx.x + k * kBlock;
        if (it >= nitems)
            break;
        const uint32_t gr = it / W2;
#pragma unroll
        for (int d = 0; d < kG; ++d) {
            const uint32_t rr = gr * kG + d;
            if (r_base + rr < r_end && acc[k][d])
                atomicAdd(bacc + rr, (unsigned long long)acc[k][d]);
        }
    }
    __syncthreads();
    for (uint32_t rr = threadIdx.x; rr < r_end - r_base; rr += kBlock)
        if (bacc[rr])
            atomicAdd(anti + r_base + rr, bacc[rr]);
}

// x axis.  Thread (q, ph): shift group q covers m = 16q .. 16q+15; phase ph
// picks rows.  Rows are staged in LDS in chunks of P rows (P phases), both E
// and O words.  Partial sums stay in registers over all rows of the thread.
__global__ void __launch_bounds__(kBlock) k_corr_x(uint32_t L, uint32_t W, const uint32_t *P0,
                                                  const uint32_t *P1, unsigned long long *anti,
                                                  unsigned long long *ones)
{
    extern __shared__ uint32_t sm[];
    const uint32_t P = kBlock / W;                  // rows per chunk (phases)
    const uint32_t q = threadIdx.x % W, ph = threadIdx.x / W;
    const bool active = ph < P;
    const uint32_t W2 = 2 * W;
    const uint64_t nrows = (uint64_t)L * L;
    const uint64_t nchunks = (nrows + P - 1) / P;
    const uint32_t quarter = L / 4;                 // m ranges over [0, L/4)
    const uint32_t qq = (16 * q) / 32, sb = (16 * q) % 32;
    // r = L/2 (m = L/4): word offset and bit offset of that rotation
    const uint32_t hq = quarter / 32, hs = quarter % 32;

    uint32_t ae[16], ao[16];
#pragma unroll
    for (int s = 0; s < 16; ++s)
        ae[s] = ao[s] = 0u;
    uint32_t half = 0, my_ones = 0;

    for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < P * W2; k += kBlock) {
            const uint32_t rr = k / W2, cw = k % W2;
            const uint64_t row = ch * P + rr;
            uint32_t v = 0;
            if (row < nrows) {
                const uint32_t y = (uint32_t)(row % L), z = (uint32_t)(row / L);
                const uint32_t ce = (y + z) & 1u;             // colour of the even-x sites
                const uint32_t c = (cw < W) ? ce : 1u - ce;   // first W words: E, then O
                v = (c ? P1 : P0)[(size_t)row * W + (cw % W)];
            }
            sm[k] = v;
        }
        __syncthreads();
        const uint64_t row = ch * P + ph;
        if (!active || row >= nrows)
            continue;
        const uint32_t *E = sm + ph * W2, *O = E + W;
        for (uint32_t w = 0; w < W; ++w) {
            const uint32_t e0 = E[w], o0 = O[w];
            const uint32_t ea = E[(w + qq) % W], eb = E[(w + qq + 1) % W];
            const uint32_t oa = O[(w + qq) % W], ob = O[(w + qq + 1) % W];
            // re[k] = rot(E, 16q + k) for k = 0..16; shift 32 is the next word
            uint32_t re[17];
#pragma unroll
            for (int k = 0; k < 16; ++k)
                re[k] = funnel(eb, ea, sb + k);
            re[16] = (sb == 0u) ? funnel(eb, ea, 16) : eb;
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const uint32_t ro = funnel(ob, oa, sb + s);                   // rot(O, m)
                ae[s] = popc_acc(o0 ^ ro, popc_acc(e0 ^ re[s], ae[s]));
                ao[s] = popc_acc(o0 ^ re[s + 1], popc_acc(e0 ^ ro, ao[s]));
            }
            if (q == 0) {
                my_ones += __builtin_popcount(e0) + __builtin_popcount(o0);
                const uint32_t ha = E[(w + hq) % W], hb = E[(w + hq + 1) % W];
                const uint32_t ga = O[(w + hq) % W], gb = O[(w + hq + 1) % W];
                half += __builtin_popcount(e0 ^ funnel(hb, ha, hs)) +
                        __builtin_popcount(o0 ^ funnel(gb, ga, hs));
            }
        }
    }
    // flush
    __syncthreads();
    const uint32_t R = L / 2 + 1;
    unsigned long long *bacc = reinterpret_cast<unsigned long long *>(sm);
    for (uint32_t r = threadIdx.x; r <= R; r += kBlock)
        bacc[r] = 0ull;                 // bacc[R] collects the up-spin count
    __syncthreads();
    if (active) {
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const uint32_t m = 16 * q + s;
            if (m < quarter) {
                if (ae[s])
                    atomicAdd(bacc + 2 * m, (unsigned long long)ae[s]);
                if (ao[s])
                    atomicAdd(bacc + 2 * m + 1, (unsigned long long)ao[s]);
            }
        }
        if (q == 0) {
            if (half)
                atomicAdd(bacc + R - 1, (unsigned long long)half);
            if (my_ones)
                atomicAdd(bacc + R, (unsigned long long)my_ones);
        }
    }
    __syncthreads();
    for (uint32_t r = threadIdx.x; r < R; r += kBlock)
        if (bacc[r])
            atomicAdd(anti + r, bacc[r]);
    if (threadIdx.x == 0 && bacc[R])
        atomicAdd(ones, bacc[R]);
}

// ---------------------------------------------------------------------------
// Axis sums on the matrix cores (y and z directly, x through the copy with x
// and y swapped, below).  For axis a, row u is the plane of sites
// at coordinate u along a, and column k one of the L^2 lines along a; with
// b = 1 for up spins, the Gram matrix G[u][u'] = sum_k b(u,k) b(u',k) gives
//   T(r) = sum_u G[u][(u + r) mod L]   (up-up pairs at separation r),
// and the anti-aligned pair count is anti(r) = 2 (N_up - T(r)), since every
// site has one partner at +r: the pairs with at least one up spin number
// 2 N_up - T(r), of which T(r) are up-up.
//
// G is a plain matrix product of 0/1 entries: each wave owns a 128 x 32 NB
// tile of G (4 x NB blocks of 32 x 32) over a chunk of the lines; G is
// symmetric, so only tiles that reach the diagonal or beyond are computed and
// their entries below it are skipped.  The products run on the matrix cores
// with four-bit operands (E2M1: 0 and 0.5 are exact, so each up-up pair adds
// exactly 0.25 to a float accumulator), the densest exact form gfx950 has.
// A row's lines come as 32-bit words: word kappa = (o * 2 + p) * W + w holds
// the 32 lines (o, x = 64 w + 2 j + p) of row u, o being the third
// coordinate, from colour plane (p + u + o) & 1.  Both operands of an
// instruction must pair the same lines in the same order, and which ones does
// not matter: lane half h of a wave takes word kk = kappa0 + 4h + s of the
// row (s = 0..3) for instruction s, so 8 words feed 4 instructions per block.
// ---------------------------------------------------------------------------

constexpr uint32_t kGramTile = 128;   // rows of a wave's tile
constexpr int kGramNB = 4;            // 32-column blocks of a wave's tile (128 x 128)

struct GramGeom {
    uint32_t L, W, nT;     // nT = L / 128 row blocks
    uint32_t CW, ncb;      // tile columns (32 NB) and column blocks L / CW
    uint32_t ntile;        // tiles that reach the diagonal or beyond
    uint32_t nsplit;       // line chunks per tile
    uint32_t kchunk;       // words (of 32 lines) per chunk, a multiple of 8
    uint32_t NK;           // words per row, 2 L W
};

typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// The 32 lines of a word as 32 four-bit E2M1 values, 0 (down) or 0.5 (up,
// code 0001): dword d holds bits d, 4 + d, ..., 28 + d in its eight nibbles
// (mask 0x11111111; mask 0 gives all zeros).
// Every operand expands its words the same way, so both sides of an
// instruction pair the same lines; the upper four dwords are not read.
__device__ __forceinline__ v8i expand_fp4(uint32_t y, uint32_t mask)
{
    v8i f;
    f[0] = (int)(y & mask);
    f[1] = (int)((y >> 1) & mask);
    f[2] = (int)((y >> 2) & mask);
    f[3] = (int)((y >> 3) & mask);
    f[4] = f[5] = f[6] = f[7] = 0;
    return f;
}

// NB = 4: 128 x 128 tiles, one wave per SIMD (256 accumulator registers);
// NB = 2: 128 x 64 tiles, two waves per SIMD.  Each instruction
// (v_mfma_scale_f32_32x32x64_f8f6f4 on four-bit operands, unit scales)
// takes one word of 32 lines per row and lane half: 64 lines, products of
// 0.25 per up-up pair, exact in the float accumulators while a chunk holds
// fewer than 2^24 lines.
template <int AX, int NB>
__global__ void __launch_bounds__(256, 4 / NB) k_corr_gram(GramGeom g, const uint32_t *P0,
                                                  const uint32_t *P1, unsigned long long *tb)
{
    __shared__ uint32_t dsum[4][256];   // per wave: the tile's diagonals d - dbase
    const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint32_t i = lane & 31u, h = lane >> 5;
    // workgroups of one XCD take consecutive items (tiles of one chunk that
    // share row blocks), so that its L2 serves their common rows
    const uint32_t item = xcd_tile(blockIdx.x, gridDim.x) * 4u + wv;
    if (item >= g.ntile * g.nsplit)      // whole wave
        return;
    uint32_t *ds = dsum[wv];
    for (uint32_t k = lane; k < 256u; k += 64u)
        ds[k] = 0u;
    // chunk-major: the waves in flight work on the same few chunks of lines,
    // whose words (all rows) then stay in the last-level cache
    const uint32_t tile = item % g.ntile, split = item / g.ntile;
    // tile -> (bi, bj), row by row; row block bi starts at column block
    // 128 bi / CW (tiles wholly below the diagonal are mirrors: skipped)
    uint32_t bi = 0, rem = tile;
    while (rem >= g.ncb - kGramTile * bi / g.CW) {
        rem -= g.ncb - kGramTile * bi / g.CW;
        ++bi;
    }
    const uint32_t bj = kGramTile * bi / g.CW + rem;
    const uint32_t L = g.L, W = g.W, W2 = 2u * g.W;
    const uint32_t k_begin = split * g.kchunk, k_end = min(g.NK, k_begin + g.kchunk);

    v16f acc[4][NB];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                acc[m][n][r] = 0.0f;
    // Word kk of row u sits at word offset roff(u) + koff(kk) of colour plane
    // (p + u + o) & 1: roff = u W for y (o = z), u L W for z (o = y).  Every
    // row of a lane has the parity of i, so one plane serves all its rows.
    const uint32_t roffs = (AX == 1) ? W : L * W;
    uint32_t ra[4], rb[NB];
#pragma unroll
    for (int m = 0; m < 4; ++m)
        ra[m] = (bi * kGramTile + 32u * m + i) * roffs;
#pragma unroll
    for (int n = 0; n < NB; ++n)
        rb[n] = (bj * g.CW + 32u * n + i) * roffs;
    // Words come in groups of 8 (4 instruction steps).  Three groups are in
    // flight in three named buffers, so that a group's loads are issued about
    // two groups of multiplies before their first use (with one buffer copied
    // into another each group, the compiler waits for the loads at the top of
    // the next group instead).  The loop runs a multiple of 3 groups with no
    // branch inside, since a branch makes the compiler wait for every load at
    // the loop's head: a group past the chunk reloads the last group and is
    // multiplied with its A operand masked to zero, adding nothing.
    const uint32_t ng = (k_end - k_begin) / 8u;
    auto fetch = [&](uint4 (&xa)[4], uint4 (&xb)[NB], uint32_t gi) {
        const uint32_t kk = k_begin + 8u * min(gi, ng - 1u) + 4u * h;
        const uint32_t o = kk / W2, p = (kk / W) & 1u, w = kk % W;
        const uint32_t koff = (AX == 1) ? o * L * W + w : o * W + w;
        const uint32_t *P = ((p + i + o) & 1u) ? P1 : P0;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            xa[m] = *reinterpret_cast<const uint4 *>(P + (ra[m] + koff));
#pragma unroll
        for (int n = 0; n < NB; ++n)
            xb[n] = *reinterpret_cast<const uint4 *>(P + (rb[n] + koff));
    };
    auto word = [](const uint4 &q, int s) -> uint32_t {
        return s == 0 ? q.x : s == 1 ? q.y : s == 2 ? q.z : q.w;
    };
    // expansion mask of group gi's A operands: zero past the chunk
    auto amask = [&](uint32_t gi) -> uint32_t { return gi < ng ? 0x11111111u : 0u; };
    uint4 a0[4], b0[NB], a1[4], b1[NB], a2[4], b2[NB];
    fetch(a0, b0, 0u);
    fetch(a1, b1, 1u);
    fetch(a2, b2, 2u);
    v8i fa[4], fb[NB];
#pragma unroll
    for (int m = 0; m < 4; ++m)
        fa[m] = expand_fp4(a0[m].x, amask(0u));
#pragma unroll
    for (int n = 0; n < NB; ++n)
        fb[n] = expand_fp4(b0[n].x, 0x11111111u);
    // the 4 steps of one group (words ca, cb, A mask mc); the last step
    // expands the first word of the next group (na, nb, mask mn)
    auto group = [&](const uint4 (&ca)[4], const uint4 (&cb)[NB], uint32_t mc,
                     const uint4 (&na)[4], const uint4 (&nb)[NB], uint32_t mn) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            v8i ga[4], gb[NB];
#pragma unroll
            for (int m = 0; m < 4; ++m)
                ga[m] = st < 3 ? expand_fp4(word(ca[m], st + 1), mc) : expand_fp4(na[m].x, mn);
#pragma unroll
            for (int n = 0; n < NB; ++n)
                gb[n] = expand_fp4(st < 3 ? word(cb[n], st + 1) : nb[n].x, 0x11111111u);
#pragma unroll
            for (int m = 0; m < 4; ++m)
#pragma unroll
                for (int n = 0; n < NB; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                        fa[m], fb[n], acc[m][n], 4, 4, 0, 127, 0, 127);
            // one MFMA, then up to four VALU instructions, for each MFMA
#pragma unroll
            for (int q = 0; q < 4 * NB; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < 4; ++m)
                fa[m] = ga[m];
#pragma unroll
            for (int n = 0; n < NB; ++n)
                fb[n] = gb[n];
        }
    };
    for (uint32_t gi = 0; gi < ng; gi += 3u) {
        group(a0, b0, amask(gi), a1, b1, amask(gi + 1u));
        fetch(a0, b0, gi + 3u);
        group(a1, b1, amask(gi + 1u), a2, b2, amask(gi + 2u));
        fetch(a1, b1, gi + 4u);
        group(a2, b2, amask(gi + 2u), a0, b0, amask(gi + 3u));
        fetch(a2, b2, gi + 5u);
    }
    // diagonals of the tile: entry (row, col) of block (m, n) in register r of
    // this lane is row 32 m + 8 (r / 4) + 4 h + r % 4, column 32 n + i; its
    // separation is d = CW bj + col - 128 bi - row; entries with d < 0 are
    // the mirrors of entries of other tiles
    const int dbase = (int)(bj * g.CW) - (int)(bi * kGramTile) - 127;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 32 * m + 8 * (r / 4) + 4 * (int)h + (r % 4);
                const int col = 32 * n + (int)i;
                const uint32_t v = (uint32_t)(acc[m][n][r] * 4.0f);   // 0.25 per pair
                if (v != 0u && dbase + 127 + col - row >= 0)
                    atomicAdd(ds + (col - row + 127), v);
            }
    // fold: an entry at separation d (u < u') is the pair (u, u') at +d and
    // the pair (u', u) at +(L - d); T keeps r = 0 .. L/2
    const int half = (int)(L / 2);
    for (uint32_t k = lane; k < 255u; k += 64u) {
        const int d = dbase + (int)k;
        const uint32_t v = ds[k];
        if (v == 0u || d < 0)
            continue;
        if (d == 0) {
            atomicAdd(tb, (unsigned long long)v);
            continue;
        }
        if (d <= half)
            atomicAdd(tb + d, (unsigned long long)v);
        if (d >= half)
            atomicAdd(tb + ((int)L - d), (unsigned long long)v);
    }
}

// anti(r) = 2 (N_up - T(r)) in place, one block per axis from axis a0 on,
// with N_up = T(0) (the up-up pairs at separation 0); with x among the axes
// (a0 = 0) the block of axis 0 also stores N_up at *ones
__global__ void k_corr_gram_finish(unsigned long long *tb, uint32_t R, uint32_t a0,
                                   unsigned long long *ones)
{
    __shared__ unsigned long long t0;
    unsigned long long *t = tb + (size_t)(a0 + blockIdx.x) * R;
    if (threadIdx.x == 0) {
        t0 = t[0];
        if (a0 + blockIdx.x == 0)
            *ones = t0;
    }
    __syncthreads();
    for (uint32_t r = threadIdx.x; r < R; r += blockDim.x)
        t[r] = 2ull * (t0 - t[r]);
}

// ---------------------------------------------------------------------------
// Swap the x and y axes of a 1-bit lattice into Q: Q holds the lattice s' with
// s'(x', y', z) = s(y', x', z), in the same colour-separated layout (the
// colour x + y + z is unchanged), so the y-axis sums of Q are the x-axis sums
// of P and the x axis runs on the matrix cores too, with the row order of the
// y axis (rows of one z-plane, adjacent in memory).
//
// A block of 64 y by 64 x sites of one z-plane splits by the parities of y
// and x into four 32 x 32 bit matrices: with y = 2 yh + p and x = 2 xh + q,
// the word of the x-parity slot q in row y holds bits xh of M_pq[yh].  The
// word of Q's row y' = x, slot p (the parity of x' = y), holds bit yh of the
// transpose of M_pq.  A wave holds the 64 rows y of a block, one per lane,
// with p at lane bit 2 and the five bits of yh at lane bits 0, 1, 3, 4, 5,
// and transposes its two words (q = 0, 1) in five steps; step j exchanges
// with the lane that differs in the lane bit of yh's bit j (lane xor 1, 2, 8,
// 16, 32: quad permutes, a row rotation and the two lane-half swaps, all
// without LDS) and moves j x j bit blocks with a rotate and a bit select.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, int lx)
{
    if (lx == 1)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);  // quad [1,0,3,2]
    if (lx == 2)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);  // quad [2,3,0,1]
    if (lx == 8)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false); // row_ror:8
    // the swaps return this lane's own value in one result and the partner's
    // in the other (equal values make either choice right)
    if (lx == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return r[0] == v ? r[1] : r[0];
    }
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return r[0] == v ? r[1] : r[0];
}

// One transposition step on the 32-bit row v of this lane: bits k with
// (k & j) != 0 of the lane whose yh bit j is clear (a) trade places with bits
// k - j of its partner (b).  a keeps its bits in m and takes the partner's
// rotated left by j elsewhere; b keeps the bits outside m and takes the
// partner's rotated right by j in m.
template <int J, int LX>
__device__ __forceinline__ uint32_t transpose_step(uint32_t v, uint32_t lane)
{
    constexpr uint32_t m = J == 1 ? 0x55555555u : J == 2 ? 0x33333333u : J == 4 ? 0x0F0F0F0Fu
                         : J == 8 ? 0x00FF00FFu : 0x0000FFFFu;
    const uint32_t o = xor_lane(v, LX);
    const bool a = (lane & LX) == 0;
    const uint32_t t = __builtin_amdgcn_alignbit(o, o, a ? 32 - J : J);
    const uint32_t keep = a ? m : ~m;
    return (v & keep) | (t & ~keep);
}

__device__ __forceinline__ uint32_t transpose32(uint32_t v, uint32_t lane)
{
    v = transpose_step<1, 1>(v, lane);
    v = transpose_step<2, 2>(v, lane);
    v = transpose_step<4, 8>(v, lane);
    v = transpose_step<8, 16>(v, lane);
    return transpose_step<16, 32>(v, lane);
}

constexpr uint32_t kSwapIn = 520;      // words of a block in LDS: [slot][word][65 rows, padded]
constexpr uint32_t kSwapOut = 514;     // words per yb in LDS: [row pair][slot][row parity], padded

// Blocks yb held in LDS before they are written out: 16 (64-byte pieces of
// the output rows) where W allows, else all W of them.
__host__ __device__ inline uint32_t swap_span(uint32_t W) { return (W & 15u) == 0u ? 16u : W; }

// P16: W is a multiple of 16, so pieces are 16 blocks and a piece is
// complete after every kAhead = 8 pairs, at the same step of the unrolled
// pair loop.  With the stores at one place in the loop (and no early exit)
// each step waits only for its own oldest load; with a flush the compiler
// cannot place, every step waited for everything in flight.
template <bool P16>
__global__ void __launch_bounds__(256) k_bit_swap_xy(uint32_t L, uint32_t W, const uint32_t *P0,
                                                    const uint32_t *P1, uint32_t *Q0, uint32_t *Q1)
{
    // One workgroup of 256 threads per (z, group xg of four 64-column blocks,
    // one per wave): it builds the 256 rows (y' = x, z) of Q for x in
    // [256 xg, 256 xg + 256) in LDS, F blocks yb at a time, and writes out
    // each row's F words of those blocks (F = swap_span(W): with 64-byte
    // pieces the LDS of three workgroups fits a CU).
    extern __shared__ uint32_t sm[];
    const uint32_t F = P16 ? 16u : swap_span(W);
    uint32_t *out = sm;                   // [F blocks][128 row pairs][2 slots][2 rows]
    uint32_t *in = sm + kSwapOut * F;     // [2 buffers][2 blocks][kSwapIn]
    const uint32_t ngroups = W / 4;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);   // a z's groups share an XCD
    const uint32_t z = tile / ngroups, xg = tile % ngroups;
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    // Words 4 xg .. 4 xg + 3 of row (z, y) of one colour plane are one
    // 16-byte segment; block yb is the 128 segments of rows y = 64 yb + r,
    // both parity slots (slot 0 = even x).  Blocks come in pairs, one per half
    // of the workgroup (thread t: segment t & 127 of block 2 pp + t / 128),
    // and kAhead pairs are loaded ahead, so that many 16-byte loads per lane
    // are in flight.  The row y = 64 (2 pp + half) + sr has the parity of sr,
    // so a thread reads one colour plane, 128 rows further on per pair.
    const uint32_t seg = threadIdx.x & 127u, half = threadIdx.x >> 7;
    const uint32_t sr = seg >> 1, sslot = seg & 1u;
    const uint32_t c0 = sslot ^ ((z + sr) & 1u);   // colour holding the parity slot
    const uint32_t *seg0 = (c0 ? P1 : P0) + ((size_t)z * L + 64u * half + sr) * W + 4u * xg;
    const size_t pstride = (size_t)128u * W;
    auto fetch = [&](uint32_t pp) -> uint4 {
        return *reinterpret_cast<const uint4 *>(seg0 + pp * pstride);
    };
    // The pair loop is unrolled by kAhead, so that each prefetch buffer keeps
    // its registers: shifting the buffers down every pair made the compiler
    // wait for the load it had just issued before the copy.
    constexpr uint32_t kAhead = 8;
    const uint32_t npairs = W / 2;
    uint4 pre[kAhead];
    // issued in the order they are used, so that each wait below is for the
    // oldest loads only
#pragma unroll
    for (uint32_t a = 0; a < kAhead; ++a) {
        pre[a] = fetch(min(a, npairs - 1u));
        __builtin_amdgcn_sched_barrier(0);
    }
    // this lane's row of a block: y = 2 yh + p
    const uint32_t yh = (lane & 3u) | ((lane >> 3) << 2), p = (lane >> 2) & 1u;
    const uint32_t ry = 2u * yh + p;
    const uint32_t nq = F / 4;            // 16-byte quads of a row's piece
    for (uint32_t p0 = 0; p0 < npairs; p0 += kAhead)
#pragma unroll
    for (uint32_t a = 0; a < kAhead; ++a) {
        const uint32_t pp = p0 + a;
        if (!P16 && pp >= npairs)   // with P16, npairs is a multiple of kAhead
            break;
        // the pair's segments into this iteration's buffer; the other buffer
        // was last read before the previous barrier
        uint32_t *ib = in + (pp & 1u) * (2u * kSwapIn);
        {
            uint32_t *d = ib + half * kSwapIn + sslot * 4u * 65u + sr;
            d[0] = pre[a].x;
            d[65] = pre[a].y;
            d[130] = pre[a].z;
            d[195] = pre[a].w;
        }
        pre[a] = fetch(min(pp + kAhead, npairs - 1u));
        __syncthreads();
        const uint32_t yb0 = 2u * pp - (2u * pp) % F;      // first block of this piece
#pragma unroll
        for (uint32_t hb = 0; hb < 2; ++hb) {
            const uint32_t yl = 2u * pp + hb - yb0;
            const uint32_t *bb = ib + hb * kSwapIn;
            // wave wv: x block 4 xg + wv, word wv of each segment
            const uint32_t we = transpose32(bb[wv * 65u + ry], lane);          // q = 0
            const uint32_t wo = transpose32(bb[(4u + wv) * 65u + ry], lane);   // q = 1
            // rows y' = 64 wv + 2 yh + q of Q's group, slot p, word yb
            const uint32_t r2 = 32u * wv + yh;
            *reinterpret_cast<uint2 *>(out + yl * kSwapOut + r2 * 4u + p * 2u) = make_uint2(we, wo);
        }
        if (P16 ? a + 1 < kAhead : 2u * pp + 2u - yb0 < F)
            continue;
        // the piece is complete: rows y' = 256 xg + row, parity slot p' to
        // colour (p' + y' + z) & 1; item it: quad w4 of (row, slot)'s piece.
        // The next pair's LDS writes come after its barrier, so no thread
        // overwrites the piece before every thread has written it out.
        __syncthreads();
        for (uint32_t it = threadIdx.x; it < 512u * nq; it += blockDim.x) {
            const uint32_t rs = it / nq, w4 = it - rs * nq;
            const uint32_t row = rs >> 1, slot = rs & 1u;
            const uint32_t *src = out + (4u * w4) * kSwapOut + (row >> 1) * 4u + slot * 2u + (row & 1u);
            const uint4 v = make_uint4(src[0], src[kSwapOut], src[2u * kSwapOut], src[3u * kSwapOut]);
            const uint32_t yp = 256u * xg + row;
            const uint32_t c = slot ^ ((yp + z) & 1u);
            *reinterpret_cast<uint4 *>((c ? Q1 : Q0) + ((size_t)z * L + yp) * W + yb0 + 4u * w4) = v;
        }
    }
}

GramGeom gram_geom(uint32_t L, uint32_t NB)
{
    GramGeom g;
    g.L = L;
    g.W = L / 64;
    g.nT = L / kGramTile;
    g.CW = 32 * NB;
    g.ncb = L / g.CW;
    g.ntile = 0;
    for (uint32_t bi = 0; bi < g.nT; ++bi)
        g.ntile += g.ncb - kGramTile * bi / g.CW;
    g.NK = 2 * L * g.W;
    // at least two rounds of resident waves over the launch (1024 SIMDs,
    // 4 / NB waves each), chunks of at most 2048 words (all rows of a chunk:
    // 16 MiB at L = 2048, so the chunks in flight fit in the last-level
    // cache), at least 64 words, fewer than 2^24 lines per chunk (each float
    // accumulator then counts up-up pairs exactly in units of 0.25) and
    // per-wave diagonal sums below 2^32
    const uint32_t resident = 1024 * (4 / NB);   // waves in one round over the chip
    const uint32_t waves = 2 * resident;
    uint32_t nsplit = std::max((waves + g.ntile - 1) / g.ntile, (g.NK + 2047) / 2048);
    const uint32_t kmax = (1u << 19) - 8;   // 32 lines per word, 128 entries per diagonal
    auto chunk_of = [&](uint32_t ns) {
        uint32_t kc = ((g.NK + ns - 1) / ns + 7) / 8 * 8;
        return std::min(std::max(kc, 64u), kmax);
    };
    // among slightly fewer chunks (up to a quarter longer, 2560 words at
    // most), the count whose last round of waves is fullest: the launch takes
    // rounds x chunk length, plus a fixed cost per wave for its diagonals
    uint32_t best = nsplit;
    uint64_t best_cost = ~0ull;
    for (uint32_t ns = std::max(1u, nsplit - nsplit / 4); ns <= nsplit; ++ns) {
        const uint32_t kc = chunk_of(ns);
        if (kc > 2560 && ns != nsplit)
            continue;
        const uint32_t n = (g.NK + kc - 1) / kc;
        const uint64_t rounds = ((uint64_t)g.ntile * n + resident - 1) / resident;
        const uint64_t cost = rounds * (kc + 128);
        if (cost < best_cost) {
            best_cost = cost;
            best = ns;
        }
    }
    g.kchunk = chunk_of(best);
    g.nsplit = (g.NK + g.kchunk - 1) / g.kchunk;
    return g;
}

LineGeom line_geom(uint32_t L)
{
    LineGeom g;
    g.L = L;
    g.W = L / 64;
    g.R = L / 2 + 1;
    // separations per block: kG per register block, at most kItems items per
    // thread over the 2W columns, no more than the separations there are
    uint32_t ngr = (kItems * kBlock) / (2 * g.W);
    if (ngr < 1)
        ngr = 1;
    uint32_t Rr = ngr * kG;
    const uint32_t Rmax = ((g.R + kG - 1) / kG) * kG;
    if (Rr > Rmax)
        Rr = Rmax;
    uint32_t Cy = L < 64 ? L : 64;
    if (Rr > 64 && line_lds_bytes(g.W, Cy, Rr) > kLineLds)
        Rr = 64;
    while (line_lds_bytes(g.W, Cy, Rr) > kLineLds && Cy > kG) {
        Cy /= 2;
        Rr = Rr > kG ? Rr / 2 : Rr;
    }
    g.Cy = Cy;
    g.Rr = Rr;
    g.nrc = (g.R + Rr - 1) / Rr;
    return g;
}

}  // namespace

hipError_t bit_corr(hipStream_t st, uint32_t L, const uint32_t *P0, const uint32_t *P1,
                    unsigned long long *anti, unsigned long long *ones, uint32_t *Q0,
                    uint32_t *Q1)
{
    const uint32_t W = L / 64;
    const uint32_t R = L / 2 + 1;
    LineGeom g = line_geom(L);
    const uint32_t ntiles = L * (L / g.Cy);
    uint32_t nsplit = 8 * ((2048 / g.nrc + 7) / 8);
    if (nsplit < 8)
        nsplit = 8;
    while (nsplit > 8 && nsplit / 2 >= ntiles)
        nsplit /= 2;
    g.nsplit = nsplit;
    const size_t lds_lines = std::max<size_t>(line_lds_bytes(W, g.Cy, g.Rr), (size_t)g.Rr * 8);
    const dim3 grid_lines(g.nrc * nsplit);
    // y and z on the matrix cores where the row blocks and word quads fit
    // (L a multiple of 256), else by XOR and popcount
    const bool gram = L % 256 == 0;
    if (!gram) {
        hipLaunchKernelGGL(k_corr_lines<1>, grid_lines, dim3(kBlock), lds_lines, st, g, P0, P1,
                           anti + 1 * R);
        hipLaunchKernelGGL(k_corr_lines<2>, grid_lines, dim3(kBlock), lds_lines, st, g, P0, P1,
                           anti + 2 * R);
    }
    const bool gram_x = gram && Q0 != nullptr && Q1 != nullptr;
    if (!gram_x) {
        const uint32_t P = kBlock / W;
        const size_t lds_x = std::max<size_t>((size_t)P * 2 * W * 4, (size_t)(R + 1) * 8);
        const uint64_t nchunks = ((uint64_t)L * L + P - 1) / P;
        const uint32_t gx = (uint32_t)std::min<uint64_t>(nchunks, 2048);
        hipLaunchKernelGGL(k_corr_x, dim3(gx), dim3(kBlock), lds_x, st, L, W, P0, P1, anti, ones);
    }
    if (gram) {
        const GramGeom gg = gram_geom(L, kGramNB);
        // a multiple of 8 workgroups (whole XCD shares; the extra waves exit)
        const dim3 grid_gram(((gg.ntile * gg.nsplit + 3) / 4 + 7) / 8 * 8);
        if (gram_x) {
            // x: the y axis of the lattice with x and y swapped (into Q)
            const size_t lds = (size_t)(kSwapOut * swap_span(W) + 4 * kSwapIn) * 4;
            if ((W & 15u) == 0u)
                hipLaunchKernelGGL(k_bit_swap_xy<true>, dim3(L * (W / 4)), dim3(256), lds, st, L,
                                   W, P0, P1, Q0, Q1);
            else
                hipLaunchKernelGGL(k_bit_swap_xy<false>, dim3(L * (W / 4)), dim3(256), lds, st, L,
                                   W, P0, P1, Q0, Q1);
            hipLaunchKernelGGL((k_corr_gram<1, kGramNB>), grid_gram, dim3(256), 0, st, gg, Q0, Q1,
                               anti);
        }
        hipLaunchKernelGGL((k_corr_gram<1, kGramNB>), grid_gram, dim3(256), 0, st, gg, P0, P1,
                           anti + 1 * R);
        hipLaunchKernelGGL((k_corr_gram<2, kGramNB>), grid_gram, dim3(256), 0, st, gg, P0, P1,
                           anti + 2 * R);
        const uint32_t a0 = gram_x ? 0u : 1u;
        hipLaunchKernelGGL(k_corr_gram_finish, dim3(3 - a0), dim3(256), 0, st, anti, R, a0, ones);
    }
    return hipGetLastError();
}

}  // namespace qz
