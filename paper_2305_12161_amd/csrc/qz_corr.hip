// qz_corr.hip -- axis correlation sums of the 1-bit layout.
//
// S_a(r) = sum_i s_i s_{i + r e_a} = N - 2 * anti_a(r), where anti_a(r) counts
// the site pairs at separation r along axis a whose spins differ; the kernels
// accumulate anti_a(r) for r = 0..L/2 with XOR + popcount on 32 sites at a
// time (the integer pieces of C(r,t), Results, eq:correlation function).
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
                    unsigned long long *anti, unsigned long long *ones)
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
    hipLaunchKernelGGL(k_corr_lines<1>, grid_lines, dim3(kBlock), lds_lines, st, g, P0, P1,
                       anti + 1 * R);
    hipLaunchKernelGGL(k_corr_lines<2>, grid_lines, dim3(kBlock), lds_lines, st, g, P0, P1,
                       anti + 2 * R);
    const uint32_t P = kBlock / W;
    const size_t lds_x = std::max<size_t>((size_t)P * 2 * W * 4, (size_t)(R + 1) * 8);
    const uint64_t nchunks = ((uint64_t)L * L + P - 1) / P;
    const uint32_t gx = (uint32_t)std::min<uint64_t>(nchunks, 2048);
    hipLaunchKernelGGL(k_corr_x, dim3(gx), dim3(kBlock), lds_x, st, L, W, P0, P1, anti, ones);
    return hipGetLastError();
}

}  // namespace qz
