// qz_batch.hip -- one launch sweeps many independent 1-bit lattices (replicas).
//
// Each replica uses the colour-separated 1-bit layout of the single-lattice
// path (plane c = words [z][y][W], W = L/64) with two copies (read / write).
// A launch performs ONE sweep (colour 0 then colour 1, Methods "Checkerboard
// update") of every active replica, each at its own time t, so replicas of
// different L and different ages can share a launch.  The work is cut into
// sub-tiles: Tz consecutive planes (whole planes) of one replica.  A lane owns
// a quad -- 4 consecutive words of a plane, i.e. exactly one Philox block of
// tie bits -- so no lane draws bits it does not use, even when a row is only
// one or two words long.  A workgroup of 256 lanes runs 256/Q sub-tiles of one
// lattice size in lockstep (Q = quads per plane), streaming along z as the
// single-lattice kernel does: colour 0 of plane q, then colour 1 of plane q-1,
// with the other colour's plane exchanged through LDS.
#include "qz_device.hpp"
#include "qz_internal.hpp"

namespace qz {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// A value the caller knows to be the same in every active lane of the wave,
// read from the first one into a scalar register (so that the arithmetic on
// it runs on the scalar unit).
__device__ __forceinline__ uint32_t wave_u32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ uint64_t wave_u64(uint64_t v)
{
    return ((uint64_t)wave_u32((uint32_t)(v >> 32)) << 32) | wave_u32((uint32_t)v);
}
template <class T>
__device__ __forceinline__ T *wave_ptr(T *p)
{
    return reinterpret_cast<T *>(wave_u64(reinterpret_cast<uintptr_t>(p)));
}

// The body of one workgroup's sweep.  WK = words per colour row when the
// rows are 1, 2 or 4 words long (L = 64, 128, 256): a lane's quad then holds
// whole rows, so its x-neighbour words are its own and its y-neighbour words
// are its own or one vector read of the next lane's quad.  WK = 0: any L, with
// per-word neighbour indices.
template <int WK>
__device__ __forceinline__ void batch_body(const BatchArgs &A)
{
    extern __shared__ uint32_t lds[];
    const uint32_t tid = threadIdx.x;
    const BatchGroup G = A.groups[blockIdx.x];          // all sub-tiles of this block share L, nz
    const uint32_t L = WK ? 64u * WK : G.L;
    const uint32_t W = L / 64, PW = L * W;             // words per plane
    const uint32_t Q = PW / 4;                          // quads (lanes) per plane
    const uint32_t S = kBatchBlock / Q >= 1 ? kBatchBlock / Q : 1;
    const uint32_t sub = tid / Q, lane = tid % Q;
    const uint32_t nz = G.nz;

    // this lane's sub-tile
    bool act = false;
    BatchTile T = {0u, 0u};
    BatchReplica R;
    if (sub < S && G.first + sub < G.last) {
        T = A.tiles[G.first + sub];
        R = A.reps[T.slot];
        // a replica that has reached its t_max is skipped like a parked one
        act = R.active != 0u && (R.t_max == 0u || R.t + A.step < R.t_max);
    }
    uint64_t t64 = act ? R.t + A.step : 0;
    uint32_t rd = act ? ((R.cur ^ A.step) & 1u) : 0u;
    uint32_t k0 = act ? (uint32_t)R.seed : 0u, k1 = act ? (uint32_t)(R.seed >> 32) : 0u;
    uint32_t *base = act ? R.base : nullptr;
    unsigned long long *trace = act ? R.trace : nullptr;
    if constexpr (WK == 2 || WK == 4) {
        // Q is a multiple of 64 here, so a wave lies in one sub-tile: the
        // replica, its time and key and the first plane are the same in all
        // its lanes, and in scalar registers the Philox key schedule, the
        // plane steps and the plane addresses leave the vector unit
        act = wave_u32(act ? 1u : 0u) != 0u;
        t64 = wave_u64(t64);
        rd = wave_u32(rd);
        k0 = wave_u32(k0);
        k1 = wave_u32(k1);
        base = wave_ptr(base);
        trace = wave_ptr(trace);
        T.z0 = wave_u32(T.z0);
    }
    const uint32_t t = (uint32_t)t64;
    const size_t pw_all = (size_t)L * PW;                // words of one colour plane set
    const uint32_t *S0 = act ? base + (2 * rd + 0) * pw_all : nullptr;
    const uint32_t *S1 = act ? base + (2 * rd + 1) * pw_all : nullptr;
    uint32_t *D0 = act ? base + (2 * (1 - rd) + 0) * pw_all : nullptr;
    uint32_t *D1 = act ? base + (2 * (1 - rd) + 1) * pw_all : nullptr;
    const bool counting = act && A.every != 0u && trace != nullptr && (t64 % A.every) == 0u;

    // word geometry of this lane's quad within a plane
    const uint32_t g0 = 4 * lane;
    uint32_t yv[4], gym[4], gyp[4], gpr[4], gnx[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const uint32_t g = g0 + v, y = g / W, w = g % W;
        yv[v] = y;
        gym[v] = (g + PW - W) % PW;
        gyp[v] = (g + W) % PW;
        gpr[v] = (w == 0) ? g + W - 1 : g - 1;          // x-neighbour at colour index k-1
        gnx[v] = (w == W - 1) ? g + 1 - W : g + 1;      // x-neighbour at colour index k+1
    }
    // WK > 0: the quad is rows y0 .. y0 + 4/WK - 1; the words of row y0 - 1
    // start at lm, those of the row after the quad at lp
    const uint32_t y0 = g0 / W, rows = 4 / W;
    const uint32_t lm = ((y0 + L - 1) % L) * W, lp = ((y0 + rows) % L) * W;

    uint32_t *X1base = lds + (size_t)sub * 4 * PW;       // [2 buffers][X1 | X0][PW]
    uint32_t c1m[4], c1c[4], c1p[4], c0o[4], n0m2[4], n0m1[4], n0c[4], c1n[4], pf1[4], pf0[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
        c1m[v] = c1c[v] = c1p[v] = c0o[v] = n0m2[v] = n0m1[v] = n0c[v] = c1n[v] = pf1[v] = pf0[v] = 0u;
    // global-memory accesses spelled out: the replica pointers come from a
    // table, and flat accesses would also be waited for by every LDS wait
    auto ld4 = [&](const uint32_t *P, uint32_t z, uint32_t (&r)[4]) {
        const u32x4 q = *(const __attribute__((address_space(1))) u32x4 *)(P + (z * PW + g0));
        r[0] = q.x; r[1] = q.y; r[2] = q.z; r[3] = q.w;
    };
    auto st4 = [&](uint32_t *P, uint32_t z, const uint32_t (&r)[4]) {
        *(__attribute__((address_space(1))) u32x4 *)(P + (z * PW + g0)) = u32x4{r[0], r[1], r[2], r[3]};
    };
    const uint32_t z0 = T.z0;
    if (act) {
        ld4(S1, (z0 + L - 2) % L, c1m);
        ld4(S1, (z0 + L - 1) % L, c1c);
        ld4(S1, z0 % L, c1p);
        ld4(S0, (z0 + L - 1) % L, c0o);
    }
    int bonds = 0;

    // one colour update of the lane's quad; Xo = other colour's plane in LDS,
    // same = the lane's own words of that plane, zm/zp = planes below/above
    // r = the quad's tie words (one Philox block), drawn beforehand
    auto update = [&](const uint32_t *Xo, const uint32_t (&own)[4], const uint32_t (&same)[4],
                      const uint32_t (&zmn)[4], const uint32_t (&zpn)[4], uint32_t zp_plane,
                      uint32_t colour, const uint32_t (&r)[4], uint32_t (&out)[4], bool count) {
        // the two neighbour triples: (same, shifted, y-1) and (y+1, z-1, z+1)
        uint32_t n0[4], n1[4], n2[4];
        if constexpr (WK == 4) {
            const uint4 m = *reinterpret_cast<const uint4 *>(Xo + lm);
            const uint4 q = *reinterpret_cast<const uint4 *>(Xo + lp);
            n1[0] = m.x; n1[1] = m.y; n1[2] = m.z; n1[3] = m.w;
            n2[0] = q.x; n2[1] = q.y; n2[2] = q.z; n2[3] = q.w;
        } else if constexpr (WK == 2) {
            const uint2 m = *reinterpret_cast<const uint2 *>(Xo + lm);
            const uint2 q = *reinterpret_cast<const uint2 *>(Xo + lp);
            n1[0] = m.x; n1[1] = m.y; n1[2] = same[0]; n1[3] = same[1];
            n2[0] = same[2]; n2[1] = same[3]; n2[2] = q.x; n2[3] = q.y;
        } else if constexpr (WK == 1) {
            n1[0] = Xo[lm]; n1[1] = same[0]; n1[2] = same[1]; n1[3] = same[2];
            n2[0] = same[1]; n2[1] = same[2]; n2[2] = same[3]; n2[3] = Xo[lp];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            // pi differs between the lanes of a wave (and between the words of
            // a lane where rows are shorter than four words): select the
            // funnel's operands rather than branch on it
            const uint32_t pi = (colour + yv[v] + zp_plane) & 1u;
            if constexpr (WK == 4) {
                // both shifts from the lane's own words, then one select
                const uint32_t up = funnel(same[(v + 1) & 3], same[v], 1);
                const uint32_t dn = funnel(same[v], same[(v + 3) & 3], 31);
                n0[v] = pi ? up : dn;
            } else if constexpr (WK == 2 || WK == 1) {
                const uint32_t adj = WK == 2 ? same[v ^ 1] : same[v];
                n0[v] = funnel(pi ? adj : same[v], pi ? same[v] : adj, pi ? 1u : 31u);
            } else {
                const uint32_t adj = Xo[pi ? gnx[v] : gpr[v]];
                n0[v] = funnel(pi ? adj : same[v], pi ? same[v] : adj, pi ? 1u : 31u);
            }
            if constexpr (WK == 0) {
                n1[v] = Xo[gym[v]];
                n2[v] = Xo[gyp[v]];
            }
        }
        // majority of seven (the neighbours and s ^ r), as in the lattice
        // kernels; counting adds a = (xa ^ s) + (xb ^ s) + 2 ((ma ^ s) + (mb ^ s))
        uint32_t xa[4], ma[4], xb[4], mb[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            xa[v] = xor3(same[v], n0[v], n1[v]);
            ma[v] = maj3(same[v], n0[v], n1[v]);
            xb[v] = xor3(n2[v], zmn[v], zpn[v]);
            mb[v] = maj3(n2[v], zmn[v], zpn[v]);
            out[v] = maj3(ma[v], mb[v], maj3(xa[v], xb[v], own[v] ^ r[v]));
        }
        if (count) {
            uint32_t ones = 0, twos = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                ones = popc_acc(xa[v] ^ own[v], popc_acc(xb[v] ^ own[v], ones));
                twos = popc_acc(ma[v] ^ own[v], popc_acc(mb[v] ^ own[v], twos));
            }
            bonds += (int)(ones + 2u * twos);
        }
    };
    // The tie words depend only on the sites and the time, so each step's are
    // drawn one step ahead (unconditionally), off the chain from the colour-0
    // update to the colour-1 update.  Philox block = word index / 4.
    auto draw = [&](uint32_t z, uint32_t colour, uint32_t (&r)[4]) {
        const Words4 rb = philox10((z * PW + g0) >> 2, t, colour, 0u, k0, k1);
#pragma unroll
        for (int v = 0; v < 4; ++v)
            r[v] = rb.w[v];
    };
    // Step qi updates colour 0 of plane zq for qi = -1 .. nz and colour 1 of
    // plane zm for qi = 1 .. nz; a step's words are drawn only where its
    // update runs (the draw for step qi + 1 is made at step qi).
    uint32_t s0[4] = {0u, 0u, 0u, 0u}, s1[4] = {0u, 0u, 0u, 0u};   // next step's tie words
    if (act)
        draw((z0 + L - 1) % L, 0u, s0);

    // the step's plane zq and its neighbours, advanced with one wrap test per
    // step instead of divisions by L
    uint32_t zq = (z0 + L - 1) % L;
    uint32_t zm = (zq + L - 1) % L, z1 = (zq + 1) % L, z2 = (zq + 2) % L;
    for (int qi = -1; qi <= (int)nz; ++qi) {
        if (act && qi < (int)nz) {
            ld4(S1, z2, pf1);
            ld4(S0, z1, pf0);
        }
        uint32_t *X1 = X1base + (size_t)(qi & 1) * 2 * PW;
        uint32_t *X0 = X1 + PW;
        if (act) {
            *reinterpret_cast<uint4 *>(X1 + g0) = make_uint4(c1c[0], c1c[1], c1c[2], c1c[3]);
            *reinterpret_cast<uint4 *>(X0 + g0) = make_uint4(n0m1[0], n0m1[1], n0m1[2], n0m1[3]);
        }
        uint32_t r0[4], r1[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            r0[v] = s0[v];
            r1[v] = s1[v];
        }
        if (act && qi < (int)nz) {
            draw(z1, 0u, s0);
            if (qi >= 0)
                draw(zq, 1u, s1);
        }
        __syncthreads();
        if (act) {
            const bool mine = qi >= 0 && qi < (int)nz;
            update(X1, c0o, c1c, c1m, c1p, zq, 0u, r0, n0c, counting && mine);
            if (mine)
                st4(D0, zq, n0c);
            if (qi >= 1) {
                update(X0, c1m, n0m1, n0m2, n0c, zm, 1u, r1, c1n, false);
                st4(D1, zm, c1n);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                c1m[v] = c1c[v];
                c1c[v] = c1p[v];
                c1p[v] = pf1[v];
                c0o[v] = pf0[v];
                n0m2[v] = n0m1[v];
                n0m1[v] = n0c[v];
            }
        }
        zm = zq;
        zq = z1;
        z1 = z2;
        z2 = (z2 + 1u == L) ? 0u : z2 + 1u;
    }
    // per-sub-tile bond sums -> the replica's trace slot
    __syncthreads();
    uint32_t *sacc = lds;                                 // S counters
    if (tid < S)
        sacc[tid] = 0u;
    __syncthreads();
    if (counting && bonds)
        atomicAdd(sacc + sub, (uint32_t)bonds);
    __syncthreads();
    if (counting && lane == 0 && sacc[sub]) {
        const uint32_t slot = (uint32_t)((t64 / A.every) % A.cap);
        atomicAdd(trace + slot, (unsigned long long)sacc[sub]);
    }
}

__global__ void __launch_bounds__(kBatchBlock) k_batch_sweep(BatchArgs A)
{
    switch (A.groups[blockIdx.x].L) {
    case 64: batch_body<1>(A); break;
    case 128: batch_body<2>(A); break;
    case 256: batch_body<4>(A); break;
    default: batch_body<0>(A); break;
    }
}

// Sweeps of a group of k that replica r runs: all k, or those left before
// its t_max.
__device__ __forceinline__ uint32_t batch_steps(const BatchReplica &r, uint32_t k)
{
    if (!r.active)
        return 0u;
    if (r.t_max == 0u)
        return k;
    return r.t >= r.t_max ? 0u : (uint32_t)min((uint64_t)k, r.t_max - r.t);
}

// After a group of k sweeps: every active replica's time advances by the
// sweeps it ran and its current copy flips as often.
__global__ void k_batch_advance(BatchReplica *reps, uint32_t n, uint32_t k)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const uint32_t m = batch_steps(reps[i], k);
        reps[i].t += m;
        reps[i].cur ^= (m & 1u);
    }
}

// ---------------------------------------------------------------------------
// Replicas of side 64 entirely on chip.  Both colour planes of one replica
// (2 x 4096 words, 32 KiB) fit in the LDS of a workgroup, so one workgroup
// runs all k sweeps of a group for its replica without leaving the chip: per
// half-sweep every lane updates two quads of colour p in place from the other
// colour (a colour-p update reads only colour 1 - p, so no site is read after
// another lane wrote it), and a barrier separates the half-sweeps.  There are
// no halo planes and no launch per sweep; the lattice is read from and
// written back to the replica's buffer once per group.  Word g = 64 z + y of a
// plane holds row (y, z) (one word per colour row at L = 64), so a quad is
// four consecutive rows of one plane and one Philox block of tie bits.
// ---------------------------------------------------------------------------
constexpr uint32_t kOnchipBlock = 512;
constexpr uint32_t kOnchipWords = 4096;     // words of one colour plane set at L = 64

__global__ void __launch_bounds__(kOnchipBlock)
    k_batch_onchip64(const BatchReplica *reps, const uint32_t *slots, uint32_t k, uint32_t every,
                     uint32_t cap)
{
    __shared__ u32x4 planes[2 * kOnchipWords / 4];
    __shared__ unsigned long long part[kOnchipBlock / 64];
    uint32_t *P = reinterpret_cast<uint32_t *>(planes);
    const uint32_t tid = threadIdx.x;
    const BatchReplica R = reps[slots[blockIdx.x]];
    const uint32_t m = batch_steps(R, k);          // the same in every lane
    if (m == 0u)
        return;
    const uint32_t *src = R.base + (size_t)(2u * R.cur) * kOnchipWords;
    for (uint32_t i = tid; i < 2u * kOnchipWords / 4; i += kOnchipBlock)
        planes[i] = *(const __attribute__((address_space(1))) u32x4 *)(src + 4u * i);
    __syncthreads();
    const uint32_t k0 = (uint32_t)R.seed, k1 = (uint32_t)(R.seed >> 32);
    for (uint32_t s = 0; s < m; ++s) {
        const uint64_t t64 = R.t + s;
        const uint32_t t = (uint32_t)t64;
        const bool counting = every != 0u && R.trace != nullptr && (t64 % every) == 0u;
        int bonds = 0;
        for (uint32_t p = 0; p < 2u; ++p) {
            const uint32_t *O = P + (1u - p) * kOnchipWords;
            uint32_t *Q = P + p * kOnchipWords;
#pragma unroll
            for (uint32_t h = 0; h < 2u; ++h) {
                const uint32_t qd = tid + kOnchipBlock * h;      // quad: words 4 qd .. 4 qd + 3
                const uint32_t g0 = 4u * qd, z = g0 >> 6, y0 = g0 & 63u;
                const uint32_t zmo = ((z + 63u) & 63u) << 6, zpo = ((z + 1u) & 63u) << 6;
                const u32x4 so = *reinterpret_cast<const u32x4 *>(O + g0);
                const u32x4 sm = *reinterpret_cast<const u32x4 *>(O + zmo + y0);
                const u32x4 sp = *reinterpret_cast<const u32x4 *>(O + zpo + y0);
                const u32x4 ow = *reinterpret_cast<const u32x4 *>(Q + g0);
                const uint32_t below = O[(z << 6) + ((y0 + 63u) & 63u)];
                const uint32_t above = O[(z << 6) + ((y0 + 4u) & 63u)];
                const uint32_t same[4] = {so.x, so.y, so.z, so.w};
                const uint32_t zmn[4] = {sm.x, sm.y, sm.z, sm.w};
                const uint32_t zpn[4] = {sp.x, sp.y, sp.z, sp.w};
                const uint32_t own[4] = {ow.x, ow.y, ow.z, ow.w};
                const uint32_t ym[4] = {below, same[0], same[1], same[2]};
                const uint32_t yp[4] = {same[1], same[2], same[3], above};
                uint32_t xa[4], ma[4], xb[4], mb[4], ties = 0u;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    // the x neighbours: the same word and its rotation by one
                    // site, towards lower or higher x by the row's parity
                    const uint32_t pi = (p + y0 + (uint32_t)v + z) & 1u;
                    const uint32_t sh = pi ? funnel(same[v], same[v], 1) : funnel(same[v], same[v], 31);
                    xa[v] = xor3(same[v], sh, ym[v]);
                    ma[v] = maj3(same[v], sh, ym[v]);
                    xb[v] = xor3(yp[v], zmn[v], zpn[v]);
                    mb[v] = maj3(yp[v], zmn[v], zpn[v]);
                    ties |= (xa[v] ^ xb[v]) & (ma[v] ^ mb[v]);
                }
                uint32_t r[4] = {0u, 0u, 0u, 0u};
                if (ties != 0u) {
                    const Words4 rb = philox10(qd, t, p, 0u, k0, k1);
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        r[v] = rb.w[v];
                }
                uint32_t out[4];
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    out[v] = maj3(ma[v], mb[v], maj3(xa[v], xb[v], own[v] ^ r[v]));
                *reinterpret_cast<u32x4 *>(Q + g0) = u32x4{out[0], out[1], out[2], out[3]};
                if (counting && p == 0u) {
                    uint32_t ones = 0, twos = 0;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        ones = popc_acc(xa[v] ^ own[v], popc_acc(xb[v] ^ own[v], ones));
                        twos = popc_acc(ma[v] ^ own[v], popc_acc(mb[v] ^ own[v], twos));
                    }
                    bonds += (int)(ones + 2u * twos);
                }
            }
            __syncthreads();
        }
        if (counting) {
            // the replica's bond count entering sweep t: one workgroup owns
            // the replica, so its ring entry is written, not accumulated
            const unsigned long long w = wave_sum_u64((unsigned long long)bonds);
            if ((tid & 63u) == 0u)
                part[tid >> 6] = w;
            __syncthreads();
            if (tid == 0u) {
                unsigned long long tot = 0;
                for (uint32_t i = 0; i < kOnchipBlock / 64; ++i)
                    tot += part[i];
                R.trace[(t64 / every) % cap] = tot;
            }
            __syncthreads();
        }
    }
    uint32_t *dst = R.base + (size_t)(2u * ((R.cur ^ m) & 1u)) * kOnchipWords;
    for (uint32_t i = tid; i < 2u * kOnchipWords / 4; i += kOnchipBlock)
        *(__attribute__((address_space(1))) u32x4 *)(dst + 4u * i) = planes[i];
}

// Zero trace slots of active replicas for times [t0, t0 + span) before they
// are accumulated (launched as a kernel so that it can sit inside a graph).
__global__ void k_batch_clear_trace(BatchReplica *reps, uint32_t n, uint32_t span, uint32_t every,
                                    uint32_t cap)
{
    const uint32_t i = blockIdx.x;
    if (i >= n || reps[i].trace == nullptr)
        return;
    const uint64_t t0 = reps[i].t;
    const uint32_t m = batch_steps(reps[i], span);
    for (uint32_t d = threadIdx.x; d < m; d += blockDim.x) {
        const uint64_t t = t0 + d;
        if (t % every == 0u)
            reps[i].trace[(t / every) % cap] = 0ull;
    }
}

}  // namespace

hipError_t batch_sweep(hipStream_t st, const BatchArgs &a, uint32_t ngroups)
{
    if (ngroups == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_batch_sweep, dim3(ngroups), dim3(kBatchBlock), a.lds_bytes, st, a);
    return hipGetLastError();
}

hipError_t batch_onchip64(hipStream_t st, const BatchReplica *reps, const uint32_t *slots,
                          uint32_t nslots, uint32_t k, uint32_t every, uint32_t cap)
{
    if (nslots == 0 || k == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_batch_onchip64, dim3(nslots), dim3(kOnchipBlock), 0, st, reps, slots, k,
                       every, cap);
    return hipGetLastError();
}

hipError_t batch_advance(hipStream_t st, BatchReplica *reps, uint32_t n, uint32_t k)
{
    hipLaunchKernelGGL(k_batch_advance, dim3((n + 255) / 256), dim3(256), 0, st, reps, n, k);
    return hipGetLastError();
}

hipError_t batch_clear_trace(hipStream_t st, BatchReplica *reps, uint32_t n, uint32_t span,
                             uint32_t every, uint32_t cap)
{
    if (n == 0 || every == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_batch_clear_trace, dim3(n), dim3(64), 0, st, reps, n, span, every, cap);
    return hipGetLastError();
}

}  // namespace qz
