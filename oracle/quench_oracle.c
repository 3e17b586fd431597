/*
 * quench_oracle.c -- plain CPU oracle for the zero-temperature checkerboard
 * quench of the d=3 nearest-neighbour Ising model (Gessert, Christiansen,
 * Janke, "Superdiffusion-like behavior in zero-temperature coarsening of the
 * d=3 Ising model", arXiv:2305.12161).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library) never calls it, links it or shares code with it.
 *
 * Everything here is the plain definition, written out with int8 spins
 * (+1/-1), scalar triple loops and 64-bit integer sums.  The only concession
 * to speed is an OpenMP "parallel for" over z, which is valid because sites of
 * one checkerboard colour never interact (Methods, "Checkerboard update") and
 * every sum is an integer sum.
 *
 * Conventions (shared with the product only through this written contract):
 *   lattice index   i = x + L*(y + L*z), x fastest, periodic in all axes
 *   colour          c = (x + y + z) mod 2      (colour 0 = "red", updated first)
 *   colour index    j = floor(x/2) + (L/2)*(y + L*z), unique within a colour
 *   random bits     Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *                   key = (seed mod 2^32, seed >> 32),
 *                   dynamics counter (floor(j/128), t, p, 0),
 *                   initial-state counter (floor(i/128), 0, 0, 1),
 *                   bit of index k = (w[(k>>5)&3] >> (k&31)) & 1.
 *   The paper names no generator; this keying is our own definition.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (SC'11, "Parallel random     */
/* numbers: as easy as 1, 2, 3"): ten rounds of two 32x32->64 multiplies,    */
/* the key advanced by the two Weyl constants between rounds.                */
/* ------------------------------------------------------------------------ */
#define OR_PHILOX_M0 0xD2511F53u
#define OR_PHILOX_M1 0xCD9E8D57u
#define OR_PHILOX_W0 0x9E3779B9u
#define OR_PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t r0 = ctr[0], r1 = ctr[1], r2 = ctr[2], r3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += OR_PHILOX_W0;
            k1 += OR_PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)OR_PHILOX_M0 * (uint64_t)r0;
        uint64_t p1 = (uint64_t)OR_PHILOX_M1 * (uint64_t)r2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ r1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ r3 ^ k1;
        uint32_t n3 = lo0;
        r0 = n0; r1 = n1; r2 = n2; r3 = n3;
    }
    out[0] = r0; out[1] = r1; out[2] = r2; out[3] = r3;
}

/* Bit k of the 128-bit block addressed by (floor(k/128), c1, c2, c3). */
static int or_bit_of(uint64_t seed, uint64_t k, uint32_t c1, uint32_t c2, uint32_t c3)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { (uint32_t)(k >> 7), c1, c2, c3 };
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    return (int)((w[(k >> 5) & 3] >> (k & 31)) & 1u);
}

/* Tie bit for colour index j during half-sweep p of sweep t (0-based). */
int or_tie_bit(uint64_t seed, uint32_t t, int p, uint64_t j)
{
    return or_bit_of(seed, j, t, (uint32_t)p, 0u);
}

/* Initial-state bit for lattice index i. */
int or_init_bit(uint64_t seed, uint64_t i)
{
    return or_bit_of(seed, i, 0u, 0u, 1u);
}

/* ------------------------------------------------------------------------ */
/* Lattice helpers.                                                          */
/* ------------------------------------------------------------------------ */
static inline int64_t or_idx(int L, int x, int y, int z)
{
    return (int64_t)x + (int64_t)L * ((int64_t)y + (int64_t)L * (int64_t)z);
}

static inline int or_wrap(int v, int L)
{
    return v < 0 ? v + L : (v >= L ? v - L : v);
}

/* Number of the six nearest neighbours whose spin differs from site (x,y,z). */
static int or_antialigned(int L, const int8_t *s, int x, int y, int z)
{
    int8_t me = s[or_idx(L, x, y, z)];
    int a = 0;
    a += s[or_idx(L, or_wrap(x + 1, L), y, z)] != me;
    a += s[or_idx(L, or_wrap(x - 1, L), y, z)] != me;
    a += s[or_idx(L, x, or_wrap(y + 1, L), z)] != me;
    a += s[or_idx(L, x, or_wrap(y - 1, L), z)] != me;
    a += s[or_idx(L, x, y, or_wrap(z + 1, L))] != me;
    a += s[or_idx(L, x, y, or_wrap(z - 1, L))] != me;
    return a;
}

/* ------------------------------------------------------------------------ */
/* Initial state: infinite-temperature start, each spin an independent fair  */
/* coin (Results: random configurations with m close to 0).                  */
/* ------------------------------------------------------------------------ */
void or_init(int L, uint64_t seed, int8_t *s)
{
    int64_t N = (int64_t)L * L * L;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i)
        s[i] = or_init_bit(seed, (uint64_t)i) ? (int8_t)1 : (int8_t)-1;
}

/* The same start restricted to a W^3 window with global corner (ox, oy, oz),
 * taken periodically; w is indexed like a lattice of side W. */
void or_init_window(int L, uint64_t seed, int ox, int oy, int oz, int W, int8_t *w)
{
#pragma omp parallel for schedule(static)
    for (int lz = 0; lz < W; ++lz)
        for (int ly = 0; ly < W; ++ly)
            for (int lx = 0; lx < W; ++lx) {
                int gx = (ox + lx) % L, gy = (oy + ly) % L, gz = (oz + lz) % L;
                w[or_idx(W, lx, ly, lz)] =
                    or_init_bit(seed, (uint64_t)or_idx(L, gx, gy, gz)) ? (int8_t)1 : (int8_t)-1;
            }
}

/* ------------------------------------------------------------------------ */
/* One half-sweep over colour p (Methods, "Checkerboard update"), each       */
/* proposal accepted by the T -> 0 limit of the Glauber probability          */
/* (Methods, equation equ:glauberAcceptance):                                */
/*   dE = 2 s_i h_i = 12 - 4a, a = number of anti-aligned neighbours, so     */
/*   dE < 0  <=> a >= 4  -> flip;                                            */
/*   dE = 0  <=> a == 3  -> flip iff the tie bit is 1 (probability 1/2);     */
/*   dE > 0  <=> a <= 2  -> keep.                                            */
/* Colour-p sites read only colour 1-p, so updating in place in any order     */
/* equals the concurrent update.  Returns the number of flips.               */
/* ------------------------------------------------------------------------ */
int64_t or_half_sweep(int L, uint64_t seed, uint32_t t, int p, int8_t *s)
{
    int64_t flips = 0;
#pragma omp parallel for schedule(static) reduction(+ : flips)
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                if (((x + y + z) & 1) != p)
                    continue;
                int a = or_antialigned(L, s, x, y, z);
                int flip = 0;
                if (a >= 4) {
                    flip = 1;
                } else if (a == 3) {
                    uint64_t j = (uint64_t)(x / 2) +
                                 (uint64_t)(L / 2) * ((uint64_t)y + (uint64_t)L * (uint64_t)z);
                    flip = or_tie_bit(seed, t, p, j);
                }
                if (flip) {
                    int64_t i = or_idx(L, x, y, z);
                    s[i] = (int8_t)-s[i];
                    ++flips;
                }
            }
    return flips;
}

/* One Monte Carlo sweep (N proposals, Methods "Random-site-flip update"):   */
/* colour 0 then colour 1, the same order every sweep (the "01 cycle" of     */
/* Supplementary Methods I B).  t is the 0-based index of this sweep.        */
int64_t or_sweep(int L, uint64_t seed, uint32_t t, int8_t *s)
{
    int64_t f = or_half_sweep(L, seed, t, 0, s);
    f += or_half_sweep(L, seed, t, 1, s);
    return f;
}

/* ------------------------------------------------------------------------ */
/* Mixed cycle (Supplementary Methods I B): which sublattice goes first is   */
/* drawn at random for every sweep, independently of the others.  Our draw:  */
/* colour 1 goes first in sweep t iff bit 0 of word 0 of the Philox block    */
/* with counter (0, t, 2, 0) is set.                                         */
/* ------------------------------------------------------------------------ */
int or_first_colour(uint64_t seed, uint32_t t)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { 0u, t, 2u, 0u };
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    return (int)(w[0] & 1u);
}

int64_t or_sweep_mixed(int L, uint64_t seed, uint32_t t, int8_t *s)
{
    int first = or_first_colour(seed, t);
    int64_t f = or_half_sweep(L, seed, t, first, s);
    f += or_half_sweep(L, seed, t, 1 - first, s);
    return f;
}

/* ------------------------------------------------------------------------ */
/* Double checkerboard (Supplementary Methods I A): cubes of side B form a    */
/* coarse checkerboard, coarse colour cc = (x/B + y/B + z/B) mod 2; a sweep   */
/* updates the coarse-colour-0 cubes (fine colour 0 sites, then fine colour   */
/* 1 sites), then the coarse-colour-1 cubes the same way.  Sites of one       */
/* (coarse, fine) pair never touch, so each phase updates in place.  The tie  */
/* bit of a site is the one of the plain checkerboard (same j, t, fine        */
/* colour p).  Needs L % (2B) == 0.                                           */
/* ------------------------------------------------------------------------ */
static int64_t or_phase(int L, int B, uint64_t seed, uint32_t t, int cc, int p, int8_t *s)
{
    int64_t flips = 0;
#pragma omp parallel for schedule(static) reduction(+ : flips)
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                if (((x + y + z) & 1) != p || ((x / B + y / B + z / B) & 1) != cc)
                    continue;
                int a = or_antialigned(L, s, x, y, z);
                int flip = 0;
                if (a >= 4) {
                    flip = 1;
                } else if (a == 3) {
                    uint64_t j = (uint64_t)(x / 2) +
                                 (uint64_t)(L / 2) * ((uint64_t)y + (uint64_t)L * (uint64_t)z);
                    flip = or_tie_bit(seed, t, p, j);
                }
                if (flip) {
                    int64_t i = or_idx(L, x, y, z);
                    s[i] = (int8_t)-s[i];
                    ++flips;
                }
            }
    return flips;
}

int64_t or_sweep_double(int L, int B, uint64_t seed, uint32_t t, int8_t *s)
{
    int64_t f = 0;
    for (int cc = 0; cc < 2; ++cc)
        for (int p = 0; p < 2; ++p)
            f += or_phase(L, B, seed, t, cc, p, s);
    return f;
}

/* ------------------------------------------------------------------------ */
/* Mixed cycle of the double checkerboard (Supplementary Methods I B): once   */
/* per sweep the coarse colour updated first is drawn, and, independently,    */
/* each coarse cube draws which fine colour it updates first.  Our draws:     */
/*   coarse order: coarse colour 1 first iff bit 0 of word 0 of the block     */
/*                 (0, t, 3, 0);                                              */
/*   fine order of cube b = bx + nb*(by + nb*bz), nb = L/B, (bx, by, bz) =    */
/*                 (x/B, y/B, z/B): fine colour 1 first iff bit b of the      */
/*                 blocks (floor(b/128), t, 4, 0), extracted as the tie bits. */
/* A sweep: for the two coarse colours in the drawn order, two steps; in      */
/* step k every cube of that coarse colour updates its fine colour            */
/* (first ^ k).  Cubes of one coarse colour never touch, so a step updates    */
/* in place.  Tie bits are those of the plain checkerboard (j, t, fine p).    */
/* ------------------------------------------------------------------------ */
int or_coarse_first(uint64_t seed, uint32_t t)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { 0u, t, 3u, 0u };
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    return (int)(w[0] & 1u);
}

int or_fine_first(uint64_t seed, uint32_t t, uint64_t b)
{
    return or_bit_of(seed, b, t, 4u, 0u);
}

static int64_t or_step_mixed(int L, int B, uint64_t seed, uint32_t t, int cc, int k,
                             const uint8_t *first, int8_t *s)
{
    const int nb = L / B;
    int64_t flips = 0;
#pragma omp parallel for schedule(static) reduction(+ : flips)
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                if (((x / B + y / B + z / B) & 1) != cc)
                    continue;
                int64_t b = (int64_t)(x / B) + (int64_t)nb * ((int64_t)(y / B) + (int64_t)nb * (z / B));
                int p = (x + y + z) & 1;
                if (p != (first[b] ^ k))
                    continue;
                int a = or_antialigned(L, s, x, y, z);
                int flip = 0;
                if (a >= 4) {
                    flip = 1;
                } else if (a == 3) {
                    uint64_t j = (uint64_t)(x / 2) +
                                 (uint64_t)(L / 2) * ((uint64_t)y + (uint64_t)L * (uint64_t)z);
                    flip = or_tie_bit(seed, t, p, j);
                }
                if (flip) {
                    int64_t i = or_idx(L, x, y, z);
                    s[i] = (int8_t)-s[i];
                    ++flips;
                }
            }
    return flips;
}

/* Returns the number of flips, or -1 if the order table cannot be allocated. */
int64_t or_sweep_double_mixed(int L, int B, uint64_t seed, uint32_t t, int8_t *s)
{
    const int64_t nb = L / B, ncubes = nb * nb * nb;
    uint8_t *first = (uint8_t *)malloc((size_t)ncubes);
    if (!first)
        return -1;
    for (int64_t b = 0; b < ncubes; ++b)
        first[b] = (uint8_t)or_fine_first(seed, t, (uint64_t)b);
    const int c0 = or_coarse_first(seed, t);
    int64_t f = 0;
    for (int m = 0; m < 2; ++m)
        for (int k = 0; k < 2; ++k)
            f += or_step_mixed(L, B, seed, t, c0 ^ m, k, first, s);
    free(first);
    return f;
}

/* ------------------------------------------------------------------------ */
/* Unsatisfied-bond counts per axis: B_a = #{i : s_i != s_{i+e_a}}.          */
/* Energy E = -(3N - 2B), B = B_x + B_y + B_z.                               */
/* ------------------------------------------------------------------------ */
void or_bonds(int L, const int8_t *s, int64_t B[3])
{
    int64_t bx = 0, by = 0, bz = 0;
#pragma omp parallel for schedule(static) reduction(+ : bx, by, bz)
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                int8_t me = s[or_idx(L, x, y, z)];
                bx += s[or_idx(L, or_wrap(x + 1, L), y, z)] != me;
                by += s[or_idx(L, x, or_wrap(y + 1, L), z)] != me;
                bz += s[or_idx(L, x, y, or_wrap(z + 1, L))] != me;
            }
    B[0] = bx; B[1] = by; B[2] = bz;
}

/* ------------------------------------------------------------------------ */
/* Axis correlation sums S_a(r) = sum_i s_i s_{i + r e_a}, r = 0..L/2, and   */
/* the magnetisation M = sum_i s_i.  These are the integer pieces of the      */
/* two-point function C(r,t) = <s_i s_j> - <s_i><s_j> (Results, equation     */
/* eq:correlation function) restricted to separations along the axes.        */
/* Output S is laid out [axis][r], axis 0 = x, 1 = y, 2 = z.                 */
/* ------------------------------------------------------------------------ */
void or_corr(int L, const int8_t *s, int64_t *S, int64_t *M)
{
    int R = L / 2 + 1;
    for (int a = 0; a < 3; ++a)
        for (int r = 0; r < R; ++r) {
            int64_t acc = 0;
#pragma omp parallel for schedule(static) reduction(+ : acc)
            for (int z = 0; z < L; ++z)
                for (int y = 0; y < L; ++y)
                    for (int x = 0; x < L; ++x) {
                        int xs = x, ys = y, zs = z;
                        if (a == 0) xs = (x + r) % L;
                        if (a == 1) ys = (y + r) % L;
                        if (a == 2) zs = (z + r) % L;
                        acc += (int64_t)s[or_idx(L, x, y, z)] * (int64_t)s[or_idx(L, xs, ys, zs)];
                    }
            S[a * R + r] = acc;
        }
    int64_t m = 0;
    int64_t N = (int64_t)L * L * L;
#pragma omp parallel for schedule(static) reduction(+ : m)
    for (int64_t i = 0; i < N; ++i)
        m += s[i];
    *M = m;
}

/* ------------------------------------------------------------------------ */
/* A run of n sweeps starting at time t0.  If every > 0, trace receives      */
/* B(t0 + k*every) for k = 0 .. n/every - 1, each the total bond count of    */
/* the state at the start of that sweep.  mixed != 0 selects the mixed      */
/* cycle, else the 01 cycle.                                                 */
/* ------------------------------------------------------------------------ */
void or_run_cycle(int L, uint64_t seed, int8_t *s, uint64_t t0, uint64_t n, uint64_t every,
                  int64_t *trace, int mixed)
{
    for (uint64_t k = 0; k < n; ++k) {
        if (every > 0 && trace != NULL && (k % every) == 0) {
            int64_t B[3];
            or_bonds(L, s, B);
            trace[k / every] = B[0] + B[1] + B[2];
        }
        if (mixed)
            or_sweep_mixed(L, seed, (uint32_t)(t0 + k), s);
        else
            or_sweep(L, seed, (uint32_t)(t0 + k), s);
    }
}

void or_run(int L, uint64_t seed, int8_t *s, uint64_t t0, uint64_t n, uint64_t every,
            int64_t *trace)
{
    or_run_cycle(L, seed, s, t0, n, every, trace, 0);
}

/* ------------------------------------------------------------------------ */
/* Window replay.  w holds a W^3 cube of the periodic L^3 lattice whose       */
/* corner sits at global (ox, oy, oz); w is indexed like the lattice, local  */
/* x fastest.  T sweeps starting at global time t0 are applied to the cube   */
/* using global coordinates for the colour and the colour index.  The cube's */
/* faces are never updated (their outside neighbours are unknown); since a   */
/* half-sweep moves information by one site, after T sweeps every site at    */
/* local distance >= 2T from each face holds the exact global result.        */
/* ------------------------------------------------------------------------ */
/* mixed != 0: the mixed cycle (Supplementary Methods I B), whose sweep t     */
/* updates colour or_first_colour(seed, t) first; else the 01 cycle.         */
void or_window_advance_cycle(int L, uint64_t seed, int ox, int oy, int oz, int W, int8_t *w,
                             uint64_t t0, uint64_t T, int mixed)
{
    for (uint64_t k = 0; k < T; ++k) {
        uint32_t t = (uint32_t)(t0 + k);
        int first = mixed ? or_first_colour(seed, t) : 0;
        for (int half = 0; half < 2; ++half) {
            int p = half ? 1 - first : first;
#pragma omp parallel for schedule(static)
            for (int lz = 1; lz < W - 1; ++lz)
                for (int ly = 1; ly < W - 1; ++ly)
                    for (int lx = 1; lx < W - 1; ++lx) {
                        int gx = (ox + lx) % L, gy = (oy + ly) % L, gz = (oz + lz) % L;
                        if (((gx + gy + gz) & 1) != p)
                            continue;
                        int64_t i = or_idx(W, lx, ly, lz);
                        int8_t me = w[i];
                        int a = 0;
                        a += w[or_idx(W, lx + 1, ly, lz)] != me;
                        a += w[or_idx(W, lx - 1, ly, lz)] != me;
                        a += w[or_idx(W, lx, ly + 1, lz)] != me;
                        a += w[or_idx(W, lx, ly - 1, lz)] != me;
                        a += w[or_idx(W, lx, ly, lz + 1)] != me;
                        a += w[or_idx(W, lx, ly, lz - 1)] != me;
                        int flip = 0;
                        if (a >= 4) {
                            flip = 1;
                        } else if (a == 3) {
                            uint64_t j = (uint64_t)(gx / 2) +
                                         (uint64_t)(L / 2) *
                                             ((uint64_t)gy + (uint64_t)L * (uint64_t)gz);
                            flip = or_tie_bit(seed, t, p, j);
                        }
                        if (flip)
                            w[i] = (int8_t)-me;
                    }
        }
    }
}

void or_window_advance(int L, uint64_t seed, int ox, int oy, int oz, int W, int8_t *w,
                       uint64_t t0, uint64_t T)
{
    or_window_advance_cycle(L, seed, ox, oy, oz, W, w, t0, T, 0);
}

/* Thread control for the OpenMP loops; returns the count now in effect. */
int or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
