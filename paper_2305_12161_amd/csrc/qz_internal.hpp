// qz_internal.hpp -- host-side declarations shared by the library's
// translation units: the lattice object, tuning knobs and kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "qz_batch_plan.hpp"

namespace qz {

// Device-memory map of one lattice inside the caller's buffer.  Offsets are
// 256-byte aligned.
struct StateMap {
    size_t spins_off;     // I8: N bytes.  BIT: two copies of [plane0 | plane1]
    size_t spins_bytes;   //   each plane N/16 bytes (N/8 per copy)
    size_t counter_off;   // 64 uint64 counters for measurements
    size_t corr_off;      // 3*(L/2+1) + 1 int64 correlation accumulators
    size_t trace_off;     // kTraceCap uint64 trace slots for host-trace runs
    size_t flips_off;     // kTraceCap uint64 accepted-flip slots for host-trace runs
    size_t stage_off;     // staging bytes for host copies
    size_t stage_bytes;
    size_t total;
};

constexpr size_t kTraceCap = 4096;
constexpr size_t kStageMax = size_t(4) << 20;   // at least one L*L plane is always allowed

bool state_map(uint32_t L, int layout, StateMap *m);

// Tuning of the fused bit-sweep kernel (see qz_bit.hip).
struct BitTuning {
    int V;    // 32-bit words per lane along x: 1, 2 or 4
    int Ty;   // rows (y) owned per tile; Ty == L means whole planes, no y halo
    int Tz;   // planes (z) per tile
};
bool bit_tuning_valid(uint32_t L, const BitTuning &t);
BitTuning bit_tuning_default(uint32_t L);
// Tuning of the two-sweep pass (qz_bit2.hip): Ty owned rows, E = Ty + 8 held.
bool bit_tuning2_valid(uint32_t L, const BitTuning &t);
BitTuning bit_tuning2_default(uint32_t L);
int bit_pass_default(uint32_t L);

// ----- int8 layout -----
hipError_t i8_init(hipStream_t st, uint32_t L, uint64_t seed, int8_t *s);
// which = 0: first half-sweep of sweep t (colour 0, or the drawn colour in the
// mixed cycle), which = 1: the second.
// bond_acc / flip_acc (nullable): bond count of the state entering the pass,
// accepted flips of the pass.
// Small lattices (L = 16 or 32): n sweeps from time t0 in one
// launch of one workgroup with the lattice in LDS; sweep t0 + k with
// k % every == 0 (every > 0) adds its entering bond count to dev_B[k / every]
// and its flips to dev_F[k / every] (either may be null).
bool i8_onchip_ok(uint32_t L);
hipError_t i8_onchip_run(hipStream_t st, uint32_t L, uint64_t seed, uint32_t t0, uint32_t n,
                         bool mixed, int8_t *s, uint32_t every, unsigned long long *dev_B,
                         unsigned long long *dev_F);
hipError_t i8_half_sweep(hipStream_t st, uint32_t L, uint64_t seed, uint32_t t, int which,
                         bool mixed, int8_t *s, unsigned long long *bond_acc,
                         unsigned long long *flip_acc);
hipError_t i8_bonds(hipStream_t st, uint32_t L, const int8_t *s, unsigned long long *acc3);
hipError_t i8_corr(hipStream_t st, uint32_t L, const int8_t *s, long long *S, long long *M);
hipError_t i8_check_pm1(hipStream_t st, size_t n, const int8_t *s, unsigned long long *bad);

// ----- bit layout -----
// planes: copy k (0/1) at base + k*N/8 bytes, colour c at + c*N/16.
hipError_t bit_init(hipStream_t st, uint32_t L, uint64_t seed, uint32_t *P0, uint32_t *P1);
hipError_t bit_sweep(hipStream_t st, uint32_t L, uint64_t seed, uint32_t t, const BitTuning &tu,
                     const uint32_t *S0, const uint32_t *S1, uint32_t *D0, uint32_t *D1,
                     unsigned long long *bond_acc, bool mixed,
                     unsigned long long *flip_acc = nullptr);
// Sweeps t and t+1 in one pass (copy S -> copy D); acc_a / acc_c (nullable)
// receive the bond counts of the states entering them.  first: the colour
// sweep t updates first; swap: sweep t+1 updates the other colour first (the
// mixed cycle's pairs of different orders), else the same one.
hipError_t bit_sweep2(hipStream_t st, uint32_t L, uint64_t seed, uint32_t t, const BitTuning &tu,
                      const uint32_t *S0, const uint32_t *S1, uint32_t *D0, uint32_t *D1,
                      unsigned long long *acc_a, unsigned long long *acc_c,
                      unsigned long long *flip_a = nullptr, unsigned long long *flip_c = nullptr,
                      uint32_t first = 0, bool swap = false);
hipError_t bit_bonds(hipStream_t st, uint32_t L, const uint32_t *P0, const uint32_t *P1,
                     unsigned long long *acc3);
hipError_t bit_bonds_total(hipStream_t st, uint32_t L, const uint32_t *P0, const uint32_t *P1,
                           unsigned long long *acc);
// Double-checkerboard sweep in place (B a power of two >= 2, L % 2B == 0).
hipError_t bit_double_sweep(hipStream_t st, uint32_t L, uint32_t B, uint64_t seed, uint32_t t,
                            uint32_t *P0, uint32_t *P1, bool mixed,
                            unsigned long long *flip_acc = nullptr);
// One phase of bit_double_sweep, in place: fine colour p of the cubes of
// coarse colour kc (its position in the sweep's order when mixed), step
// `step` of the mixed cycle's per-cube fine order.
hipError_t bit_double_phase(hipStream_t st, uint32_t L, uint32_t B, uint64_t seed, uint32_t t,
                            uint32_t *P0, uint32_t *P1, uint32_t kc, uint32_t p, uint32_t step,
                            bool mixed, unsigned long long *flip_acc);
// Whether bit_double_sweep2 takes tiling tu at side L (the mixed cycle runs
// with fewer rows per tile, about 256 lanes, and needs at most 512).
bool bit_double_sweep2_fits(uint32_t L, const BitTuning &tu, bool mixed);
// One double-checkerboard sweep in one pass of the two-sweep kernel (copy S ->
// copy D, tiling tu); bond_acc / flip_acc (nullable) receive the bond count
// of the entering state and the flips of the pass.  mixed: the mixed cycle's
// stages A-D; its last step (fine colour 0 of the second coarse colour's
// cubes that take fine colour 1 first) is then left to bit_double_phase(kc =
// 1, p = 0, step = 1) on copy D.
hipError_t bit_double_sweep2(hipStream_t st, uint32_t L, uint32_t B, uint64_t seed, uint32_t t,
                             const BitTuning &tu, const uint32_t *S0, const uint32_t *S1,
                             uint32_t *D0, uint32_t *D1, bool mixed,
                             unsigned long long *bond_acc, unsigned long long *flip_acc);
// Q0, Q1: scratch colour planes of the same size (the lattice's idle copy;
// overwritten), or null.  With scratch and L a multiple of 256 all three axes
// run on the matrix cores, else x (and, for other L, y and z) by XOR and
// popcount.
hipError_t bit_corr(hipStream_t st, uint32_t L, const uint32_t *P0, const uint32_t *P1,
                    unsigned long long *anti /* 3*(L/2+1) */, unsigned long long *ones,
                    uint32_t *Q0 = nullptr, uint32_t *Q1 = nullptr);
// Unpack planes z in [z0, z0+nz) to int8 (index (z-z0)*L*L + y*L + x).
hipError_t bit_unpack(hipStream_t st, uint32_t L, const uint32_t *P0, const uint32_t *P1,
                      uint32_t z0, uint32_t nz, int8_t *out);
// Pack planes z in [z0, z0+nz) from int8; counts entries that are not +-1.
hipError_t bit_pack(hipStream_t st, uint32_t L, uint32_t *P0, uint32_t *P1, uint32_t z0,
                    uint32_t nz, const int8_t *in, unsigned long long *bad);
// Extract window planes lz in [lz0, lz0+nz) of a W^3 window at origin o.
hipError_t bit_window(hipStream_t st, uint32_t L, const uint32_t *P0, const uint32_t *P1,
                      uint32_t ox, uint32_t oy, uint32_t oz, uint32_t W, uint32_t lz0,
                      uint32_t nz, int8_t *out);
hipError_t i8_window(hipStream_t st, uint32_t L, const int8_t *s, uint32_t ox, uint32_t oy,
                     uint32_t oz, uint32_t W, uint32_t lz0, uint32_t nz, int8_t *out);

hipError_t fill_u64(hipStream_t st, unsigned long long *p, size_t n, unsigned long long v);

// ----- FFT correlation (qz_fft.hip) -----
uint32_t fft_pad(uint32_t L);
uint32_t fft_nbins(uint32_t L);
// layout 1: spins0/spins1 = colour planes; layout 0: spins0 = int8 lattice
hipError_t fft_unpack(hipStream_t st, uint32_t L, int layout, const void *spins0,
                      const void *spins1, double *X);
hipError_t fft_power(hipStream_t st, uint32_t L, double *X, uint32_t nb, double *sk_sum,
                     unsigned long long *sk_cnt, double *M_out);
hipError_t fft_radial(hipStream_t st, uint32_t L, const double *X, uint32_t nb, double *c_sum,
                      unsigned long long *c_cnt);
hipError_t fft_zero(hipStream_t st, double *d, size_t n);

// ----- batched replicas (qz_batch.hip; tables planned in qz_batch_plan.hpp) -----
struct BatchArgs {
    const BatchReplica *reps;
    const BatchTile *tiles;
    const BatchGroup *groups;
    uint32_t step;                  // sweeps already done in this group of sweeps
    uint32_t every, cap;            // bond count every `every` sweeps into a ring of `cap`
    size_t lds_bytes;
};
hipError_t batch_sweep(hipStream_t st, const BatchArgs &a, uint32_t ngroups);
hipError_t batch_advance(hipStream_t st, BatchReplica *reps, uint32_t n, uint32_t k);
// k sweeps of the listed replicas of side 64, each held on chip by one workgroup
hipError_t batch_onchip64(hipStream_t st, const BatchReplica *reps, const uint32_t *slots,
                          uint32_t nslots, uint32_t k, uint32_t every, uint32_t cap);
hipError_t batch_clear_trace(hipStream_t st, BatchReplica *reps, uint32_t n, uint32_t span,
                             uint32_t every, uint32_t cap);

}  // namespace qz
