/*
 * quench.h -- C ABI of libquench, the MI355X (gfx950) library for the
 * zero-temperature single-spin-flip quench of the d=3 nearest-neighbour Ising
 * model with checkerboard updates (Gessert, Christiansen, Janke,
 * arXiv:2305.12161).
 *
 * Model (Methods, "Spin updates"): spins s = +-1 on a periodic L^3 simple-cubic
 * lattice, ferromagnetic coupling J = 1, k_B = 1.  A proposal to flip s_i with
 * a anti-aligned neighbours changes the energy by dE = 12 - 4a and is accepted
 * with the T -> 0 Glauber probability (Methods, equation
 * equ:glauberAcceptance): always if dE < 0 (a >= 4), with probability 1/2 if
 * dE = 0 (a == 3), never if dE > 0.
 *
 * Sweep (Methods, "Checkerboard update"; Supplementary Methods I B): all
 * sites of colour 0, (x+y+z) even, are updated concurrently, then all sites of
 * colour 1; the same "01 cycle" order every sweep.  One sweep is N = L^3
 * proposals, one Monte Carlo sweep (MCS).
 *
 * Random bits (the paper names no generator; this is the library's contract):
 * Philox4x32-10 (Salmon et al., SC'11) with key (seed mod 2^32, seed >> 32).
 *   lattice index  i = x + L*(y + L*z);  colour index j = x/2 + (L/2)*(y + L*z)
 *   tie bit of a colour-p site during 0-based sweep t:
 *       counter (j/128, t, p, 0), bit (w[(j>>5)&3] >> (j&31)) & 1, flip iff 1
 *   initial spin of site i (infinite-temperature start, Results):
 *       counter (i/128, 0, 0, 1), bit (w[(i>>5)&3] >> (i&31)) & 1, +1 iff 1
 * Results are therefore a pure function of (L, seed, t): they do not depend on
 * the layout, tiling, batching or anything else running on the device.
 *
 * Measurements:
 *   B(t)   unsigned count of unsatisfied bonds, B = sum over axes a of
 *          #{i : s_i != s_{i+e_a}}; energy E = -(3N - 2B).  The paper measures
 *          length through C(r,t); 3N/B (energy-excess length) is an addition.
 *   S_a(r) = sum_i s_i s_{i + r e_a} for r = 0..L/2 and a = x, y, z, and
 *   M      = sum_i s_i: the integer pieces of the two-point function
 *          C(r,t) = <s_i s_j> - <s_i><s_j> (Results, eq:correlation function)
 *          along the axes.  ell is where C crosses 1/2 (Results).
 *
 * Conventions for every entry point:
 *   Memory   -- device memory is owned by the caller (e.g. a torch tensor) and
 *               must outlive the handle; the library allocates no device
 *               memory of its own (the FFT plans made by qz_fft_prepare hold
 *               hipFFT's internal tables).  Host arrays are caller-allocated.
 *   Streams  -- all device work is enqueued on the stream given at creation.
 *               Calls that return host data synchronise that stream; the others
 *               are asynchronous.
 *   Errors   -- every call returns a qz_status; nothing is thrown across the
 *               ABI.  qz_last_error() gives the text of the calling thread's
 *               last failure.  After a QZ_EDEVICE failure the handle answers
 *               QZ_ESTATE to everything but qz_destroy.
 *   Threads  -- a handle is not thread-safe; use one handle per host thread.
 */
#ifndef QUENCH_H
#define QUENCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QZ_ABI_VERSION 2

typedef enum {
    QZ_OK = 0,
    QZ_EINVAL = -1,       /* bad argument: L odd or < 4, null pointer, bad layout, ...   */
    QZ_ENOMEM = -2,       /* caller's device buffer smaller than qz_state_bytes()        */
    QZ_EDEVICE = -3,      /* a HIP call failed; text in qz_last_error()                  */
    QZ_ESTATE = -4,       /* handle unusable after an earlier device failure             */
    QZ_EUNSUPPORTED = -5  /* the layout cannot hold this L (see qz_layout)               */
} qz_status;

/* Spin storage.
 *   QZ_LAYOUT_I8:  one int8 (+1/-1) per site, index i; any even L >= 4.
 *   QZ_LAYOUT_BIT: one bit per site (1 = +1), colour-separated: plane c holds
 *                  the colour-c sites as words [z][y][L/64] of 32 bits, bit b of
 *                  word w = site x = 64w + 2b + ((c+y+z)&1).  Needs L % 64 == 0.
 *                  Two copies (read / write) are kept so that both colours of a
 *                  sweep are updated in one pass over memory. */
typedef enum { QZ_LAYOUT_I8 = 0, QZ_LAYOUT_BIT = 1 } qz_layout;

typedef struct qz_lattice qz_lattice; /* opaque, library-owned host object */

/* ABI version of the loaded library (QZ_ABI_VERSION when it matches this header). */
int qz_abi_version(void);

/* Device bytes a lattice of side L needs in `layout`, spins plus counters and
 * staging space; 0 if L or layout is invalid for the layout. */
size_t qz_state_bytes(uint32_t L, int layout);

/* Create a lattice of side L in caller memory dev_mem (dev_bytes >=
 * qz_state_bytes) and draw the infinite-temperature start from `seed`
 * (Results: random configurations, m close to 0); t := 0.  hip_stream is a
 * hipStream_t (NULL = the default stream).  Errors: QZ_EINVAL, QZ_ENOMEM,
 * QZ_EUNSUPPORTED, QZ_EDEVICE. */
int qz_create(uint32_t L, uint64_t seed, int layout, void *dev_mem, size_t dev_bytes,
              void *hip_stream, qz_lattice **out);

/* Release the host object (the caller's device memory is left alone). */
int qz_destroy(qz_lattice *q);

/* Advance n_sweeps MCS from the current time t0.  If trace_every > 0 (and
 * n_sweeps % trace_every == 0), host_trace receives n_sweeps/trace_every
 * values B(t0 + k*trace_every), each the bond count of the state at the start
 * of that sweep, computed inside the sweep itself; this call then synchronises.
 * With trace_every == 0 it is asynchronous.  Errors: QZ_EINVAL, QZ_ESTATE,
 * QZ_EDEVICE. */
int qz_run(qz_lattice *q, uint64_t n_sweeps, uint64_t trace_every, uint64_t *host_trace);

/* As qz_run, but the trace goes to caller device memory dev_trace
 * (n_sweeps/trace_every uint64 values, zeroed by the library) and the call
 * never synchronises. */
int qz_run_device(qz_lattice *q, uint64_t n_sweeps, uint64_t trace_every, uint64_t *dev_trace);

/* As qz_run / qz_run_device, with a second trace: flips[k] receives the number
 * of spins that sweep t0 + k*trace_every flipped (accepted moves, the physics
 * output beside the attempts; each site is proposed once per sweep, Methods
 * "Checkerboard update", so this is also the Hamming distance between the
 * states before and after that sweep).  B or flips may be null (not both when
 * trace_every > 0).  The batch engine does not trace flips. */
int qz_run_traced(qz_lattice *q, uint64_t n_sweeps, uint64_t trace_every, uint64_t *host_B,
                  uint64_t *host_flips);
int qz_run_device_traced(qz_lattice *q, uint64_t n_sweeps, uint64_t trace_every, uint64_t *dev_B,
                         uint64_t *dev_flips);

/* As qz_run_traced / qz_run_device_traced, but the traced sweeps are listed:
 * at[0 .. n_at-1] are sweep offsets within the run (0 <= at[i] < n_sweeps,
 * strictly increasing; QZ_EINVAL otherwise), and entry i of B / flips belongs
 * to sweep t0 + at[i] (the bond count of the state entering it, the spins it
 * flips).  This fits measurement schedules that are not uniform, such as the
 * log-spaced times of the Results.  Listed sweeps do not break the pairing of
 * sweeps into passes over memory (qz_set_pass): either sweep of a pass can be
 * counted inside the pass.  B or flips may be null (not both when n_at > 0).
 * qz_run_at writes host arrays and synchronises; qz_run_device_at writes
 * caller device memory (n_at uint64 values each, zeroed by the library) and
 * never synchronises; the list itself is host memory, read before the call
 * returns. */
int qz_run_at(qz_lattice *q, uint64_t n_sweeps, const uint64_t *at, size_t n_at,
              uint64_t *host_B, uint64_t *host_flips);
int qz_run_device_at(qz_lattice *q, uint64_t n_sweeps, const uint64_t *at, size_t n_at,
                     uint64_t *dev_B, uint64_t *dev_flips);

/* Per-axis unsatisfied-bond counts [B_x, B_y, B_z] of the current state. */
int qz_bonds(qz_lattice *q, uint64_t out_B_axes[3]);

/* As qz_bonds, but the three counts go to caller device memory dev_B_axes
 * (8-byte aligned, zeroed by the library) on the lattice's stream, and the
 * call never synchronises: a caller can enqueue it behind a run and read the
 * counts when its own event on that stream has completed.  Errors: QZ_EINVAL
 * (null or misaligned pointer), QZ_ESTATE, QZ_EDEVICE. */
int qz_bonds_device(qz_lattice *q, uint64_t *dev_B_axes);

/* Axis correlation sums of the current state: out_S[a*(L/2+1) + r] = S_a(r)
 * for a = 0 (x), 1 (y), 2 (z) and r = 0..L/2, and *out_M = M.  For the bit
 * layout with L a multiple of 256 they come from the matrix cores (Gram
 * matrix of the spins along each axis), and the x axis uses the state
 * buffer's idle copy (the one the next sweep overwrites) as scratch; the
 * results are the same integers as by direct summation. */
int qz_corr(qz_lattice *q, int64_t *out_S, int64_t *out_M);

/* For callers that cannot allocate device memory or touch the lattice's idle
 * copy (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): qz_corr with the same outputs, whose accumulators live
 * in a 64 KiB device array of the library (one per device, found at the
 * call's first use on that device) instead of the lattice's buffer, and whose
 * x axis never uses the idle copy.  It calls no allocation routine.  Every
 * call on a device shares that array: calls that overlap on one device (from
 * several threads or streams) race and must be serialised by the caller.
 * QZ_EINVAL if 3 (L/2 + 1) + 1 > 8192 (never for the layouts' sides). */
int qz_corr_noalloc(qz_lattice *q, int64_t *out_S, int64_t *out_M);

/* Current time t (completed sweeps). */
int qz_time(const qz_lattice *q, uint64_t *t);

/* Copy the whole lattice to host as int8 +-1, index i (N = L^3 bytes). */
int qz_download_spins(qz_lattice *q, int8_t *host);

/* Replace the lattice by host int8 values (each must be +1 or -1, else
 * QZ_EINVAL and the state is unspecified) and set the time to t (used for
 * special initial states and for resuming from a checkpoint). */
int qz_upload_spins(qz_lattice *q, const int8_t *host, uint64_t t);

/* Copy a W^3 cube whose corner is at global origin[0..2] = (x, y, z), taken
 * periodically, to host as int8, local x fastest.  1 <= W <= L. */
int qz_download_window(qz_lattice *q, const uint32_t origin[3], uint32_t W, int8_t *host);

/* Tuning of the fused one-pass sweep of the bit layout: V 32-bit words per
 * lane along x (1, 2 or 4, dividing L/64), Ty rows of y per tile (Ty == L
 * means whole planes with no halo rows) and Tz planes of z per tile.  Results
 * never depend on the tuning.  QZ_EINVAL if the triple does not fit this L
 * (at most 1024 threads and 60 KiB of LDS per workgroup); QZ_EUNSUPPORTED for
 * the int8 layout, which has no tuning.  Default: whole planes (Tz = 8) up to
 * L = 128, else tiles of 28 owned rows (fewer for long rows) and Tz = 8. */
int qz_set_tuning(qz_lattice *q, int V, int Ty, int Tz);
int qz_get_tuning(const qz_lattice *q, int out_V_Ty_Tz[3]);

/* Sweeps per pass over memory (bit layout).  sweeps = 1: every sweep reads
 * and writes the lattice once.  sweeps = 2: sweeps t and t+1 run
 * in one pass that keeps the state after sweep t on chip, halving the memory
 * traffic per sweep; the trajectory, the bond trace and every measurement are
 * identical to sweeps = 1 (Methods, "Checkerboard update").  Runs of an odd
 * number of sweeps end with one single sweep; in the mixed cycle two sweeps
 * share a pass whichever first colours they draw; the double checkerboard
 * runs one sweep per pass (see qz_set_double_checkerboard).
 * V, Ty, Tz tune the two-sweep kernel as in qz_set_tuning
 * (V words per lane, Ty owned rows per tile, Ty + 8 rows held, Tz planes);
 * all three 0 selects the default for L.  QZ_EINVAL for another sweep count
 * or a tuning that does not fit (at most 1024 threads and 64 KiB of LDS per
 * workgroup); QZ_EUNSUPPORTED for the int8 layout.  qz_get_pass reports
 * (sweeps, V, Ty, Tz).  Default: 2 for L >= 1024 (where the one-sweep pass is
 * bound by HBM bandwidth), else 1. */
int qz_set_pass(qz_lattice *q, int sweeps, int V, int Ty, int Tz);
int qz_get_pass(const qz_lattice *q, int out_sweeps_V_Ty_Tz[4]);

/* Sublattice order (Supplementary Methods I B).  QZ_CYCLE_01 (the default, the
 * paper's main runs): colour 0 then colour 1 in every sweep.  QZ_CYCLE_MIXED:
 * the colour updated first in sweep t is drawn at random for each sweep --
 * colour 1 first iff bit 0 of word 0 of Philox block (0, t, 2, 0) is set --
 * which restores detailed balance.  With the double checkerboard the mixed
 * cycle draws the coarse order and each cube's fine order instead (see
 * qz_set_double_checkerboard).  The bond trace of a sweep is still the bond
 * count of the state entering it. */
enum { QZ_CYCLE_01 = 0, QZ_CYCLE_MIXED = 1 };
int qz_set_cycle(qz_lattice *q, int cycle);

/* Double checkerboard (Supplementary Methods I A; bit layout).  Cubes of side
 * B form a coarse checkerboard, coarse colour (x/B + y/B + z/B) mod 2.  In the
 * 01 cycle a sweep updates the coarse-colour-0 cubes (fine colour 0 sites,
 * then fine colour 1 sites), then the coarse-colour-1 cubes the same way.  In
 * the mixed cycle (Supplementary Methods I B) the coarse colour taken first in
 * sweep t is 1 iff bit 0 of word 0 of Philox block (0, t, 3, 0) is set, and
 * cube b = x/B + (L/B)(y/B + (L/B) z/B) updates fine colour 1 first iff bit b
 * of the blocks (b/128, t, 4, 0) is set (bit extraction as for the tie bits).
 * Each site draws the same tie bit as in the plain checkerboard.  B must be a
 * power of two >= 2 with L % (2B) == 0 (QZ_EINVAL otherwise); B = 0 returns to
 * the plain checkerboard.  QZ_EUNSUPPORTED on the int8 layout.  The paper does
 * not state its block size.  With two sweeps per pass (qz_set_pass; the
 * default from L = 1024) a sweep runs in one pass over memory between the two
 * copies (the mixed cycle adds one in-place pass for its last step; tiles of
 * more than 512 lanes run it as phases); otherwise each phase is a pass that
 * updates the lattice in place.  The results are the same. */
int qz_set_double_checkerboard(qz_lattice *q, uint32_t B);

/* The paper's own correlation measurement (Methods, "Calculating the
 * correlation function", eq:sisik): G(d) = (1/N) sum_i s_i s_{i+d} for every
 * displacement d by a double-precision real FFT (in place), then averaged over
 * spherical shells.  Shell b holds the displacements d (minimum image, each
 * component in [-L/2, L/2)) with round(|d|) == b, and the wavevectors k
 * (integer components in [-L/2, L/2), units 2 pi / L) with round(|k|) == b,
 * for b < qz_fft_nbins(L) = round(sqrt(3) L / 2) + 2.
 *   out_C[b]  = mean of G over shell b minus m^2 (connected C(r), Results)
 *   out_Sk[b] = mean of |F s(k)|^2 / N over shell b (structure factor S(k))
 *   out_nr[b], out_nk[b] = shell populations;  *out_m = M / N.
 * qz_fft_prepare makes the FFT plans (kept with the handle) and reports the
 * scratch bytes qz_fft_corr needs: about 8 L^2 (L + 2) bytes plus the FFT
 * library's work area.  The scratch is caller-owned device memory; the
 * library allocates nothing.  Synchronises. */
uint32_t qz_fft_nbins(uint32_t L);
int qz_fft_prepare(qz_lattice *q, size_t *scratch_bytes);
int qz_fft_corr(qz_lattice *q, void *dev_scratch, size_t bytes, double *out_C, double *out_Sk,
                uint64_t *out_nr, uint64_t *out_nk, double *out_m);

/* ------------------------------------------------------------------------
 * Batched replicas.  Many independent lattices ("replicas", each its own L
 * and seed, 1-bit layout with L % 64 == 0 and L <= 256) held in one caller
 * buffer and advanced together: one kernel launch sweeps every active replica
 * once, each at its own time t, and groups of sweeps are replayed from a
 * captured HIP graph.  Every replica follows exactly the trajectory a single
 * lattice created from the same (L, seed) would follow: batching never changes
 * results.  The paper runs 40 independent realisations per lattice size
 * (Results); a batch runs such ensembles side by side, and a server keeps one
 * batch resident and refills its slots (qz_batch_slot_replace).
 * ------------------------------------------------------------------------ */
typedef struct qz_batch qz_batch;  /* opaque, library-owned host object */

typedef struct {
    uint32_t L;      /* side; L % 64 == 0 and 64 <= L <= 256 */
    uint64_t seed;   /* seed of the T = infinity start and of the tie bits */
    uint64_t t_max;  /* the replica stops (is skipped) from this time on; 0 = never */
} qz_replica_spec;

/* Device bytes for n replica slots with a bond-count ring of trace_cap
 * entries per slot; 0 if a size is unsupported.  Slot i is sized for
 * specs[i].L and can later hold any side up to that one. */
size_t qz_batch_state_bytes(const qz_replica_spec *specs, size_t n, uint32_t trace_cap);

/* Create the batch in caller memory and draw every slot's start (t := 0, all
 * slots active).  If trace_every > 0, the sweep starting at each time t with
 * t % trace_every == 0 records B(t) of that slot into its ring of trace_cap
 * entries (entry (t / trace_every) % trace_cap).
 * tuning_json (nullable) fixes the launch shape, e.g.
 *     {"graph_sweeps": 100, "tz": {"64": 8, "128": 8, "256": 8}}
 * -- planes per sub-tile for slots of side L (each must divide L; sides not
 * named take the default, 8) and sweeps per captured graph (0: no graph;
 * default 100; at most trace_cap * trace_every).  With tuning_json == NULL
 * the library autotunes: for each side in the batch it times a few sweeps of
 * the whole batch per candidate plane count (2, 4, 8, 16, 32) and keeps the
 * fastest, then draws the starts again (the choice never changes results).
 * The library also creates a private stream, used only to capture graphs.
 * Errors: QZ_EINVAL (also for malformed tuning_json), QZ_ENOMEM,
 * QZ_EUNSUPPORTED, QZ_EDEVICE. */
int qz_batch_create(const qz_replica_spec *specs, size_t n, uint32_t trace_every,
                    uint32_t trace_cap, void *dev_mem, size_t dev_bytes, void *hip_stream,
                    const char *tuning_json, qz_batch **out);
int qz_batch_destroy(qz_batch *b);

/* Advance every active slot by n_sweeps MCS (a slot with t_max stops there).
 * host_traces == NULL or trace_every == 0: asynchronous.  Otherwise
 * trace_every must equal the batch's, the call synchronises, and for slot s
 * entry i of host_traces[s * P .. s * P + P - 1], P = ceil(n_sweeps /
 * trace_every), is B(tau_s + i * trace_every), where tau_s is the first
 * multiple of trace_every at or after the slot's time t0_s when the call
 * starts -- or UINT64_MAX where the slot did not reach that time in this run
 * (parked, at its t_max, or past the run's end). */
int qz_batch_run(qz_batch *b, uint64_t n_sweeps, uint64_t trace_every, uint64_t *host_traces);

/* Wait for the batch's work and refresh the host view of slot times. */
int qz_batch_sync(qz_batch *b);

/* Serving: put a new replica into a slot -- side spec->L (at most the side the
 * slot was created with, QZ_EINVAL otherwise), seed, t_max -- drawing its
 * start at t = 0 and making it active (synchronises; rebuilds the launch's
 * tile tables if the side changes). */
int qz_batch_slot_replace(qz_batch *b, size_t slot, const qz_replica_spec *spec);

/* Restart a slot from a new T = infinity start drawn from `seed`, at t = 0,
 * keeping its side and t_max, and make it active (synchronises). */
int qz_batch_slot_reset(qz_batch *b, size_t slot, uint64_t seed);

/* Park (active = 0) or resume (active = 1) a slot (synchronises). */
int qz_batch_slot_active(qz_batch *b, size_t slot, int active);

/* Current time of a slot (synchronises). */
int qz_batch_slot_time(qz_batch *b, size_t slot, uint64_t *t);

/* host[i] = B(t_from + i*trace_every) for i < count, from the slot's ring;
 * QZ_EINVAL if t_from is not a multiple of trace_every, if an entry lies at
 * or beyond the slot's current time, or if it has been overwritten. */
int qz_batch_trace(qz_batch *b, size_t slot, uint64_t t_from, uint64_t count, uint64_t *host);

/* A slot's lattice as int8 +-1 (L^3 bytes, index i), per-axis bond counts and
 * axis correlation sums, with the meanings of qz_download_spins, qz_bonds and
 * qz_corr (all synchronise; qz_batch_corr also uses the slot's idle copy as
 * scratch). */
int qz_batch_download(qz_batch *b, size_t slot, int8_t *host);
int qz_batch_bonds(qz_batch *b, size_t slot, uint64_t out_B_axes[3]);
int qz_batch_corr(qz_batch *b, size_t slot, int64_t *out_S, int64_t *out_M);

/* Planes per sub-tile for slots of side L (Tz divides L; 0 keeps the current
 * value) and sweeps per captured graph (0 = no graph; at most
 * trace_cap * trace_every, larger values are reduced to that, so that one
 * graph never reuses a ring entry).  Results never depend on it. */
int qz_batch_set_tuning(qz_batch *b, uint32_t L, uint32_t Tz, uint32_t graph_sweeps);

/* The launch shape in use as text (NUL-terminated, at most len bytes):
 * {"source": "json" | "autotune" | "set", "graph_sweeps": G,
 *  "tz": {"L": Tz, ...}} for every side in the batch. */
int qz_batch_tuning_json(const qz_batch *b, char *buf, size_t len);

/* Text for a status code, and the calling thread's last error message. */
const char *qz_status_string(int status);
const char *qz_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QUENCH_H */
