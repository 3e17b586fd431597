// qz_api.hip -- the C ABI declared in include/quench.h.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>

#include <hipfft/hipfft.h>

#include <vector>

#include "../../include/quench.h"
#include "qz_internal.hpp"

#define QZ_EXPORT extern "C" __attribute__((visibility("default")))

// Scratch of qz_corr_noalloc: the correlation accumulators of one call,
// 3 (L/2 + 1) + 1 counters, held by the library itself so that the call
// allocates nothing.  Every device the library runs on has its own copy at
// its own address (found with hipGetSymbolAddress); host code never passes
// the array's name to a kernel.  64 KiB covers every side the layouts take.
constexpr size_t kNoAllocWords = 8192;
static __device__ __align__(256) unsigned long long scratch[kNoAllocWords];

struct qz_lattice {
    uint32_t L;
    uint64_t seed;
    int layout;
    uint64_t t;
    uint8_t *base;
    size_t bytes;
    hipStream_t st;
    qz::StateMap map;
    int cur;                 // bit layout: which copy holds the current state
    qz::BitTuning tune;
    int pass;                // sweeps per pass over memory (1 or 2; bit layout)
    qz::BitTuning tune2;     // tuning of the two-sweep pass
    bool mixed;              // mixed cycle instead of the 01 cycle
    uint32_t dcb;            // > 0: double checkerboard with coarse cubes of this side
    bool failed;
    bool fft_ready;          // FFT plans made (qz_fft_prepare)
    hipfftHandle fft_fwd, fft_inv;
    size_t fft_work;
};

namespace {

thread_local std::string g_last_error;

int fail(int status, const std::string &msg)
{
    g_last_error = msg;
    return status;
}

int device_fail(qz_lattice *q, hipError_t e, const char *where)
{
    if (q)
        q->failed = true;
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    return fail(QZ_EDEVICE, buf);
}

#define QZ_HIP(q, call)                                   \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess)                             \
            return device_fail((q), e_, #call);           \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

bool layout_ok(uint32_t L, int layout)
{
    if (L < 4 || (L & 1u))
        return false;
    if (layout == QZ_LAYOUT_I8)
        return L <= 4096;
    if (layout == QZ_LAYOUT_BIT)
        return L % 64 == 0 && L <= 4096;
    return false;
}

uint64_t n_sites(uint32_t L) { return (uint64_t)L * L * L; }

int8_t *i8_spins(qz_lattice *q) { return reinterpret_cast<int8_t *>(q->base + q->map.spins_off); }

uint32_t *bit_plane(qz_lattice *q, int copy, int colour)
{
    const size_t plane_bytes = n_sites(q->L) / 16;
    return reinterpret_cast<uint32_t *>(q->base + q->map.spins_off +
                                        (size_t)copy * 2 * plane_bytes +
                                        (size_t)colour * plane_bytes);
}

unsigned long long *counters(qz_lattice *q)
{
    return reinterpret_cast<unsigned long long *>(q->base + q->map.counter_off);
}

int check_handle(qz_lattice *q)
{
    if (!q)
        return fail(QZ_EINVAL, "null handle");
    if (q->failed)
        return fail(QZ_ESTATE, "handle unusable after an earlier device failure");
    return QZ_OK;
}

// One sweep of the current state; bond_acc / flip_acc (device, may be null)
// receive the bond count of the state entering the sweep and the number of
// spins the sweep flips.
int sweep_once(qz_lattice *q, unsigned long long *bond_acc, unsigned long long *flip_acc)
{
    const uint32_t t = (uint32_t)q->t;
    if (q->layout == QZ_LAYOUT_I8) {
        QZ_HIP(q, qz::i8_half_sweep(q->st, q->L, q->seed, t, 0, q->mixed, i8_spins(q), bond_acc,
                                    flip_acc));
        QZ_HIP(q, qz::i8_half_sweep(q->st, q->L, q->seed, t, 1, q->mixed, i8_spins(q), nullptr,
                                    flip_acc));
    } else if (q->dcb > 0 && q->pass == 2 && qz::bit_double_sweep2_fits(q->L, q->tune2, q->mixed)) {
        // the 01 cycle's four phases in one pass over memory; the mixed
        // cycle's first four steps likewise, and its last one in place
        const int a = q->cur, b = 1 - q->cur;
        QZ_HIP(q, qz::bit_double_sweep2(q->st, q->L, q->dcb, q->seed, t, q->tune2,
                                        bit_plane(q, a, 0), bit_plane(q, a, 1), bit_plane(q, b, 0),
                                        bit_plane(q, b, 1), q->mixed, bond_acc, flip_acc));
        if (q->mixed)
            QZ_HIP(q, qz::bit_double_phase(q->st, q->L, q->dcb, q->seed, t, bit_plane(q, b, 0),
                                           bit_plane(q, b, 1), 1u, 0u, 1u, true, flip_acc));
        q->cur = b;
    } else if (q->dcb > 0) {
        const int c = q->cur;
        if (bond_acc)
            QZ_HIP(q, qz::bit_bonds_total(q->st, q->L, bit_plane(q, c, 0), bit_plane(q, c, 1),
                                          bond_acc));
        QZ_HIP(q, qz::bit_double_sweep(q->st, q->L, q->dcb, q->seed, t, bit_plane(q, c, 0),
                                       bit_plane(q, c, 1), q->mixed, flip_acc));
    } else {
        const int a = q->cur, b = 1 - q->cur;
        QZ_HIP(q, qz::bit_sweep(q->st, q->L, q->seed, t, q->tune, bit_plane(q, a, 0),
                                bit_plane(q, a, 1), bit_plane(q, b, 0), bit_plane(q, b, 1),
                                bond_acc, q->mixed, flip_acc));
        q->cur = b;
    }
    q->t += 1;
    return QZ_OK;
}

// Sweeps t and t+1 in one pass (bit layout, plain checkerboard); sweep t
// updates colour `first` first (always colour 0 in the 01 cycle), sweep t+1
// the same colour first, or the other one when swap is set.
int sweep_pair(qz_lattice *q, unsigned long long *acc_a, unsigned long long *acc_c,
               unsigned long long *flip_a, unsigned long long *flip_c, uint32_t first, bool swap)
{
    const int a = q->cur, b = 1 - q->cur;
    QZ_HIP(q, qz::bit_sweep2(q->st, q->L, q->seed, (uint32_t)q->t, q->tune2, bit_plane(q, a, 0),
                             bit_plane(q, a, 1), bit_plane(q, b, 0), bit_plane(q, b, 1), acc_a,
                             acc_c, flip_a, flip_c, first, swap));
    q->cur = b;
    q->t += 2;
    return QZ_OK;
}

// Bit 0 of word 0 of the Philox4x32-10 block (0, t, 2, 0) under the key
// (seed mod 2^32, seed >> 32): 1 when colour 1 goes first in sweep t of the
// mixed cycle (Supplementary Methods I B), as the sweep kernels draw it.  The
// host needs it to find consecutive sweeps with the same order.
uint32_t mixed_first_colour(uint64_t seed, uint32_t t)
{
    uint32_t c0 = 0u, c1 = t, c2 = 2u, c3 = 0u;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa = (uint64_t)0xD2511F53u * c0, pb = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c0 & 1u;
}

// Which sweeps of a run are traced: every `every`-th one (k % every == 0,
// entry k / every), or those listed in `at` (sorted, strictly increasing;
// entry i for the sweep at[i]).  Neither: no sweep.
struct TracePlan {
    uint64_t every = 0;
    const uint64_t *at = nullptr;
    size_t n_at = 0;
    // entry of sweep k, or -1; sweeps are asked for in increasing order
    mutable size_t next = 0;
    int64_t entry(uint64_t k) const
    {
        if (every > 0)
            return k % every == 0 ? (int64_t)(k / every) : -1;
        while (next < n_at && at[next] < k)
            ++next;
        return (next < n_at && at[next] == k) ? (int64_t)next : -1;
    }
};

int run_plan(qz_lattice *q, uint64_t n, const TracePlan &plan, unsigned long long *dev_trace,
             unsigned long long *dev_flips)
{
    if (q->layout == QZ_LAYOUT_I8 && qz::i8_onchip_ok(q->L) && plan.n_at == 0 &&
        plan.every <= 0xFFFFFFFFull) {
        // a small int8 lattice: all the sweeps on chip, in launches of whole
        // multiples of the trace cadence
        const uint64_t every = plan.every;
        const uint64_t piece = every > 0 ? std::max<uint64_t>(every, 65536 / every * every) : 65536;
        for (uint64_t k = 0; k < n;) {
            const uint64_t m = std::min<uint64_t>(piece, n - k);
            const uint64_t e = every > 0 ? k / every : 0;
            QZ_HIP(q, qz::i8_onchip_run(q->st, q->L, q->seed, (uint32_t)q->t, (uint32_t)m, q->mixed,
                                        i8_spins(q), (uint32_t)every,
                                        dev_trace != nullptr ? dev_trace + e : nullptr,
                                        dev_flips != nullptr ? dev_flips + e : nullptr));
            q->t += m;
            k += m;
        }
        return QZ_OK;
    }
    const bool pairs = q->pass == 2 && q->layout == QZ_LAYOUT_BIT && q->dcb == 0;
    auto slot = [&](unsigned long long *base, int64_t e) -> unsigned long long * {
        return (base != nullptr && e >= 0) ? base + e : nullptr;
    };
    for (uint64_t k = 0; k < n;) {
        const int64_t e0 = plan.entry(k);
        int rc;
        uint32_t first = 0u;
        bool swap = false;
        const bool pair = pairs && n - k >= 2;
        if (pair && q->mixed) {
            // the pass takes both orders of the second sweep
            first = mixed_first_colour(q->seed, (uint32_t)q->t);
            swap = mixed_first_colour(q->seed, (uint32_t)q->t + 1u) != first;
        }
        if (pair) {
            const int64_t e1 = plan.entry(k + 1);
            rc = sweep_pair(q, slot(dev_trace, e0), slot(dev_trace, e1), slot(dev_flips, e0),
                            slot(dev_flips, e1), first, swap);
            k += 2;
        } else {
            rc = sweep_once(q, slot(dev_trace, e0), slot(dev_flips, e0));
            k += 1;
        }
        if (rc != QZ_OK)
            return rc;
    }
    return QZ_OK;
}

// n sweeps; with every > 0, sweep k (k % every == 0) adds its entering bond
// count to dev_trace[k / every] and its accepted flips to dev_flips[k / every]
// (either pointer may be null).
int run_impl(qz_lattice *q, uint64_t n, uint64_t every, unsigned long long *dev_trace,
             unsigned long long *dev_flips)
{
    TracePlan plan;
    plan.every = every;
    return run_plan(q, n, plan, every > 0 ? dev_trace : nullptr, every > 0 ? dev_flips : nullptr);
}

// The list of traced sweeps must be strictly increasing and inside the run.
int check_list(const uint64_t *at, size_t n_at, uint64_t n_sweeps)
{
    if (n_at > 0 && !at)
        return fail(QZ_EINVAL, "null list of traced sweeps");
    for (size_t i = 0; i < n_at; ++i) {
        if (at[i] >= n_sweeps)
            return fail(QZ_EINVAL, "a traced sweep lies beyond the run");
        if (i > 0 && at[i] <= at[i - 1])
            return fail(QZ_EINVAL, "traced sweeps must be strictly increasing");
    }
    return QZ_OK;
}

// Device address of `scratch` on device dev, looked up once per device with
// that device current, and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long *g_scratch_ptr[kMaxDevices];

int scratch_on(int dev, unsigned long long **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return fail(QZ_EDEVICE, "device ordinal out of range for the static scratch");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev)
            e = hipSetDevice(dev);
        void *p = nullptr;
        if (e == hipSuccess)
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess)
                e = e2;
        }
        if (e != hipSuccess)
            return device_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
        if (!p)
            return fail(QZ_EDEVICE, "hipGetSymbolAddress(scratch) returned null");
        g_scratch_ptr[dev] = reinterpret_cast<unsigned long long *>(p);
    }
    *out = g_scratch_ptr[dev];
    return QZ_OK;
}

}  // namespace

namespace qz {
int set_error(int status, const char *msg) { return fail(status, msg); }

bool state_map(uint32_t L, int layout, StateMap *m)
{
    if (!layout_ok(L, layout))
        return false;
    const uint64_t N = n_sites(L);
    size_t off = 0;
    m->spins_off = off;
    m->spins_bytes = (layout == QZ_LAYOUT_I8) ? (size_t)N : (size_t)(N / 8) * 2;
    off = align256(off + m->spins_bytes);
    m->counter_off = off;
    off = align256(off + 64 * 8);
    m->corr_off = off;
    off = align256(off + (size_t)(3 * (L / 2 + 1) + 1) * 8);
    m->trace_off = off;
    off = align256(off + kTraceCap * 8);
    m->flips_off = off;
    off = align256(off + kTraceCap * 8);
    m->stage_off = off;
    m->stage_bytes = std::min<size_t>((size_t)N, kStageMax);
    m->stage_bytes = std::max<size_t>(m->stage_bytes, (size_t)L * L);
    off = align256(off + m->stage_bytes);
    m->total = off;
    return true;
}
}  // namespace qz

QZ_EXPORT int qz_abi_version(void) { return QZ_ABI_VERSION; }

QZ_EXPORT size_t qz_state_bytes(uint32_t L, int layout)
{
    qz::StateMap m;
    return qz::state_map(L, layout, &m) ? m.total : 0;
}

QZ_EXPORT int qz_create(uint32_t L, uint64_t seed, int layout, void *dev_mem, size_t dev_bytes,
                        void *hip_stream, qz_lattice **out)
{
    if (!out)
        return fail(QZ_EINVAL, "null output pointer");
    *out = nullptr;
    if (layout != QZ_LAYOUT_I8 && layout != QZ_LAYOUT_BIT)
        return fail(QZ_EINVAL, "unknown layout");
    if (L < 4 || (L & 1u))
        return fail(QZ_EINVAL, "L must be even and >= 4");
    if (!layout_ok(L, layout))
        return fail(QZ_EUNSUPPORTED, "the bit layout needs L % 64 == 0 (and L <= 4096)");
    if (!dev_mem)
        return fail(QZ_EINVAL, "null device buffer");
    if ((reinterpret_cast<uintptr_t>(dev_mem) & 255u) != 0)
        return fail(QZ_EINVAL, "device buffer must be 256-byte aligned");
    qz::StateMap m;
    qz::state_map(L, layout, &m);
    if (dev_bytes < m.total)
        return fail(QZ_ENOMEM, "device buffer smaller than qz_state_bytes()");
    qz_lattice *q = new (std::nothrow) qz_lattice();
    if (!q)
        return fail(QZ_ENOMEM, "host allocation failed");
    q->L = L;
    q->seed = seed;
    q->layout = layout;
    q->t = 0;
    q->base = reinterpret_cast<uint8_t *>(dev_mem);
    q->bytes = dev_bytes;
    q->st = reinterpret_cast<hipStream_t>(hip_stream);
    q->map = m;
    q->cur = 0;
    q->mixed = false;
    q->dcb = 0;
    q->pass = 1;
    q->failed = false;
    q->fft_ready = false;
    if (layout == QZ_LAYOUT_BIT) {
        q->tune = qz::bit_tuning_default(L);
        q->tune2 = qz::bit_tuning2_default(L);
        q->pass = qz::bit_pass_default(L);
    }
    hipError_t e;
    if (layout == QZ_LAYOUT_I8)
        e = qz::i8_init(q->st, L, seed, i8_spins(q));
    else
        e = qz::bit_init(q->st, L, seed, bit_plane(q, 0, 0), bit_plane(q, 0, 1));
    if (e != hipSuccess) {
        int rc = device_fail(nullptr, e, "init kernel");
        delete q;
        return rc;
    }
    *out = q;
    return QZ_OK;
}

QZ_EXPORT int qz_destroy(qz_lattice *q)
{
    if (!q)
        return fail(QZ_EINVAL, "null handle");
    if (q->fft_ready) {
        hipfftDestroy(q->fft_fwd);
        hipfftDestroy(q->fft_inv);
    }
    delete q;
    return QZ_OK;
}

QZ_EXPORT int qz_run_traced(qz_lattice *q, uint64_t n_sweeps, uint64_t trace_every,
                            uint64_t *host_B, uint64_t *host_flips)
{
    int rc = check_handle(q);
    if (rc != QZ_OK)
        return rc;
    if (trace_every == 0)
        return run_impl(q, n_sweeps, 0, nullptr, nullptr);
    if (!host_B && !host_flips)
        return fail(QZ_EINVAL, "null trace buffers");
    if (n_sweeps % trace_every)
        return fail(QZ_EINVAL, "n_sweeps must be a multiple of trace_every");
    unsigned long long *slots =
        reinterpret_cast<unsigned long long *>(q->base + q->map.trace_off);
    unsigned long long *fslots =
        reinterpret_cast<unsigned long long *>(q->base + q->map.flips_off);
    const uint64_t points = n_sweeps / trace_every;
    uint64_t done = 0;
    while (done < points) {
        const uint64_t chunk = std::min<uint64_t>(points - done, qz::kTraceCap);
        if (host_B)
            QZ_HIP(q, qz::fill_u64(q->st, slots, chunk, 0ull));
        if (host_flips)
            QZ_HIP(q, qz::fill_u64(q->st, fslots, chunk, 0ull));
        rc = run_impl(q, chunk * trace_every, trace_every, host_B ? slots : nullptr,
                      host_flips ? fslots : nullptr);
        if (rc != QZ_OK)
            return rc;
        if (host_B)
            QZ_HIP(q, hipMemcpyAsync(host_B + done, slots, chunk * 8, hipMemcpyDeviceToHost,
                                     q->st));
        if (host_flips)
            QZ_HIP(q, hipMemcpyAsync(host_flips + done, fslots, chunk * 8,
                                     hipMemcpyDeviceToHost, q->st));
        QZ_HIP(q, hipStreamSynchronize(q->st));
        done += chunk;
    }
    return QZ_OK;
}

QZ_EXPORT int qz_run(qz_lattice *q, uint64_t n_sweeps, uint64_t trace_every, uint64_t *host_trace)
{
    if (q && trace_every > 0 && !host_trace)
        return fail(QZ_EINVAL, "null trace buffer");
    return qz_run_traced(q, n_sweeps, trace_every, host_trace, nullptr);
}

QZ_EXPORT int qz_run_device_traced(qz_lattice *q, uint64_t n_sweeps, uint64_t trace_every,
                                   uint64_t *dev_B, uint64_t *dev_flips)
{
    int rc = check_handle(q);
    if (rc != QZ_OK)
        return rc;
    if (trace_every == 0)
        return run_impl(q, n_sweeps, 0, nullptr, nullptr);
    if (!dev_B && !dev_flips)
        return fail(QZ_EINVAL, "null trace buffers");
    if (n_sweeps % trace_every)
        return fail(QZ_EINVAL, "n_sweeps must be a multiple of trace_every");
    unsigned long long *slots = reinterpret_cast<unsigned long long *>(dev_B);
    unsigned long long *fslots = reinterpret_cast<unsigned long long *>(dev_flips);
    if (slots)
        QZ_HIP(q, qz::fill_u64(q->st, slots, n_sweeps / trace_every, 0ull));
    if (fslots)
        QZ_HIP(q, qz::fill_u64(q->st, fslots, n_sweeps / trace_every, 0ull));
    return run_impl(q, n_sweeps, trace_every, slots, fslots);
}

QZ_EXPORT int qz_run_device(qz_lattice *q, uint64_t n_sweeps, uint64_t trace_every,
                            uint64_t *dev_trace)
{
    if (q && trace_every > 0 && !dev_trace)
        return fail(QZ_EINVAL, "null trace buffer");
    return qz_run_device_traced(q, n_sweeps, trace_every, dev_trace, nullptr);
}

QZ_EXPORT int qz_run_device_at(qz_lattice *q, uint64_t n_sweeps, const uint64_t *at,
                               size_t n_at, uint64_t *dev_B, uint64_t *dev_flips)
{
    int rc = check_handle(q);
    if (rc != QZ_OK)
        return rc;
    if ((rc = check_list(at, n_at, n_sweeps)) != QZ_OK)
        return rc;
    unsigned long long *slots = reinterpret_cast<unsigned long long *>(dev_B);
    unsigned long long *fslots = reinterpret_cast<unsigned long long *>(dev_flips);
    if (n_at > 0 && !slots && !fslots)
        return fail(QZ_EINVAL, "null trace buffers");
    if (n_at > 0 && slots)
        QZ_HIP(q, qz::fill_u64(q->st, slots, n_at, 0ull));
    if (n_at > 0 && fslots)
        QZ_HIP(q, qz::fill_u64(q->st, fslots, n_at, 0ull));
    TracePlan plan;
    plan.at = at;
    plan.n_at = n_at;
    return run_plan(q, n_sweeps, plan, n_at > 0 ? slots : nullptr, n_at > 0 ? fslots : nullptr);
}

QZ_EXPORT int qz_run_at(qz_lattice *q, uint64_t n_sweeps, const uint64_t *at, size_t n_at,
                        uint64_t *host_B, uint64_t *host_flips)
{
    int rc = check_handle(q);
    if (rc != QZ_OK)
        return rc;
    if ((rc = check_list(at, n_at, n_sweeps)) != QZ_OK)
        return rc;
    if (n_at == 0)
        return run_impl(q, n_sweeps, 0, nullptr, nullptr);
    if (!host_B && !host_flips)
        return fail(QZ_EINVAL, "null trace buffers");
    unsigned long long *slots =
        reinterpret_cast<unsigned long long *>(q->base + q->map.trace_off);
    unsigned long long *fslots =
        reinterpret_cast<unsigned long long *>(q->base + q->map.flips_off);
    // runs of at most kTraceCap listed sweeps, each through the handle's rings
    uint64_t k0 = 0;
    size_t done = 0;
    while (done < n_at) {
        const size_t chunk = std::min<size_t>(n_at - done, qz::kTraceCap);
        // this piece ends just before the first listed sweep of the next one
        const uint64_t k1 = (done + chunk < n_at) ? at[done + chunk] : n_sweeps;
        std::vector<uint64_t> rel(chunk);
        for (size_t i = 0; i < chunk; ++i)
            rel[i] = at[done + i] - k0;
        if (host_B)
            QZ_HIP(q, qz::fill_u64(q->st, slots, chunk, 0ull));
        if (host_flips)
            QZ_HIP(q, qz::fill_u64(q->st, fslots, chunk, 0ull));
        TracePlan plan;
        plan.at = rel.data();
        plan.n_at = chunk;
        rc = run_plan(q, k1 - k0, plan, host_B ? slots : nullptr, host_flips ? fslots : nullptr);
        if (rc != QZ_OK)
            return rc;
        if (host_B)
            QZ_HIP(q, hipMemcpyAsync(host_B + done, slots, chunk * 8, hipMemcpyDeviceToHost,
                                     q->st));
        if (host_flips)
            QZ_HIP(q, hipMemcpyAsync(host_flips + done, fslots, chunk * 8,
                                     hipMemcpyDeviceToHost, q->st));
        QZ_HIP(q, hipStreamSynchronize(q->st));
        done += chunk;
        k0 = k1;
    }
    return QZ_OK;
}

QZ_EXPORT int qz_bonds(qz_lattice *q, uint64_t out_B_axes[3])
{
    int rc = check_handle(q);
    if (rc != QZ_OK)
        return rc;
    if (!out_B_axes)
        return fail(QZ_EINVAL, "null output");
    unsigned long long *c = counters(q);
    QZ_HIP(q, qz::fill_u64(q->st, c, 3, 0ull));
    if (q->layout == QZ_LAYOUT_I8)
        QZ_HIP(q, qz::i8_bonds(q->st, q->L, i8_spins(q), c));
    else
        QZ_HIP(q, qz::bit_bonds(q->st, q->L, bit_plane(q, q->cur, 0), bit_plane(q, q->cur, 1), c));
    unsigned long long h[3];
    QZ_HIP(q, hipMemcpyAsync(h, c, sizeof h, hipMemcpyDeviceToHost, q->st));
    QZ_HIP(q, hipStreamSynchronize(q->st));
    for (int a = 0; a < 3; ++a)
        out_B_axes[a] = h[a];
    return QZ_OK;
}

QZ_EXPORT int qz_bonds_device(qz_lattice *q, uint64_t *dev_B_axes)
{
    int rc = check_handle(q);
    if (rc != QZ_OK)
        return rc;
    if (!dev_B_axes || (reinterpret_cast<uintptr_t>(dev_B_axes) & 7u))
        return fail(QZ_EINVAL, "null or misaligned device output");
    unsigned long long *c = reinterpret_cast<unsigned long long *>(dev_B_axes);
    QZ_HIP(q, qz::fill_u64(q->st, c, 3, 0ull));
    if (q->layout == QZ_LAYOUT_I8)
        QZ_HIP(q, qz::i8_bonds(q->st, q->L, i8_spins(q), c));
    else
        QZ_HIP(q, qz::bit_bonds(q->st, q->L, bit_plane(q, q->cur, 0), bit_plane(q, q->cur, 1), c));
    return QZ_OK;
}

QZ_EXPORT int qz_corr(qz_lattice *q, int64_t *out_S, int64_t *out_M)
{
    int rc = check_handle(q);
    if (rc != QZ_OK)
        return rc;
    if (!out_S || !out_M)
        return fail(QZ_EINVAL, "null output");
    const uint32_t R = q->L / 2 + 1;
    const size_t nvals = 3 * (size_t)R + 1;
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(q->base + q->map.corr_off);
    QZ_HIP(q, qz::fill_u64(q->st, acc, nvals, 0ull));
    if (q->layout == QZ_LAYOUT_I8)
        QZ_HIP(q, qz::i8_corr(q->st, q->L, i8_spins(q), reinterpret_cast<long long *>(acc),
                              reinterpret_cast<long long *>(acc + 3 * R)));
    else
        // the idle copy (the next sweep overwrites it) serves as scratch
        QZ_HIP(q, qz::bit_corr(q->st, q->L, bit_plane(q, q->cur, 0), bit_plane(q, q->cur, 1), acc,
                               acc + 3 * R, bit_plane(q, 1 - q->cur, 0),
                               bit_plane(q, 1 - q->cur, 1)));
    unsigned long long *h = new (std::nothrow) unsigned long long[nvals];
    if (!h)
        return fail(QZ_ENOMEM, "host allocation failed");
    hipError_t e = hipMemcpyAsync(h, acc, nvals * 8, hipMemcpyDeviceToHost, q->st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(q->st);
    if (e != hipSuccess) {
        delete[] h;
        return device_fail(q, e, "qz_corr copy");
    }
    const int64_t N = (int64_t)n_sites(q->L);
    if (q->layout == QZ_LAYOUT_I8) {
        for (size_t k = 0; k < 3 * (size_t)R; ++k)
            out_S[k] = (int64_t)h[k];
        *out_M = (int64_t)h[3 * R];
    } else {
        // anti-aligned pair counts -> S = N - 2*anti; up-spin count -> M = 2*ones - N
        for (size_t k = 0; k < 3 * (size_t)R; ++k)
            out_S[k] = N - 2 * (int64_t)h[k];
        *out_M = 2 * (int64_t)h[3 * R] - N;
    }
    delete[] h;
    return QZ_OK;
}

QZ_EXPORT int qz_corr_noalloc(qz_lattice *q, int64_t *out_S, int64_t *out_M)
{
    int rc = check_handle(q);
    if (rc != QZ_OK)
        return rc;
    if (!out_S || !out_M)
        return fail(QZ_EINVAL, "null output");
    const uint32_t R = q->L / 2 + 1;
    const size_t nvals = 3 * (size_t)R + 1;
    if (nvals > kNoAllocWords)
        return fail(QZ_EINVAL, "L too large for the static correlation scratch "
                               "(3 (L/2 + 1) + 1 <= 8192 counters)");
    hipPointerAttribute_t attr;
    QZ_HIP(q, hipPointerGetAttributes(&attr, q->base));
    unsigned long long *acc = nullptr;
    if ((rc = scratch_on(attr.device, &acc)) != QZ_OK)
        return rc;
    // the array keeps the previous call's sums: clear them first (a kernel,
    // so that the call can also be captured into a graph)
    QZ_HIP(q, qz::fill_u64(q->st, acc, nvals, 0ull));
    if (q->layout == QZ_LAYOUT_I8)
        QZ_HIP(q, qz::i8_corr(q->st, q->L, i8_spins(q), reinterpret_cast<long long *>(acc),
                              reinterpret_cast<long long *>(acc + 3 * R)));
    else
        // no scratch copy: the x axis by funnel-rotated row pairs
        QZ_HIP(q, qz::bit_corr(q->st, q->L, bit_plane(q, q->cur, 0), bit_plane(q, q->cur, 1), acc,
                               acc + 3 * R, nullptr, nullptr));
    // straight into the caller's arrays, converted there
    QZ_HIP(q, hipMemcpyAsync(out_S, acc, 3 * (size_t)R * 8, hipMemcpyDeviceToHost, q->st));
    QZ_HIP(q, hipMemcpyAsync(out_M, acc + 3 * R, 8, hipMemcpyDeviceToHost, q->st));
    QZ_HIP(q, hipStreamSynchronize(q->st));
    if (q->layout == QZ_LAYOUT_BIT) {
        const int64_t N = (int64_t)n_sites(q->L);
        for (size_t k = 0; k < 3 * (size_t)R; ++k)
            out_S[k] = N - 2 * out_S[k];
        *out_M = 2 * *out_M - N;
    }
    return QZ_OK;
}

QZ_EXPORT int qz_time(const qz_lattice *q, uint64_t *t)
{
    if (!q || !t)
        return fail(QZ_EINVAL, "null argument");
    *t = q->t;
    return QZ_OK;
}

QZ_EXPORT int qz_download_spins(qz_lattice *q, int8_t *host)
{
    int rc = check_handle(q);
    if (rc != QZ_OK)
        return rc;
    if (!host)
        return fail(QZ_EINVAL, "null output");
    const uint32_t L = q->L;
    const uint64_t N = n_sites(L);
    if (q->layout == QZ_LAYOUT_I8) {
        QZ_HIP(q, hipMemcpyAsync(host, i8_spins(q), N, hipMemcpyDeviceToHost, q->st));
        QZ_HIP(q, hipStreamSynchronize(q->st));
        return QZ_OK;
    }
    int8_t *stage = reinterpret_cast<int8_t *>(q->base + q->map.stage_off);
    const uint64_t plane = (uint64_t)L * L;
    const uint32_t nzc = (uint32_t)std::max<uint64_t>(1, q->map.stage_bytes / plane);
    for (uint32_t z0 = 0; z0 < L; z0 += nzc) {
        const uint32_t nz = std::min<uint32_t>(nzc, L - z0);
        QZ_HIP(q, qz::bit_unpack(q->st, L, bit_plane(q, q->cur, 0), bit_plane(q, q->cur, 1), z0,
                                 nz, stage));
        QZ_HIP(q, hipMemcpyAsync(host + (uint64_t)z0 * plane, stage, (size_t)nz * plane,
                                 hipMemcpyDeviceToHost, q->st));
        QZ_HIP(q, hipStreamSynchronize(q->st));
    }
    return QZ_OK;
}

QZ_EXPORT int qz_upload_spins(qz_lattice *q, const int8_t *host, uint64_t t)
{
    int rc = check_handle(q);
    if (rc != QZ_OK)
        return rc;
    if (!host)
        return fail(QZ_EINVAL, "null input");
    const uint32_t L = q->L;
    const uint64_t N = n_sites(L);
    unsigned long long *bad = counters(q) + 3;
    QZ_HIP(q, qz::fill_u64(q->st, bad, 1, 0ull));
    if (q->layout == QZ_LAYOUT_I8) {
        QZ_HIP(q, hipMemcpyAsync(i8_spins(q), host, N, hipMemcpyHostToDevice, q->st));
        QZ_HIP(q, qz::i8_check_pm1(q->st, N, i8_spins(q), bad));
    } else {
        int8_t *stage = reinterpret_cast<int8_t *>(q->base + q->map.stage_off);
        const uint64_t plane = (uint64_t)L * L;
        const uint32_t nzc = (uint32_t)std::max<uint64_t>(1, q->map.stage_bytes / plane);
        for (uint32_t z0 = 0; z0 < L; z0 += nzc) {
            const uint32_t nz = std::min<uint32_t>(nzc, L - z0);
            QZ_HIP(q, hipMemcpyAsync(stage, host + (uint64_t)z0 * plane, (size_t)nz * plane,
                                     hipMemcpyHostToDevice, q->st));
            QZ_HIP(q, qz::bit_pack(q->st, L, bit_plane(q, q->cur, 0), bit_plane(q, q->cur, 1), z0,
                                   nz, stage, bad));
            // the stage is reused by the next chunk: wait for this pack to finish
            QZ_HIP(q, hipStreamSynchronize(q->st));
        }
    }
    unsigned long long nbad = 0;
    QZ_HIP(q, hipMemcpyAsync(&nbad, bad, 8, hipMemcpyDeviceToHost, q->st));
    QZ_HIP(q, hipStreamSynchronize(q->st));
    q->t = t;
    if (nbad)
        return fail(QZ_EINVAL, "uploaded spins must all be +1 or -1");
    return QZ_OK;
}

QZ_EXPORT int qz_download_window(qz_lattice *q, const uint32_t origin[3], uint32_t W, int8_t *host)
{
    int rc = check_handle(q);
    if (rc != QZ_OK)
        return rc;
    if (!origin || !host)
        return fail(QZ_EINVAL, "null argument");
    const uint32_t L = q->L;
    if (W < 1 || W > L)
        return fail(QZ_EINVAL, "window side must be in [1, L]");
    const uint32_t ox = origin[0] % L, oy = origin[1] % L, oz = origin[2] % L;
    int8_t *stage = reinterpret_cast<int8_t *>(q->base + q->map.stage_off);
    const uint64_t plane = (uint64_t)W * W;
    const uint32_t nzc = (uint32_t)std::max<uint64_t>(1, q->map.stage_bytes / plane);
    for (uint32_t lz0 = 0; lz0 < W; lz0 += nzc) {
        const uint32_t nz = std::min<uint32_t>(nzc, W - lz0);
        if (q->layout == QZ_LAYOUT_I8)
            QZ_HIP(q, qz::i8_window(q->st, L, i8_spins(q), ox, oy, oz, W, lz0, nz, stage));
        else
            QZ_HIP(q, qz::bit_window(q->st, L, bit_plane(q, q->cur, 0), bit_plane(q, q->cur, 1),
                                     ox, oy, oz, W, lz0, nz, stage));
        QZ_HIP(q, hipMemcpyAsync(host + (uint64_t)lz0 * plane, stage, (size_t)nz * plane,
                                 hipMemcpyDeviceToHost, q->st));
        QZ_HIP(q, hipStreamSynchronize(q->st));
    }
    return QZ_OK;
}

QZ_EXPORT int qz_set_tuning(qz_lattice *q, int V, int Ty, int Tz)
{
    if (!q)
        return fail(QZ_EINVAL, "null handle");
    if (q->layout != QZ_LAYOUT_BIT)
        return fail(QZ_EUNSUPPORTED, "only the bit layout has a tuning");
    qz::BitTuning t;
    t.V = V;
    t.Ty = Ty;
    t.Tz = Tz;
    if (!qz::bit_tuning_valid(q->L, t))
        return fail(QZ_EINVAL, "tuning does not fit this lattice size");
    q->tune = t;
    return QZ_OK;
}

QZ_EXPORT int qz_get_tuning(const qz_lattice *q, int out_V_Ty_Tz[3])
{
    if (!q || !out_V_Ty_Tz)
        return fail(QZ_EINVAL, "null argument");
    if (q->layout != QZ_LAYOUT_BIT)
        return fail(QZ_EUNSUPPORTED, "only the bit layout has a tuning");
    out_V_Ty_Tz[0] = q->tune.V;
    out_V_Ty_Tz[1] = q->tune.Ty;
    out_V_Ty_Tz[2] = q->tune.Tz;
    return QZ_OK;
}

QZ_EXPORT int qz_set_pass(qz_lattice *q, int sweeps, int V, int Ty, int Tz)
{
    if (!q)
        return fail(QZ_EINVAL, "null handle");
    if (q->layout != QZ_LAYOUT_BIT)
        return fail(QZ_EUNSUPPORTED, "only the bit layout has multi-sweep passes");
    if (sweeps == 1) {
        q->pass = 1;
        return QZ_OK;
    }
    if (sweeps != 2)
        return fail(QZ_EINVAL, "sweeps per pass must be 1 or 2");
    qz::BitTuning t = qz::bit_tuning2_default(q->L);
    if (V != 0 || Ty != 0 || Tz != 0) {
        t.V = V;
        t.Ty = Ty;
        t.Tz = Tz;
    }
    if (!qz::bit_tuning2_valid(q->L, t))
        return fail(QZ_EINVAL, "two-sweep tuning does not fit this lattice size");
    q->tune2 = t;
    q->pass = 2;
    return QZ_OK;
}

QZ_EXPORT int qz_get_pass(const qz_lattice *q, int out_sweeps_V_Ty_Tz[4])
{
    if (!q || !out_sweeps_V_Ty_Tz)
        return fail(QZ_EINVAL, "null argument");
    if (q->layout != QZ_LAYOUT_BIT)
        return fail(QZ_EUNSUPPORTED, "only the bit layout has multi-sweep passes");
    out_sweeps_V_Ty_Tz[0] = q->pass;
    out_sweeps_V_Ty_Tz[1] = q->tune2.V;
    out_sweeps_V_Ty_Tz[2] = q->tune2.Ty;
    out_sweeps_V_Ty_Tz[3] = q->tune2.Tz;
    return QZ_OK;
}

QZ_EXPORT int qz_set_cycle(qz_lattice *q, int cycle)
{
    if (!q)
        return fail(QZ_EINVAL, "null handle");
    if (cycle != QZ_CYCLE_01 && cycle != QZ_CYCLE_MIXED)
        return fail(QZ_EINVAL, "unknown cycle");
    q->mixed = cycle == QZ_CYCLE_MIXED;
    return QZ_OK;
}

// ---------------------------------------------------------------------------
// FFT correlation (qz_fft.hip).  Scratch: X | hipFFT work area | accumulators.
// ---------------------------------------------------------------------------
namespace {
size_t fft_x_bytes(uint32_t L) { return align256((size_t)L * L * qz::fft_pad(L) * 8); }
size_t fft_acc_bytes(uint32_t nb) { return align256((size_t)nb * 32 + 8); }
}  // namespace

QZ_EXPORT uint32_t qz_fft_nbins(uint32_t L) { return qz::fft_nbins(L); }

QZ_EXPORT int qz_fft_prepare(qz_lattice *q, size_t *scratch_bytes)
{
    int rc = check_handle(q);
    if (rc != QZ_OK)
        return rc;
    if (!scratch_bytes)
        return fail(QZ_EINVAL, "null output");
    if (!q->fft_ready) {
        const int n = (int)q->L;
        size_t w1 = 0, w2 = 0;
        if (hipfftCreate(&q->fft_fwd) != HIPFFT_SUCCESS)
            return fail(QZ_EDEVICE, "hipfftCreate failed");
        if (hipfftCreate(&q->fft_inv) != HIPFFT_SUCCESS) {
            hipfftDestroy(q->fft_fwd);
            return fail(QZ_EDEVICE, "hipfftCreate failed");
        }
        bool ok = hipfftSetAutoAllocation(q->fft_fwd, 0) == HIPFFT_SUCCESS &&
                  hipfftSetAutoAllocation(q->fft_inv, 0) == HIPFFT_SUCCESS &&
                  hipfftMakePlan3d(q->fft_fwd, n, n, n, HIPFFT_D2Z, &w1) == HIPFFT_SUCCESS &&
                  hipfftMakePlan3d(q->fft_inv, n, n, n, HIPFFT_Z2D, &w2) == HIPFFT_SUCCESS &&
                  hipfftSetStream(q->fft_fwd, q->st) == HIPFFT_SUCCESS &&
                  hipfftSetStream(q->fft_inv, q->st) == HIPFFT_SUCCESS;
        if (!ok) {
            hipfftDestroy(q->fft_fwd);
            hipfftDestroy(q->fft_inv);
            return fail(QZ_EDEVICE, "hipFFT plan creation failed");
        }
        q->fft_work = align256(std::max(w1, w2));
        q->fft_ready = true;
    }
    *scratch_bytes = fft_x_bytes(q->L) + q->fft_work + fft_acc_bytes(qz::fft_nbins(q->L));
    return QZ_OK;
}

QZ_EXPORT int qz_fft_corr(qz_lattice *q, void *dev_scratch, size_t bytes, double *out_C,
                          double *out_Sk, uint64_t *out_nr, uint64_t *out_nk, double *out_m)
{
    size_t need = 0;
    int rc = qz_fft_prepare(q, &need);
    if (rc != QZ_OK)
        return rc;
    if (!dev_scratch || (reinterpret_cast<uintptr_t>(dev_scratch) & 255u))
        return fail(QZ_EINVAL, "scratch must be non-null and 256-byte aligned");
    if (bytes < need)
        return fail(QZ_ENOMEM, "scratch smaller than qz_fft_prepare() reported");
    if (!out_C || !out_Sk || !out_nr || !out_nk || !out_m)
        return fail(QZ_EINVAL, "null output");
    const uint32_t L = q->L, nb = qz::fft_nbins(L);
    uint8_t *base = reinterpret_cast<uint8_t *>(dev_scratch);
    double *X = reinterpret_cast<double *>(base);
    void *work = base + fft_x_bytes(L);
    double *acc = reinterpret_cast<double *>(base + fft_x_bytes(L) + q->fft_work);
    double *c_sum = acc, *sk_sum = acc + nb;
    unsigned long long *c_cnt = reinterpret_cast<unsigned long long *>(acc + 2 * nb);
    unsigned long long *sk_cnt = c_cnt + nb;
    double *Mdev = acc + 4 * (size_t)nb;
    QZ_HIP(q, qz::fft_zero(q->st, acc, 4 * (size_t)nb + 1));
    if (q->layout == QZ_LAYOUT_I8)
        QZ_HIP(q, qz::fft_unpack(q->st, L, 0, i8_spins(q), nullptr, X));
    else
        QZ_HIP(q, qz::fft_unpack(q->st, L, 1, bit_plane(q, q->cur, 0), bit_plane(q, q->cur, 1), X));
    if (hipfftSetWorkArea(q->fft_fwd, work) != HIPFFT_SUCCESS ||
        hipfftExecD2Z(q->fft_fwd, reinterpret_cast<hipfftDoubleReal *>(X),
                      reinterpret_cast<hipfftDoubleComplex *>(X)) != HIPFFT_SUCCESS)
        return fail(QZ_EDEVICE, "forward FFT failed");
    QZ_HIP(q, qz::fft_power(q->st, L, X, nb, sk_sum, sk_cnt, Mdev));
    if (hipfftSetWorkArea(q->fft_inv, work) != HIPFFT_SUCCESS ||
        hipfftExecZ2D(q->fft_inv, reinterpret_cast<hipfftDoubleComplex *>(X),
                      reinterpret_cast<hipfftDoubleReal *>(X)) != HIPFFT_SUCCESS)
        return fail(QZ_EDEVICE, "inverse FFT failed");
    QZ_HIP(q, qz::fft_radial(q->st, L, X, nb, c_sum, c_cnt));
    std::vector<double> h(4 * (size_t)nb + 1);
    QZ_HIP(q, hipMemcpyAsync(h.data(), acc, h.size() * 8, hipMemcpyDeviceToHost, q->st));
    QZ_HIP(q, hipStreamSynchronize(q->st));
    const double N = (double)n_sites(L);
    const double m = h[4 * (size_t)nb] / N;
    const unsigned long long *cc = reinterpret_cast<const unsigned long long *>(h.data() + 2 * nb);
    const unsigned long long *kc = cc + nb;
    for (uint32_t b = 0; b < nb; ++b) {
        out_nr[b] = cc[b];
        out_nk[b] = kc[b];
        // R(d) = N * sum_i s_i s_{i+d}: the shell mean of R / N^2 is <s_i s_{i+d}>
        out_C[b] = cc[b] ? h[b] / ((double)cc[b] * N * N) - m * m : 0.0;
        out_Sk[b] = kc[b] ? h[nb + b] / ((double)kc[b] * N) : 0.0;
    }
    *out_m = m;
    return QZ_OK;
}

QZ_EXPORT int qz_set_double_checkerboard(qz_lattice *q, uint32_t B)
{
    if (!q)
        return fail(QZ_EINVAL, "null handle");
    if (B == 0) {
        q->dcb = 0;
        return QZ_OK;
    }
    if (q->layout != QZ_LAYOUT_BIT)
        return fail(QZ_EUNSUPPORTED, "the double checkerboard runs on the bit layout");
    if (B < 2 || (B & (B - 1)) || q->L % (2 * B))
        return fail(QZ_EINVAL, "B must be a power of two >= 2 with L % (2B) == 0");
    q->dcb = B;
    return QZ_OK;
}

QZ_EXPORT const char *qz_status_string(int status)
{
    switch (status) {
    case QZ_OK: return "ok";
    case QZ_EINVAL: return "invalid argument";
    case QZ_ENOMEM: return "device buffer too small";
    case QZ_EDEVICE: return "device error";
    case QZ_ESTATE: return "handle unusable after an earlier device failure";
    case QZ_EUNSUPPORTED: return "layout cannot hold this lattice size";
    default: return "unknown status";
    }
}

QZ_EXPORT const char *qz_last_error(void) { return g_last_error.c_str(); }
