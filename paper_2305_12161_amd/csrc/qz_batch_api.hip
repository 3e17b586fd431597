// qz_batch_api.hip -- C ABI of the batched engine (include/quench.h, qz_batch_*).
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <set>
#include <new>
#include <string>
#include <vector>

#include "../../include/quench.h"
#include "qz_internal.hpp"

#define QZ_EXPORT extern "C" __attribute__((visibility("default")))

namespace qz {
// shared with qz_api.hip: sets the calling thread's last error
int set_error(int status, const char *msg);
}  // namespace qz

struct qz_batch {
    hipStream_t st;                          // caller's stream (all work)
    hipStream_t cap_st;                      // private stream used only to capture graphs
    uint8_t *base;
    size_t bytes;
    uint32_t every, cap;
    std::vector<qz_replica_spec> specs;
    std::vector<uint32_t> cap_L;             // side each slot's memory was sized for
    std::vector<qz::BatchReplica> host_reps;  // mirror of the device table
    qz::BatchReplica *d_reps;
    qz::BatchTile *d_tiles;
    qz::BatchGroup *d_groups;
    uint32_t *d_onchip;                      // slots run by the on-chip kernel (side 64)
    uint32_t ntiles, ngroups, nonchip;
    bool onchip;                             // side-64 slots on chip (else sub-tiles)
    size_t max_tiles, max_groups;            // capacity of the device tile / group tables
    size_t lds_bytes;
    int8_t *stage;
    size_t stage_bytes;
    unsigned long long *counters;            // 64 scratch counters
    unsigned long long *corr;                // correlation accumulators for the largest L
    std::map<uint32_t, uint32_t> tz;         // planes per sub-tile, by L
    uint32_t graph_sweeps;
    hipGraphExec_t graph;
    bool graph_ok;
    std::string tune_source;                 // "json", "autotune" or "set"
    bool failed;
    bool dirty;                              // host table newer than the device copy
};

namespace {

uint64_t nsites(uint32_t L) { return (uint64_t)L * L * L; }

int fail(int status, const std::string &msg) { return qz::set_error(status, msg.c_str()); }

int dev_fail(qz_batch *b, hipError_t e, const char *where)
{
    if (b)
        b->failed = true;
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    return fail(QZ_EDEVICE, buf);
}

#define BZ_HIP(b, call)                              \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess)                        \
            return dev_fail((b), e_, #call);         \
    } while (0)

uint32_t default_tz(uint32_t L) { return qz::batch_default_tz(L); }

// Sweeps per captured graph unless the tuning says otherwise.
constexpr uint32_t kDefaultGraphSweeps = 100;

// Layout of a slot list in the caller's buffer (qz_batch_plan.hpp).
bool plan(const qz_replica_spec *specs, size_t n, uint32_t cap, qz::BatchLayout *lay)
{
    std::vector<uint32_t> Ls(n);
    for (size_t i = 0; i < n; ++i)
        Ls[i] = specs[i].L;
    return qz::batch_layout(Ls.data(), n, cap, lay);
}

// Rebuild the tile and group tables for the slots' current sides and copy
// them to the device.
int build_tables(qz_batch *b)
{
    std::vector<uint32_t> Ls(b->specs.size());
    for (size_t i = 0; i < Ls.size(); ++i)
        Ls[i] = b->specs[i].L;
    std::vector<qz::BatchTile> tiles;
    std::vector<qz::BatchGroup> groups;
    std::vector<uint32_t> onchip;
    size_t lds = 0;
    if (!qz::batch_tables(Ls.data(), Ls.size(), b->tz, b->max_tiles, b->max_groups, &tiles,
                          &groups, &lds, b->onchip, &onchip))
        return fail(QZ_EINVAL, "tile tables exceed their capacity");
    b->ntiles = (uint32_t)tiles.size();
    b->ngroups = (uint32_t)groups.size();
    b->nonchip = (uint32_t)onchip.size();
    if (!onchip.empty())
        BZ_HIP(b, hipMemcpyAsync(b->d_onchip, onchip.data(), onchip.size() * sizeof(uint32_t),
                                 hipMemcpyHostToDevice, b->st));
    BZ_HIP(b, hipMemcpyAsync(b->d_tiles, tiles.data(), tiles.size() * sizeof(qz::BatchTile),
                             hipMemcpyHostToDevice, b->st));
    BZ_HIP(b, hipMemcpyAsync(b->d_groups, groups.data(), groups.size() * sizeof(qz::BatchGroup),
                             hipMemcpyHostToDevice, b->st));
    BZ_HIP(b, hipStreamSynchronize(b->st));
    b->lds_bytes = lds;
    return QZ_OK;
}

int push_reps(qz_batch *b)
{
    BZ_HIP(b, hipMemcpyAsync(b->d_reps, b->host_reps.data(),
                             b->host_reps.size() * sizeof(qz::BatchReplica),
                             hipMemcpyHostToDevice, b->st));
    BZ_HIP(b, hipStreamSynchronize(b->st));
    b->dirty = false;
    return QZ_OK;
}

// Most sweeps one group may span: the group clears its traced ring entries
// before its sweeps, so it may hold at most `cap` trace points per replica (a
// longer group would reuse an entry inside the group and add two counts).
uint32_t group_limit(const qz_batch *b)
{
    if (b->every == 0)
        return 0xFFFFFFFFu;
    const uint64_t lim = (uint64_t)b->cap * b->every;
    return lim > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)lim;
}

// Enqueue one group of k sweeps on stream s: clear the traced slots, k sweep
// launches (step = 0..k-1), then advance every active replica by k.
hipError_t enqueue_group(qz_batch *b, hipStream_t s, uint32_t k)
{
    hipError_t e = qz::batch_clear_trace(s, b->d_reps, (uint32_t)b->specs.size(), k, b->every,
                                         b->cap);
    if (e != hipSuccess)
        return e;
    // the side-64 replicas: all k sweeps in one launch, on chip
    e = qz::batch_onchip64(s, b->d_reps, b->d_onchip, b->nonchip, k, b->every, b->cap);
    if (e != hipSuccess)
        return e;
    qz::BatchArgs a;
    a.reps = b->d_reps;
    a.tiles = b->d_tiles;
    a.groups = b->d_groups;
    a.every = b->every;
    a.cap = b->cap;
    a.lds_bytes = b->lds_bytes;
    for (uint32_t j = 0; j < k; ++j) {
        a.step = j;
        e = qz::batch_sweep(s, a, b->ngroups);
        if (e != hipSuccess)
            return e;
    }
    return qz::batch_advance(s, b->d_reps, (uint32_t)b->specs.size(), k);
}

int ensure_graph(qz_batch *b)
{
    if (b->graph_ok || b->graph_sweeps == 0)
        return QZ_OK;
    hipGraph_t g = nullptr;
    BZ_HIP(b, hipStreamBeginCapture(b->cap_st, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_group(b, b->cap_st, b->graph_sweeps);
    hipError_t e2 = hipStreamEndCapture(b->cap_st, &g);
    if (e != hipSuccess)
        return dev_fail(b, e, "capturing the sweep graph");
    if (e2 != hipSuccess)
        return dev_fail(b, e2, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
        return dev_fail(b, e, "hipGraphInstantiate");
    b->graph_ok = true;
    return QZ_OK;
}

void drop_graph(qz_batch *b)
{
    if (b->graph_ok)
        (void)hipGraphExecDestroy(b->graph);
    b->graph_ok = false;
}

void release_streams(qz_batch *b)
{
    if (b->cap_st)
        (void)hipStreamDestroy(b->cap_st);
    b->cap_st = nullptr;
}

int check(qz_batch *b)
{
    if (!b)
        return fail(QZ_EINVAL, "null batch handle");
    if (b->failed)
        return fail(QZ_ESTATE, "batch unusable after an earlier device failure");
    return QZ_OK;
}

int check_slot(qz_batch *b, size_t slot)
{
    int rc = check(b);
    if (rc != QZ_OK)
        return rc;
    if (slot >= b->specs.size())
        return fail(QZ_EINVAL, "slot out of range");
    return QZ_OK;
}

// bring the host mirror's times up to date after device-side advances
int pull_reps(qz_batch *b)
{
    BZ_HIP(b, hipMemcpyAsync(b->host_reps.data(), b->d_reps,
                             b->host_reps.size() * sizeof(qz::BatchReplica),
                             hipMemcpyDeviceToHost, b->st));
    BZ_HIP(b, hipStreamSynchronize(b->st));
    return QZ_OK;
}

uint32_t *slot_plane(qz_batch *b, size_t slot, int copy, int colour)
{
    const qz::BatchReplica &r = b->host_reps[slot];
    const uint32_t L = b->specs[slot].L;
    return r.base + (size_t)(2 * copy + colour) * (nsites(L) / 64);
}

// ---- tuning text: {"graph_sweeps": G, "tz": {"64": 8, "128": 8, ...}} ----
// Both keys are optional; unknown keys are an error, so that a misspelt key
// is not silently ignored.
struct JsonIn {
    const char *p;
    void ws()
    {
        while (*p == ' ' || *p == '\n' || *p == '\t' || *p == '\r')
            ++p;
    }
    bool lit(char c)
    {
        ws();
        if (*p != c)
            return false;
        ++p;
        return true;
    }
    bool str(std::string *out)
    {
        ws();
        if (*p != '"')
            return false;
        const char *q = ++p;
        while (*p && *p != '"')
            ++p;
        if (*p != '"')
            return false;
        out->assign(q, p);
        ++p;
        return true;
    }
    bool num(uint64_t *out)
    {
        ws();
        if (*p < '0' || *p > '9')
            return false;
        uint64_t v = 0;
        while (*p >= '0' && *p <= '9') {
            v = v * 10 + (uint64_t)(*p - '0');
            if (v > 0xFFFFFFFFull)
                return false;
            ++p;
        }
        *out = v;
        return true;
    }
};

bool parse_tuning(const char *text, std::map<uint32_t, uint32_t> *tz, uint32_t *graph_sweeps,
                  bool *has_graph, bool *onchip, bool *has_onchip)
{
    JsonIn in{text};
    *has_graph = false;
    *has_onchip = false;
    if (!in.lit('{'))
        return false;
    if (in.lit('}'))
        return (in.ws(), *in.p == '\0');
    do {
        std::string key;
        if (!in.str(&key) || !in.lit(':'))
            return false;
        if (key == "graph_sweeps") {
            uint64_t v;
            if (!in.num(&v))
                return false;
            *graph_sweeps = (uint32_t)v;
            *has_graph = true;
        } else if (key == "onchip") {
            uint64_t v;
            if (!in.num(&v) || v > 1)
                return false;
            *onchip = v != 0;
            *has_onchip = true;
        } else if (key == "tz") {
            if (!in.lit('{'))
                return false;
            if (!in.lit('}')) {
                do {
                    std::string ks;
                    uint64_t v;
                    if (!in.str(&ks) || ks.empty() || ks.size() > 9 || !in.lit(':') || !in.num(&v))
                        return false;
                    for (char c : ks)
                        if (c < '0' || c > '9')
                            return false;
                    (*tz)[(uint32_t)std::stoul(ks)] = (uint32_t)v;
                } while (in.lit(','));
                if (!in.lit('}'))
                    return false;
            }
        } else {
            return false;
        }
    } while (in.lit(','));
    if (!in.lit('}'))
        return false;
    in.ws();
    return *in.p == '\0';
}

std::string tuning_text(const qz_batch *b)
{
    std::set<uint32_t> Ls;
    for (const auto &sp : b->specs)
        Ls.insert(sp.L);
    std::string o = "{\"source\": \"" + b->tune_source +
                    "\", \"graph_sweeps\": " + std::to_string(b->graph_sweeps) +
                    ", \"onchip\": " + (b->onchip ? "1" : "0") + ", \"tz\": {";
    bool first = true;
    for (uint32_t L : Ls) {
        auto it = b->tz.find(L);
        const uint32_t v = it != b->tz.end() ? it->second : default_tz(L);
        o += (first ? "\"" : ", \"") + std::to_string(L) + "\": " + std::to_string(v);
        first = false;
    }
    return o + "}}";
}

// Autotune: first whether the side-64 replicas run on chip, then, for each
// side that runs as sub-tiles, in turn, time whole-batch sweeps with each
// plane count per sub-tile that divides L and keep the fastest (the others
// held at their current choice).  The sweeps run on the drawn
// starts, which are drawn again afterwards: results never depend on this.
int autotune(qz_batch *b)
{
    std::set<uint32_t> Ls;
    for (const auto &sp : b->specs)
        Ls.insert(sp.L);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BZ_HIP(b, hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return dev_fail(b, e, "hipEventCreate");
    }
    int rc = QZ_OK;
    // groups as long as the graphs will be (up to 16 sweeps): the on-chip
    // kernel reads and writes its replicas once per group
    const uint32_t G = std::max<uint32_t>(
        1u, std::min<uint32_t>({b->graph_sweeps ? b->graph_sweeps : 1u, 16u, group_limit(b)}));
    const uint32_t timed = std::max<uint32_t>(1u, 16u / G);
    auto time_batch = [&](float *ms) -> int {
        hipError_t x = enqueue_group(b, b->st, G);
        if (x == hipSuccess)
            x = hipEventRecord(e0, b->st);
        for (uint32_t k = 0; x == hipSuccess && k < timed; ++k)
            x = enqueue_group(b, b->st, G);
        if (x == hipSuccess)
            x = hipEventRecord(e1, b->st);
        if (x == hipSuccess)
            x = hipEventSynchronize(e1);
        if (x == hipSuccess)
            x = hipEventElapsedTime(ms, e0, e1);
        return x == hipSuccess ? QZ_OK : dev_fail(b, x, "autotune timing");
    };
    // side-64 replicas: on chip (k sweeps per launch) or as sub-tiles
    if (Ls.count(qz::kOnchipSide)) {
        float ms[2] = {0.0f, 0.0f};
        for (int on = 0; on < 2 && rc == QZ_OK; ++on) {
            b->onchip = on != 0;
            if ((rc = build_tables(b)) == QZ_OK)
                rc = time_batch(&ms[on]);
        }
        b->onchip = ms[1] <= ms[0];
    }
    for (uint32_t L : Ls) {
        if (rc != QZ_OK)
            break;
        if (b->onchip && L == qz::kOnchipSide)
            continue;
        uint32_t best = default_tz(L);
        float best_ms = 0.0f;
        bool have = false;
        for (uint32_t tz : {2u, 4u, 8u, 16u, 32u}) {
            if (L % tz)
                continue;
            b->tz[L] = tz;
            if ((rc = build_tables(b)) != QZ_OK)
                break;
            float ms = 0.0f;
            if ((rc = time_batch(&ms)) != QZ_OK)
                break;
            if (!have || ms < best_ms) {
                best = tz;
                best_ms = ms;
                have = true;
            }
        }
        if (rc != QZ_OK)
            break;
        b->tz[L] = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == QZ_OK)
        rc = build_tables(b);
    return rc;
}

// Draw every slot's start and set its time to 0.
int draw_starts(qz_batch *b)
{
    for (size_t i = 0; i < b->specs.size(); ++i) {
        qz::BatchReplica &r = b->host_reps[i];
        r.t = 0;
        r.cur = 0;
        BZ_HIP(b, qz::bit_init(b->st, b->specs[i].L, b->specs[i].seed, slot_plane(b, i, 0, 0),
                               slot_plane(b, i, 0, 1)));
    }
    return push_reps(b);
}

}  // namespace

QZ_EXPORT size_t qz_batch_state_bytes(const qz_replica_spec *specs, size_t n, uint32_t trace_cap)
{
    if (!specs || n == 0)
        return 0;
    qz::BatchLayout lay;
    return plan(specs, n, trace_cap, &lay) ? lay.total : 0;
}

QZ_EXPORT int qz_batch_create(const qz_replica_spec *specs, size_t n, uint32_t trace_every,
                              uint32_t trace_cap, void *dev_mem, size_t dev_bytes,
                              void *hip_stream, const char *tuning_json, qz_batch **out)
{
    if (!out)
        return fail(QZ_EINVAL, "null output pointer");
    *out = nullptr;
    if (!specs || n == 0 || n > (1u << 20))
        return fail(QZ_EINVAL, "need 1 .. 2^20 replica specs");
    if (trace_every > 0 && trace_cap == 0)
        return fail(QZ_EINVAL, "trace_cap must be > 0 when tracing");
    for (size_t i = 0; i < n; ++i)
        if (!qz::batch_size_ok(specs[i].L))
            return fail(QZ_EUNSUPPORTED, "batched replicas need L % 64 == 0 and L <= 256");
    if (!dev_mem || (reinterpret_cast<uintptr_t>(dev_mem) & 255u))
        return fail(QZ_EINVAL, "device buffer must be non-null and 256-byte aligned");
    std::map<uint32_t, uint32_t> tz_in;
    uint32_t graph_in = 0;
    bool has_graph = false, onchip_in = true, has_onchip = false;
    if (tuning_json) {
        if (!parse_tuning(tuning_json, &tz_in, &graph_in, &has_graph, &onchip_in, &has_onchip))
            return fail(QZ_EINVAL, "tuning_json is not of the form {\"graph_sweeps\": G, "
                                   "\"onchip\": 0 | 1, \"tz\": {\"L\": Tz, ...}}");
        for (const auto &kv : tz_in)
            if (!qz::batch_size_ok(kv.first) || kv.second == 0 || kv.first % kv.second)
                return fail(QZ_EINVAL, "tuning_json: each Tz must divide its L");
    }
    qz::BatchLayout lay;
    plan(specs, n, trace_cap, &lay);
    if (dev_bytes < lay.total)
        return fail(QZ_ENOMEM, "device buffer smaller than qz_batch_state_bytes()");
    qz_batch *b = new (std::nothrow) qz_batch();
    if (!b)
        return fail(QZ_ENOMEM, "host allocation failed");
    b->st = reinterpret_cast<hipStream_t>(hip_stream);
    b->cap_st = nullptr;
    b->base = reinterpret_cast<uint8_t *>(dev_mem);
    b->bytes = dev_bytes;
    b->every = trace_every;
    b->cap = trace_every ? trace_cap : 1;
    b->specs.assign(specs, specs + n);
    b->cap_L.resize(n);
    for (size_t i = 0; i < n; ++i)
        b->cap_L[i] = specs[i].L;
    b->d_reps = reinterpret_cast<qz::BatchReplica *>(b->base + lay.reps_off);
    b->d_tiles = reinterpret_cast<qz::BatchTile *>(b->base + lay.tiles_off);
    b->d_groups = reinterpret_cast<qz::BatchGroup *>(b->base + lay.groups_off);
    b->d_onchip = reinterpret_cast<uint32_t *>(b->base + lay.onchip_off);
    b->nonchip = 0;
    b->onchip = has_onchip ? onchip_in : true;
    b->max_tiles = lay.max_tiles;
    b->max_groups = lay.max_groups;
    b->stage = reinterpret_cast<int8_t *>(b->base + lay.stage_off);
    b->stage_bytes = lay.stage_bytes;
    b->counters = reinterpret_cast<unsigned long long *>(b->base + lay.counters_off);
    b->corr = reinterpret_cast<unsigned long long *>(b->base + lay.corr_off);
    b->graph_sweeps = std::min<uint32_t>(has_graph ? graph_in : kDefaultGraphSweeps,
                                         group_limit(b));
    b->graph_ok = false;
    b->failed = false;
    b->tz = tz_in;
    b->tune_source = tuning_json ? "json" : "autotune";
    b->host_reps.resize(n);
    unsigned long long *traces = reinterpret_cast<unsigned long long *>(b->base + lay.trace_off);
    for (size_t i = 0; i < n; ++i) {
        qz::BatchReplica &r = b->host_reps[i];
        r.base = reinterpret_cast<uint32_t *>(b->base + lay.rep_off[i]);
        r.trace = trace_every ? traces + i * (size_t)trace_cap : nullptr;
        r.seed = specs[i].seed;
        r.t = 0;
        r.t_max = specs[i].t_max;
        r.cur = 0;
        r.active = 1;
    }
    hipError_t e = hipStreamCreateWithFlags(&b->cap_st, hipStreamNonBlocking);
    if (e != hipSuccess) {
        int rc = dev_fail(nullptr, e, "hipStreamCreateWithFlags");
        delete b;
        return rc;
    }
    int rc = build_tables(b);
    if (rc == QZ_OK)
        rc = draw_starts(b);
    if (rc == QZ_OK && !tuning_json) {
        // no tuning given: time the candidates on the drawn starts, then draw
        // the starts again
        rc = autotune(b);
        if (rc == QZ_OK)
            rc = draw_starts(b);
    }
    if (rc != QZ_OK) {
        release_streams(b);
        delete b;
        return rc;
    }
    *out = b;
    return QZ_OK;
}

QZ_EXPORT int qz_batch_destroy(qz_batch *b)
{
    if (!b)
        return fail(QZ_EINVAL, "null batch handle");
    drop_graph(b);
    release_streams(b);
    delete b;
    return QZ_OK;
}

QZ_EXPORT int qz_batch_set_tuning(qz_batch *b, uint32_t L, uint32_t Tz, uint32_t graph_sweeps)
{
    int rc = check(b);
    if (rc != QZ_OK)
        return rc;
    if (Tz != 0) {
        if (!qz::batch_size_ok(L) || L % Tz)
            return fail(QZ_EINVAL, "Tz must divide L");
        b->tz[L] = Tz;
    }
    b->graph_sweeps = std::min<uint32_t>(graph_sweeps, group_limit(b));
    b->tune_source = "set";
    drop_graph(b);
    return build_tables(b);
}

namespace {
// Advance every active slot by n sweeps (asynchronous): graph replays of
// graph_sweeps sweeps, then the rest as one or more plain groups.
int run_sweeps(qz_batch *b, uint64_t n_sweeps)
{
    int rc;
    if (b->dirty) {
        rc = push_reps(b);
        if (rc != QZ_OK)
            return rc;
    }
    uint64_t left = n_sweeps;
    if (b->graph_sweeps > 0 && left >= b->graph_sweeps) {
        rc = ensure_graph(b);
        if (rc != QZ_OK)
            return rc;
        while (left >= b->graph_sweeps) {
            BZ_HIP(b, hipGraphLaunch(b->graph, b->st));
            left -= b->graph_sweeps;
        }
    }
    while (left > 0) {
        const uint32_t k = (uint32_t)std::min<uint64_t>(left, group_limit(b));
        BZ_HIP(b, enqueue_group(b, b->st, k));
        left -= k;
    }
    return QZ_OK;
}
}  // namespace

QZ_EXPORT int qz_batch_run(qz_batch *b, uint64_t n_sweeps, uint64_t trace_every,
                           uint64_t *host_traces)
{
    int rc = check(b);
    if (rc != QZ_OK)
        return rc;
    if (trace_every == 0 || host_traces == nullptr)
        return run_sweeps(b, n_sweeps);
    if (b->every == 0 || trace_every != b->every)
        return fail(QZ_EINVAL, "trace_every must equal the batch's trace_every");
    const size_t n = b->specs.size();
    const uint64_t every = b->every;
    const uint64_t P = (n_sweeps + every - 1) / every;     // entries per slot
    for (size_t i = 0; i < n * P; ++i)
        host_traces[i] = ~0ull;
    if ((rc = pull_reps(b)) != QZ_OK)
        return rc;
    // per slot: first traced time tau at or after t0, and where the run ends
    std::vector<uint64_t> t0(n), tau(n), t_end(n);
    for (size_t i = 0; i < n; ++i) {
        const qz::BatchReplica &r = b->host_reps[i];
        uint64_t m = r.active ? n_sweeps : 0;
        if (r.t_max > 0)
            m = r.t >= r.t_max ? 0 : std::min<uint64_t>(m, r.t_max - r.t);
        t0[i] = r.t;
        tau[i] = (r.t + every - 1) / every * every;
        t_end[i] = r.t + m;
    }
    // pieces of at most cap * every sweeps, so that no ring entry of a piece
    // is overwritten before it is read
    const uint64_t piece = (uint64_t)b->cap * every;
    std::vector<unsigned long long> ring((size_t)b->cap * n);
    unsigned long long *d_ring = b->host_reps[0].trace;   // the slots' rings are contiguous
    for (uint64_t done = 0; done < n_sweeps;) {
        const uint64_t m = std::min<uint64_t>(piece, n_sweeps - done);
        if ((rc = run_sweeps(b, m)) != QZ_OK)
            return rc;
        BZ_HIP(b, hipMemcpyAsync(ring.data(), d_ring, ring.size() * 8, hipMemcpyDeviceToHost,
                                 b->st));
        BZ_HIP(b, hipStreamSynchronize(b->st));
        for (size_t i = 0; i < n; ++i) {
            const uint64_t a = std::max(tau[i], t0[i] + done);
            const uint64_t z = std::min(t_end[i], t0[i] + done + m);
            for (uint64_t t = (a + every - 1) / every * every; t < z; t += every)
                host_traces[i * P + (t - tau[i]) / every] = ring[i * b->cap + (t / every) % b->cap];
        }
        done += m;
    }
    return pull_reps(b);
}

QZ_EXPORT int qz_batch_sync(qz_batch *b)
{
    int rc = check(b);
    if (rc != QZ_OK)
        return rc;
    BZ_HIP(b, hipStreamSynchronize(b->st));
    return pull_reps(b);
}

QZ_EXPORT int qz_batch_slot_time(qz_batch *b, size_t slot, uint64_t *t)
{
    int rc = check_slot(b, slot);
    if (rc != QZ_OK)
        return rc;
    if (!t)
        return fail(QZ_EINVAL, "null output");
    rc = pull_reps(b);
    if (rc != QZ_OK)
        return rc;
    *t = b->host_reps[slot].t;
    return QZ_OK;
}

QZ_EXPORT int qz_batch_slot_reset(qz_batch *b, size_t slot, uint64_t seed)
{
    int rc = check_slot(b, slot);
    if (rc != QZ_OK)
        return rc;
    rc = pull_reps(b);
    if (rc != QZ_OK)
        return rc;
    qz::BatchReplica &r = b->host_reps[slot];
    r.seed = seed;
    r.t = 0;
    r.cur = 0;
    r.active = 1;
    b->specs[slot].seed = seed;
    BZ_HIP(b, qz::bit_init(b->st, b->specs[slot].L, seed, slot_plane(b, slot, 0, 0),
                           slot_plane(b, slot, 0, 1)));
    return push_reps(b);
}

QZ_EXPORT int qz_batch_slot_replace(qz_batch *b, size_t slot, const qz_replica_spec *spec)
{
    int rc = check_slot(b, slot);
    if (rc != QZ_OK)
        return rc;
    if (!spec)
        return fail(QZ_EINVAL, "null replica spec");
    if (!qz::batch_size_ok(spec->L))
        return fail(QZ_EUNSUPPORTED, "batched replicas need L % 64 == 0 and L <= 256");
    if (spec->L > b->cap_L[slot])
        return fail(QZ_EINVAL, "the slot's memory was sized for a smaller L");
    rc = pull_reps(b);
    if (rc != QZ_OK)
        return rc;
    const bool new_L = spec->L != b->specs[slot].L;
    b->specs[slot] = *spec;
    qz::BatchReplica &r = b->host_reps[slot];
    r.seed = spec->seed;
    r.t = 0;
    r.t_max = spec->t_max;
    r.cur = 0;
    r.active = 1;
    if (new_L) {
        // the launch's tiles and groups follow the slots' sides
        drop_graph(b);
        if ((rc = build_tables(b)) != QZ_OK)
            return rc;
    }
    BZ_HIP(b, qz::bit_init(b->st, spec->L, spec->seed, slot_plane(b, slot, 0, 0),
                           slot_plane(b, slot, 0, 1)));
    return push_reps(b);
}

QZ_EXPORT int qz_batch_tuning_json(const qz_batch *b, char *buf, size_t len)
{
    if (!b || !buf)
        return fail(QZ_EINVAL, "null argument");
    const std::string t = tuning_text(b);
    if (t.size() + 1 > len)
        return fail(QZ_EINVAL, "buffer too small for the tuning text");
    memcpy(buf, t.c_str(), t.size() + 1);
    return QZ_OK;
}

QZ_EXPORT int qz_batch_slot_active(qz_batch *b, size_t slot, int active)
{
    int rc = check_slot(b, slot);
    if (rc != QZ_OK)
        return rc;
    rc = pull_reps(b);
    if (rc != QZ_OK)
        return rc;
    b->host_reps[slot].active = active ? 1u : 0u;
    return push_reps(b);
}

QZ_EXPORT int qz_batch_trace(qz_batch *b, size_t slot, uint64_t t_from, uint64_t count,
                             uint64_t *host)
{
    int rc = check_slot(b, slot);
    if (rc != QZ_OK)
        return rc;
    if (b->every == 0)
        return fail(QZ_EINVAL, "the batch was created without a trace");
    if (!host && count)
        return fail(QZ_EINVAL, "null output");
    if (t_from % b->every)
        return fail(QZ_EINVAL, "t_from must be a multiple of trace_every");
    rc = pull_reps(b);
    if (rc != QZ_OK)
        return rc;
    const uint64_t tnow = b->host_reps[slot].t;
    // B(t) is recorded by sweep t, so times up to tnow - 1 are available; the
    // ring holds the last cap of them
    const uint64_t k_from = t_from / b->every;
    if (count > 0) {
        const uint64_t k_last = k_from + count - 1;
        if (k_last * b->every >= tnow)
            return fail(QZ_EINVAL, "trace requested beyond the slot's current time");
        const uint64_t k_newest = (tnow - 1) / b->every;
        if (k_newest - k_from >= b->cap)
            return fail(QZ_EINVAL, "trace entries already overwritten in the ring");
    }
    std::vector<unsigned long long> ring(b->cap);
    BZ_HIP(b, hipMemcpyAsync(ring.data(), b->host_reps[slot].trace, (size_t)b->cap * 8,
                             hipMemcpyDeviceToHost, b->st));
    BZ_HIP(b, hipStreamSynchronize(b->st));
    for (uint64_t i = 0; i < count; ++i)
        host[i] = ring[(k_from + i) % b->cap];
    return QZ_OK;
}

QZ_EXPORT int qz_batch_download(qz_batch *b, size_t slot, int8_t *host)
{
    int rc = check_slot(b, slot);
    if (rc != QZ_OK)
        return rc;
    if (!host)
        return fail(QZ_EINVAL, "null output");
    rc = pull_reps(b);
    if (rc != QZ_OK)
        return rc;
    const uint32_t L = b->specs[slot].L;
    const int c = (int)b->host_reps[slot].cur;
    const uint64_t plane = (uint64_t)L * L;
    const uint32_t nzc = (uint32_t)std::max<uint64_t>(1, b->stage_bytes / plane);
    for (uint32_t z0 = 0; z0 < L; z0 += nzc) {
        const uint32_t nz = std::min<uint32_t>(nzc, L - z0);
        BZ_HIP(b, qz::bit_unpack(b->st, L, slot_plane(b, slot, c, 0), slot_plane(b, slot, c, 1),
                                 z0, nz, b->stage));
        BZ_HIP(b, hipMemcpyAsync(host + z0 * plane, b->stage, (size_t)nz * plane,
                                 hipMemcpyDeviceToHost, b->st));
        BZ_HIP(b, hipStreamSynchronize(b->st));
    }
    return QZ_OK;
}

QZ_EXPORT int qz_batch_bonds(qz_batch *b, size_t slot, uint64_t out_B_axes[3])
{
    int rc = check_slot(b, slot);
    if (rc != QZ_OK)
        return rc;
    if (!out_B_axes)
        return fail(QZ_EINVAL, "null output");
    rc = pull_reps(b);
    if (rc != QZ_OK)
        return rc;
    const uint32_t L = b->specs[slot].L;
    const int c = (int)b->host_reps[slot].cur;
    BZ_HIP(b, qz::fill_u64(b->st, b->counters, 3, 0ull));
    BZ_HIP(b, qz::bit_bonds(b->st, L, slot_plane(b, slot, c, 0), slot_plane(b, slot, c, 1),
                            b->counters));
    unsigned long long h[3];
    BZ_HIP(b, hipMemcpyAsync(h, b->counters, sizeof h, hipMemcpyDeviceToHost, b->st));
    BZ_HIP(b, hipStreamSynchronize(b->st));
    for (int a = 0; a < 3; ++a)
        out_B_axes[a] = h[a];
    return QZ_OK;
}

QZ_EXPORT int qz_batch_corr(qz_batch *b, size_t slot, int64_t *out_S, int64_t *out_M)
{
    int rc = check_slot(b, slot);
    if (rc != QZ_OK)
        return rc;
    if (!out_S || !out_M)
        return fail(QZ_EINVAL, "null output");
    rc = pull_reps(b);
    if (rc != QZ_OK)
        return rc;
    const uint32_t L = b->specs[slot].L, R = L / 2 + 1;
    const int c = (int)b->host_reps[slot].cur;
    BZ_HIP(b, qz::fill_u64(b->st, b->corr, 3 * (size_t)R + 1, 0ull));
    // the replica's idle copy (its next sweep overwrites it) serves as scratch
    BZ_HIP(b, qz::bit_corr(b->st, L, slot_plane(b, slot, c, 0), slot_plane(b, slot, c, 1), b->corr,
                           b->corr + 3 * R, slot_plane(b, slot, 1 - c, 0),
                           slot_plane(b, slot, 1 - c, 1)));
    std::vector<unsigned long long> h(3 * (size_t)R + 1);
    BZ_HIP(b, hipMemcpyAsync(h.data(), b->corr, h.size() * 8, hipMemcpyDeviceToHost, b->st));
    BZ_HIP(b, hipStreamSynchronize(b->st));
    const int64_t N = (int64_t)nsites(L);
    for (size_t k = 0; k < 3 * (size_t)R; ++k)
        out_S[k] = N - 2 * (int64_t)h[k];
    *out_M = 2 * (int64_t)h[3 * R] - N;
    return QZ_OK;
}
