// qz_batch_plan.hpp -- host-side planning of a replica batch: where each slot
// and table lives in the caller's buffer, and how one sweep launch is cut into
// sub-tiles and workgroups.  Plain C++ with no HIP types, so that the planner
// can also be built and checked on its own on the CPU.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <vector>

namespace qz {

constexpr uint32_t kBatchBlock = 256;   // lanes per workgroup of the batch sweep

struct BatchReplica {
    uint32_t *base;                 // copy k, colour c plane at base + (2k + c) * L*L*(L/64) words
    unsigned long long *trace;      // bond-count ring (cap slots), or null
    uint64_t seed;
    uint64_t t;                     // time at the start of the current group of sweeps
    uint64_t t_max;                 // the replica stops at this time (0: never)
    uint32_t cur;                   // copy holding the state at time t
    uint32_t active;                // 0: skipped by the sweeps
};
struct BatchTile {
    uint32_t slot;                  // replica
    uint32_t z0;                    // first plane
};
struct BatchGroup {                 // the sub-tiles of one workgroup: same L and plane count
    uint32_t L, nz, first, last;    // tiles [first, last)
};

// A lane holds a quad of words (one Philox block of tie bits); a workgroup
// runs kBatchBlock / Q whole-plane sub-tiles of one size, Q = quads per plane.
inline uint32_t batch_subtiles_per_block(uint32_t L)
{
    const uint32_t Q = L * (L / 64) / 4;
    return Q >= kBatchBlock ? 1u : kBatchBlock / Q;
}

// LDS of one workgroup: two buffers of both colours' planes per sub-tile.
inline size_t batch_lds_bytes(uint32_t L)
{
    return (size_t)batch_subtiles_per_block(L) * 4 * ((size_t)L * (L / 64)) * 4;
}

// Sizes the batch engine takes: L % 64 == 0, a plane's quads fit one
// workgroup, and its LDS stays within 60 KiB.
inline bool batch_size_ok(uint32_t L)
{
    if (L < 64 || L % 64)
        return false;
    const uint32_t Q = L * (L / 64) / 4;
    if (Q > kBatchBlock)
        return false;
    return batch_lds_bytes(L) <= 60 * 1024;
}

// Planes per sub-tile unless tuned: short z-chunks give a batch launch enough
// workgroups to fill the chip.
inline uint32_t batch_default_tz(uint32_t L) { return L % 8 == 0 ? 8u : 1u; }

inline size_t batch_align256(size_t v) { return (v + 255) & ~size_t(255); }
inline size_t batch_replica_bytes(uint32_t L)
{
    return batch_align256((size_t)((uint64_t)L * L * L / 8) * 2);
}

// Byte offsets of everything in the caller's buffer.  The tile and group
// tables are sized for the smallest plane count per sub-tile (one plane): L
// tiles per slot at most, and never more groups than tiles.
struct BatchLayout {
    std::vector<size_t> rep_off;
    size_t reps_off, tiles_off, groups_off, onchip_off, trace_off, counters_off, corr_off,
        stage_off;
    size_t stage_bytes, total;
    uint32_t max_L;
    size_t max_tiles, max_groups;
};

inline bool batch_layout(const uint32_t *Ls, size_t n, uint32_t cap, BatchLayout *lay)
{
    size_t off = 0;
    lay->rep_off.resize(n);
    lay->max_L = 0;
    lay->max_tiles = 0;
    for (size_t i = 0; i < n; ++i) {
        const uint32_t L = Ls[i];
        if (!batch_size_ok(L))
            return false;
        lay->rep_off[i] = off;
        off += batch_replica_bytes(L);
        lay->max_L = std::max(lay->max_L, L);
        lay->max_tiles += L;
    }
    lay->max_groups = lay->max_tiles;
    lay->reps_off = off;
    off = batch_align256(off + n * sizeof(BatchReplica));
    lay->tiles_off = off;
    off = batch_align256(off + lay->max_tiles * sizeof(BatchTile));
    lay->groups_off = off;
    off = batch_align256(off + lay->max_groups * sizeof(BatchGroup));
    lay->onchip_off = off;                      // slot list of the on-chip kernel
    off = batch_align256(off + n * sizeof(uint32_t));
    lay->trace_off = off;
    off = batch_align256(off + n * (size_t)cap * 8);
    lay->counters_off = off;
    off = batch_align256(off + 64 * 8);
    lay->corr_off = off;
    off = batch_align256(off + (size_t)(3 * (lay->max_L / 2 + 1) + 1) * 8);
    lay->stage_off = off;
    const uint64_t NL = (uint64_t)lay->max_L * lay->max_L * lay->max_L;
    lay->stage_bytes = std::min<size_t>((size_t)NL, size_t(4) << 20);
    lay->stage_bytes = std::max<size_t>(lay->stage_bytes, (size_t)lay->max_L * lay->max_L);
    off = batch_align256(off + lay->stage_bytes);
    lay->total = off;
    return true;
}

// Side of the replicas the on-chip kernel can hold (both colour planes in
// one workgroup's LDS).
constexpr uint32_t kOnchipSide = 64;

// The sweep launch's tables for the slots' current sides: slots grouped by L,
// each cut into sub-tiles of Tz planes (tz[L], else the default; a value that
// does not divide L falls back to the default), S sub-tiles of one L per
// workgroup.  With onchip set, the slots of side 64 go to the on-chip
// kernel's list instead.  Returns false, leaving the outputs unspecified, if
// the tables would exceed their capacity.  lds_bytes receives the largest
// workgroup LDS of the sub-tile launch.
inline bool batch_tables(const uint32_t *slot_L, size_t n, const std::map<uint32_t, uint32_t> &tz,
                         size_t max_tiles, size_t max_groups, std::vector<BatchTile> *tiles,
                         std::vector<BatchGroup> *groups, size_t *lds_bytes, bool onchip,
                         std::vector<uint32_t> *onchip_slots)
{
    std::map<uint32_t, std::vector<uint32_t>> by_L;
    onchip_slots->clear();
    for (size_t i = 0; i < n; ++i) {
        if (onchip && slot_L[i] == kOnchipSide)
            onchip_slots->push_back((uint32_t)i);
        else
            by_L[slot_L[i]].push_back((uint32_t)i);
    }
    tiles->clear();
    groups->clear();
    *lds_bytes = 0;
    for (auto &kv : by_L) {
        const uint32_t L = kv.first;
        auto it = tz.find(L);
        uint32_t nz = it != tz.end() ? it->second : batch_default_tz(L);
        if (nz < 1 || L % nz)
            nz = batch_default_tz(L);
        const uint32_t S = batch_subtiles_per_block(L);
        const size_t start = tiles->size();
        for (uint32_t slot : kv.second)
            for (uint32_t z0 = 0; z0 < L; z0 += nz)
                tiles->push_back({slot, z0});
        for (size_t f = start; f < tiles->size(); f += S) {
            BatchGroup g;
            g.L = L;
            g.nz = nz;
            g.first = (uint32_t)f;
            g.last = (uint32_t)std::min(tiles->size(), f + S);
            groups->push_back(g);
        }
        *lds_bytes = std::max(*lds_bytes, batch_lds_bytes(L));
        if (tiles->size() > max_tiles || groups->size() > max_groups)
            return false;
    }
    return true;
}

}  // namespace qz
