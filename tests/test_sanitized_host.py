"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The batch planner (csrc/qz_batch_plan.hpp: buffer layout and the sweep
  launch's tile and group tables) for every batch side and every plane count
  that divides it, and for mixes and slot replacements: tables in range,
  every plane of every slot in exactly one sub-tile, groups of one size.
* The C oracle, driven through a few of each of its functions at small L, with
  the results compared against the ordinary build loaded by the tests.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_12161_amd", "csrc")
OUT = os.path.join(ROOT, "tests", "_pinbin")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc and g++")

PLAN_DRIVER = r"""
#include "qz_batch_plan.hpp"
#include <cstdio>
#include <cstdlib>
#include <set>
#include <utility>

#define CHECK(c) do { if (!(c)) { std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); std::abort(); } } while (0)

using namespace qz;

static void check_tables(const std::vector<uint32_t> &cap_L, const std::vector<uint32_t> &now_L,
                         const std::map<uint32_t, uint32_t> &tz, bool onchip = false)
{
    const size_t n = cap_L.size();
    BatchLayout lay;
    CHECK(batch_layout(cap_L.data(), n, 7, &lay));
    // slots disjoint, in order, before the tables; everything 256-aligned
    size_t end = 0;
    for (size_t i = 0; i < n; ++i) {
        CHECK(lay.rep_off[i] % 256 == 0 && lay.rep_off[i] >= end);
        end = lay.rep_off[i] + batch_replica_bytes(cap_L[i]);
        CHECK(batch_replica_bytes(now_L[i]) <= batch_replica_bytes(cap_L[i]));
    }
    CHECK(end <= lay.reps_off);
    const size_t offs[] = {lay.reps_off, lay.tiles_off, lay.groups_off, lay.onchip_off,
                           lay.trace_off, lay.counters_off, lay.corr_off, lay.stage_off,
                           lay.total};
    for (size_t k = 0; k + 1 < sizeof offs / sizeof offs[0]; ++k)
        CHECK(offs[k] % 256 == 0 && offs[k] <= offs[k + 1]);
    CHECK(lay.tiles_off - lay.reps_off >= n * sizeof(BatchReplica));
    CHECK(lay.groups_off - lay.tiles_off >= lay.max_tiles * sizeof(BatchTile));
    CHECK(lay.onchip_off - lay.groups_off >= lay.max_groups * sizeof(BatchGroup));
    CHECK(lay.trace_off - lay.onchip_off >= n * sizeof(uint32_t));
    CHECK(lay.counters_off - lay.trace_off >= n * 7 * 8);
    CHECK(lay.stage_bytes >= (size_t)lay.max_L * lay.max_L);
    std::vector<BatchTile> tiles;
    std::vector<BatchGroup> groups;
    std::vector<uint32_t> oc;
    size_t lds = 0;
    CHECK(batch_tables(now_L.data(), n, tz, lay.max_tiles, lay.max_groups, &tiles, &groups, &lds,
                       onchip, &oc));
    // the on-chip list: exactly the side-64 slots when enabled, in order
    std::vector<uint32_t> want_oc;
    for (size_t i = 0; onchip && i < n; ++i)
        if (now_L[i] == kOnchipSide)
            want_oc.push_back((uint32_t)i);
    CHECK(oc == want_oc);
    CHECK(tiles.size() <= lay.max_tiles && groups.size() <= lay.max_groups);
    CHECK(lds <= 60 * 1024);
    std::set<std::pair<uint32_t, uint32_t>> seen;
    size_t covered = 0;
    for (const BatchGroup &g : groups) {
        CHECK(g.first < g.last && g.last <= tiles.size() && g.first == covered);
        CHECK(g.last - g.first <= batch_subtiles_per_block(g.L));
        CHECK(g.nz >= 1 && g.L % g.nz == 0);
        auto it = tz.find(g.L);
        if (it != tz.end() && it->second >= 1 && g.L % it->second == 0)
            CHECK(g.nz == it->second);
        else
            CHECK(g.nz == batch_default_tz(g.L));
        for (uint32_t k = g.first; k < g.last; ++k) {
            const BatchTile &t = tiles[k];
            CHECK(t.slot < n && now_L[t.slot] == g.L);
            CHECK(t.z0 % g.nz == 0 && t.z0 + g.nz <= g.L);
            CHECK(seen.insert({t.slot, t.z0}).second);
        }
        covered = g.last;
    }
    CHECK(covered == tiles.size());
    size_t want = 0;
    for (size_t i = 0; i < n; ++i) {
        const uint32_t L = now_L[i];
        if (onchip && L == kOnchipSide)
            continue;
        auto it = tz.find(L);
        const bool given = it != tz.end() && it->second >= 1 && L % it->second == 0;
        want += L / (given ? it->second : batch_default_tz(L));
    }
    CHECK(seen.size() == want && tiles.size() == want);
}

int main()
{
    const uint32_t sides[] = {64, 128, 192, 256};
    size_t cases = 0;
    for (uint32_t L : sides) {
        CHECK(batch_size_ok(L));
        for (uint32_t tz = 1; tz <= L; ++tz) {
            if (L % tz)
                continue;
            for (size_t n : {1, 2, 3, 17}) {
                std::vector<uint32_t> Ls(n, L);
                check_tables(Ls, Ls, {{L, tz}});
                check_tables(Ls, Ls, {{L, tz}}, true);
                cases += 2;
            }
        }
    }
    for (uint32_t L : {32u, 96u, 320u, 512u, 0u})
        CHECK(!batch_size_ok(L));
    // the 584-replica mix, every plane count of each size at once, and
    // plane counts that do not divide L (the default is taken)
    std::vector<uint32_t> mix;
    for (int r = 0; r < 512; ++r) mix.push_back(64);
    for (int r = 0; r < 64; ++r) mix.push_back(128);
    for (int r = 0; r < 8; ++r) mix.push_back(256);
    for (uint32_t a : {1u, 2u, 4u, 8u, 16u, 32u, 64u})
        for (uint32_t b : {1u, 8u, 128u})
            for (uint32_t c : {1u, 4u, 256u, 3u, 0u}) {
                check_tables(mix, mix, {{64, a}, {128, b}, {256, c}});
                check_tables(mix, mix, {{64, a}, {128, b}, {256, c}}, true);
                cases += 2;
            }
    // slots refilled with smaller sides (serving), one plane per sub-tile
    std::vector<uint32_t> cap = {256, 256, 192, 128, 64, 256};
    std::vector<uint32_t> now = {64, 192, 128, 128, 64, 256};
    for (uint32_t tz : {1u, 2u, 8u}) {
        check_tables(cap, now, {{64, tz}, {128, tz}, {192, tz}, {256, tz}});
        check_tables(cap, now, {{64, tz}, {128, tz}, {192, tz}, {256, tz}}, true);
        cases += 2;
    }
    std::printf("ok %zu\n", cases);
    return 0;
}
"""

ORACLE_DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
void or_init(int L, uint64_t seed, int8_t *s);
void or_init_window(int L, uint64_t seed, int ox, int oy, int oz, int W, int8_t *w);
void or_run_cycle(int L, uint64_t seed, int8_t *s, uint64_t t0, uint64_t n, uint64_t every,
                  int64_t *trace, int mixed);
void or_bonds(int L, const int8_t *s, int64_t B[3]);
void or_corr(int L, const int8_t *s, int64_t *S, int64_t *M);
int64_t or_sweep_double(int L, int B, uint64_t seed, uint32_t t, int8_t *s);
int64_t or_sweep_double_mixed(int L, int B, uint64_t seed, uint32_t t, int8_t *s);
void or_window_advance_cycle(int L, uint64_t seed, int ox, int oy, int oz, int W, int8_t *w,
                             uint64_t t0, uint64_t T, int mixed);
int or_set_threads(int n);

static void dump(const char *tag, const int64_t *v, size_t n)
{
    printf("%s", tag);
    for (size_t i = 0; i < n; ++i)
        printf(" %lld", (long long)v[i]);
    printf("\n");
}

int main(void)
{
    or_set_threads(2);
    for (int L = 4; L <= 16; L += 4) {
        size_t N = (size_t)L * L * L;
        int8_t *s = malloc(N);
        int64_t tr[10], B[3], M, *S = malloc(sizeof(int64_t) * 3 * (L / 2 + 1));
        or_init(L, 7, s);
        or_run_cycle(L, 7, s, 0, 20, 2, tr, 0);
        dump("trace01", tr, 10);
        or_run_cycle(L, 7, s, 20, 20, 2, tr, 1);
        dump("tracemixed", tr, 10);
        or_bonds(L, s, B);
        dump("bonds", B, 3);
        or_corr(L, s, S, &M);
        dump("corr", S, 3 * (L / 2 + 1));
        dump("M", &M, 1);
        int64_t f[4];
        f[0] = or_sweep_double(L, 2, 7, 40, s);
        f[1] = or_sweep_double_mixed(L, 2, 7, 41, s);
        or_bonds(L, s, B);
        f[2] = B[0] + B[1] + B[2];
        f[3] = 0;
        dump("double", f, 4);
        int W = L;
        int8_t *w = malloc((size_t)W * W * W);
        or_init_window(L, 9, 1, 2, 3, W, w);
        or_window_advance_cycle(L, 9, 1, 2, 3, W, w, 0, 2, 1);
        int64_t sum = 0;
        for (size_t i = 0; i < (size_t)W * W * W; ++i)
            sum += w[i] * (int64_t)(i % 97);
        dump("window", &sum, 1);
        free(w);
        free(S);
        free(s);
    }
    return 0;
}
"""


def _build_and_run(name, src, compiler, extra):
    os.makedirs(OUT, exist_ok=True)
    ext = ".cpp" if compiler == "g++" else ".c"
    path = os.path.join(OUT, name + ext)
    with open(path, "w") as f:
        f.write(src)
    exe = os.path.join(OUT, name)
    subprocess.run([compiler, *SAN, *extra, path, "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env)
    assert res.returncode == 0, res.stderr[-4000:]
    return res.stdout


def test_batch_planner_under_sanitizers():
    out = _build_and_run("plan_san", PLAN_DRIVER, "g++", ["-std=c++17", "-I", CSRC])
    assert out.startswith("ok "), out


def test_oracle_under_sanitizers(orc):
    src = os.path.join(ROOT, "oracle", "quench_oracle.c")
    out = _build_and_run("oracle_san", ORACLE_DRIVER, "gcc",
                         ["-std=c11", "-fopenmp", src, "-lm"])
    lines = iter(out.strip().splitlines())

    def take(tag):
        parts = next(lines).split()
        assert parts[0] == tag
        return np.array([int(v) for v in parts[1:]], dtype=np.int64)

    for L in (4, 8, 12, 16):
        s = orc.init(L, 7)
        assert np.array_equal(take("trace01"), orc.run(s, 7, 0, 20, 2))
        assert np.array_equal(take("tracemixed"), orc.run(s, 7, 20, 20, 2, mixed=True))
        assert np.array_equal(take("bonds"), orc.bonds(s))
        S, M = orc.corr(s)
        assert np.array_equal(take("corr"), S.reshape(-1))
        assert take("M")[0] == M
        f0 = orc.sweep_double(s, 2, 7, 40)
        f1 = orc.sweep_double(s, 2, 7, 41, mixed=True)
        assert np.array_equal(take("double"), [f0, f1, int(orc.bonds(s).sum()), 0])
        w = orc.init_window(L, 9, (1, 2, 3), L)
        orc.window_advance(L, 9, (1, 2, 3), w, 0, 2, mixed=True)
        idx = np.arange(L ** 3, dtype=np.int64) % 97
        assert take("window")[0] == int((w.reshape(-1).astype(np.int64) * idx).sum())
