"""Pins of the CPU oracle against what the paper and mathematics fix.

Every check here is independent of the oracle's own code: library Philox
implementations (torch, rocRAND) used as black boxes, brute-force energy
recomputation, closed forms for special states, conservation identities and
numpy's FFT.
"""
import json
import os

import numpy as np
import pytest

from conftest import rng_rows
from paper_2305_12161_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# independent helpers (numpy, written for the tests)
# --------------------------------------------------------------------------
def energy(s):
    """E = -sum over nearest-neighbour bonds of s_i s_j (J = 1, periodic)."""
    s = s.astype(np.int64)
    return -int(sum((s * np.roll(s, -1, axis=ax)).sum() for ax in range(3)))


def antialigned(s):
    s = s.astype(np.int64)
    a = np.zeros_like(s)
    for ax in range(3):
        for sh in (1, -1):
            a += (np.roll(s, sh, axis=ax) != s)
    return a


def colour(L):
    z, y, x = np.indices((L, L, L))
    return (x + y + z) % 2


def colour_index(L):
    z, y, x = np.indices((L, L, L))
    return x // 2 + (L // 2) * (y + L * z)


def bits_from_blocks(philox, seed, idx, c1, c2, c3):
    """Bit (w[(k>>5)&3] >> (k&31)) & 1 of block (k>>7, c1, c2, c3) for each k in idx."""
    idx = np.asarray(idx, dtype=np.int64).ravel()
    blocks = sorted(set(int(k) >> 7 for k in idx))
    rows = [[b, c1, c2, c3, seed & 0xFFFFFFFF, seed >> 32] for b in blocks]
    out = dict(zip(blocks, philox(rows)))
    return np.array([(out[int(k) >> 7][(int(k) >> 5) & 3] >> (int(k) & 31)) & 1 for k in idx],
                    dtype=np.int64)


# --------------------------------------------------------------------------
# Philox and the keying contract
# --------------------------------------------------------------------------
def test_philox_matches_torch_header(orc, torch_philox):
    rows = rng_rows(300, seed=11) + [[0, 0, 0, 0, 0, 0], [2**32 - 1] * 6]
    want = torch_philox(rows)
    got = [orc.philox4x32_10(r[:4], r[4:]) for r in rows]
    assert got == want


def test_philox_matches_rocrand_header(orc, rocrand_philox):
    rows = rng_rows(300, seed=12) + [[0, 0, 0, 0, 0, 0], [2**32 - 1] * 6]
    want = rocrand_philox(rows)
    got = [orc.philox4x32_10(r[:4], r[4:]) for r in rows]
    assert got == want


def test_tie_and_init_bit_keying(orc, torch_philox):
    rng = np.random.default_rng(3)
    for _ in range(40):
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        t = int(rng.integers(0, 2**32))
        p = int(rng.integers(0, 2))
        ks = rng.integers(0, 2**33, size=8)
        want_tie = bits_from_blocks(torch_philox, seed, ks, t, p, 0)
        want_init = bits_from_blocks(torch_philox, seed, ks, 0, 0, 1)
        for k, wt, wi in zip(ks, want_tie, want_init):
            assert orc.tie_bit(seed, t, p, int(k)) == wt
            assert orc.init_bit(seed, int(k)) == wi


def test_init_matches_keying_and_is_balanced(orc, torch_philox):
    L = 16
    s = orc.init(L, 77)
    i = np.arange(L ** 3)
    want = bits_from_blocks(torch_philox, 77, i, 0, 0, 1)
    assert np.array_equal((s.ravel() > 0).astype(np.int64), want)
    L = 128
    s = orc.init(L, 5)
    N = L ** 3
    assert abs(float(s.astype(np.int64).sum())) < 5 * np.sqrt(N)
    B = int(orc.bonds(s).sum())
    # bond indicators of i.i.d. fair spins are pairwise independent Bernoulli(1/2)
    assert abs(B - 1.5 * N) < 5 * np.sqrt(3 * N / 4)


# --------------------------------------------------------------------------
# the local rule against the paper's acceptance table and brute-force energies
# --------------------------------------------------------------------------
def _golden_acceptance():
    rows = []
    with open(os.path.join(GOLDEN, "glauber_t0_acceptance.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                a, dE, p = line.split()
                rows.append((int(a), int(dE), float(p)))
    return rows


def test_golden_acceptance_table_consistent_with_energy():
    # a site with a anti-aligned neighbours: flipping it changes E by 12 - 4a
    for a, dE, p in _golden_acceptance():
        s = wl.uniform_state(4, 1)
        nbrs = [(1, 0, 0), (3, 0, 0), (0, 1, 0), (0, 3, 0), (0, 0, 1), (0, 0, 3)]
        for (x, y, z) in nbrs[:a]:
            s[z, y, x] = -1
        e0 = energy(s)
        s2 = s.copy()
        s2[0, 0, 0] = -s2[0, 0, 0]
        assert energy(s2) - e0 == dE


def test_rule_matches_golden_acceptance(orc, torch_philox):
    table = {a: p for a, _, p in _golden_acceptance()}
    L = 8
    nbrs = [(1, 0, 0), (L - 1, 0, 0), (0, 1, 0), (0, L - 1, 0), (0, 0, 1), (0, 0, L - 1)]
    for a in range(7):
        for seed in range(6):
            for t in (0, 5, 123456):
                s = wl.uniform_state(L, 1)
                # centre site (0,0,0) is colour 0; neighbours are colour 1
                for (x, y, z) in nbrs[:a]:
                    s[z, y, x] = -1
                s0 = s.copy()
                orc.half_sweep(s, seed, t, 0)
                flipped = s[0, 0, 0] != s0[0, 0, 0]
                if table[a] == 0:
                    assert not flipped
                elif table[a] == 1:
                    assert flipped
                else:
                    bit = bits_from_blocks(torch_philox, seed, [0], t, 0, 0)[0]
                    assert flipped == bool(bit)


@pytest.mark.parametrize("L", [4, 6])
def test_bruteforce_energy_random_order(orc, torch_philox, L):
    """Each proposal judged by recomputing the full energy; sites taken in a
    random order within a colour (same-colour sites do not interact)."""
    rng = np.random.default_rng(L)
    col = colour(L)
    jj = colour_index(L)
    for seed in (1, 2, 0xDEADBEEF12345):
        s_or = orc.init(L, seed)
        s_bf = s_or.copy()
        for t in range(12):
            for p in (0, 1):
                bits = bits_from_blocks(torch_philox, seed, jj.ravel(), t, p, 0).reshape(L, L, L)
                sites = np.argwhere(col == p)
                rng.shuffle(sites)
                for (z, y, x) in sites:
                    e0 = energy(s_bf)
                    s_bf[z, y, x] = -s_bf[z, y, x]
                    dE = energy(s_bf) - e0
                    accept = dE < 0 or (dE == 0 and bits[z, y, x] == 1)
                    if not accept:
                        s_bf[z, y, x] = -s_bf[z, y, x]
                orc.half_sweep(s_or, seed, t, p)
                assert np.array_equal(s_bf, s_or), (seed, t, p)


def test_half_sweep_vectorised_rule_and_bond_accounting(orc, torch_philox):
    """Vectorised restatement: flips exactly where a>=4 or (a==3 and bit);
    B never rises and changes by -sum over flipped sites of (2a - 6)."""
    L = 16
    jj = colour_index(L)
    col = colour(L)
    for seed in (9, 10):
        s = orc.init(L, seed)
        for t in range(6):
            for p in (0, 1):
                a = antialigned(s)
                B0 = int(orc.bonds(s).sum())
                bits = bits_from_blocks(torch_philox, seed, jj.ravel(), t, p, 0).reshape(L, L, L)
                want_flip = (col == p) & ((a >= 4) | ((a == 3) & (bits == 1)))
                s_prev = s.copy()
                nf = orc.half_sweep(s, seed, t, p)
                flipped = s != s_prev
                assert np.array_equal(flipped, want_flip)
                assert nf == int(flipped.sum())
                B1 = int(orc.bonds(s).sum())
                assert B1 <= B0
                assert B1 - B0 == -int((2 * a[flipped] - 6).sum())


# --------------------------------------------------------------------------
# closed forms for special states
# --------------------------------------------------------------------------
@pytest.mark.parametrize("sign", [1, -1])
def test_uniform_states_absorbing(orc, sign):
    L = 8
    s = wl.uniform_state(L, sign)
    tr = orc.run(s, 3, 0, 7, 1)
    assert np.all(s == sign)
    assert np.all(tr == 0)


@pytest.mark.parametrize("pos", [(0, 0, 0), (1, 0, 0), (3, 5, 6), (7, 7, 6)])
def test_isolated_flip_heals_in_one_sweep(orc, pos):
    L = 8
    s = wl.isolated_flip(L, pos)
    assert int(orc.bonds(s).sum()) == 6
    orc.sweep(s, 42, 0)
    assert np.all(s == 1)
    assert int(orc.bonds(s).sum()) == 0


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_flat_interfaces_frozen(orc, axis):
    L = 8
    for s in (wl.slab(L, axis), wl.flipped_plane(L, axis, 3)):
        s0 = s.copy()
        tr = orc.run(s, 5, 0, 10, 1)
        assert np.array_equal(s, s0)
        assert np.all(tr == 2 * L * L)
        assert int(orc.bonds(s).sum()) == 2 * L * L


def test_flipped_line_heals(orc):
    L = 10
    s = wl.flipped_line_x(L, 3, 4)
    assert int(orc.bonds(s).sum()) == 4 * L
    orc.half_sweep(s, 1, 0, 0)
    # colour-0 members (a = 4) flipped, colour-1 members now have a = 6
    line = s[4, 3, :]
    assert np.all(line[(np.arange(L) + 3 + 4) % 2 == 0] == 1)
    assert np.all(line[(np.arange(L) + 3 + 4) % 2 == 1] == -1)
    orc.half_sweep(s, 1, 0, 1)
    assert np.all(s == 1)


def test_neel_start_orders_in_one_half_sweep(orc):
    L = 8
    s = wl.neel(L)
    assert int(orc.bonds(s).sum()) == 3 * L ** 3
    orc.half_sweep(s, 1, 0, 0)
    assert np.all(s == -1)


def test_tie_cube_isolates_keying(orc, torch_philox):
    L = 10
    rng = np.random.default_rng(8)
    col = colour(L)
    jj = colour_index(L)
    for _ in range(25):
        seed = int(rng.integers(0, 2**40))
        t = int(rng.integers(0, 10**6))
        origin = tuple(int(v) for v in rng.integers(0, L, size=3))
        s = wl.flipped_cube(L, origin)
        a = antialigned(s)
        cube = s == -1
        assert np.all(a[cube] == 3)
        s0 = s.copy()
        orc.half_sweep(s, seed, t, 0)
        flipped = s != s0
        bits = bits_from_blocks(torch_philox, seed, jj[cube & (col == 0)], t, 0, 0)
        assert np.array_equal(flipped[cube & (col == 0)], bits == 1)
        assert not flipped[~(cube & (col == 0))].any()


def test_spin_flip_symmetry(orc):
    L = 12
    s = orc.init(L, 21)
    m = -s
    trs = orc.run(s, 21, 0, 20, 1)
    trm = orc.run(m, 21, 0, 20, 1)
    assert np.array_equal(m, -s)
    assert np.array_equal(trs, trm)


# --------------------------------------------------------------------------
# bond-count and correlation identities
# --------------------------------------------------------------------------
def test_bond_identities(orc):
    L = 14
    s = orc.init(L, 4)
    orc.run(s, 4, 0, 3)
    B = orc.bonds(s)
    a = antialigned(s)
    col = colour(L)
    assert int(B.sum()) == int(a[col == 0].sum()) == int(a[col == 1].sum())
    S, M = orc.corr(s)
    N = L ** 3
    assert np.array_equal(S[:, 1], N - 2 * B)


def test_corr_identities_and_fft(orc):
    for L, seed, sweeps in ((16, 1, 0), (16, 2, 5), (32, 3, 8)):
        s = orc.init(L, seed)
        orc.run(s, seed, 0, sweeps)
        S, M = orc.corr(s)
        N = L ** 3
        assert np.all(S[:, 0] == N)
        assert M == int(s.astype(np.int64).sum())
        f = s.astype(np.float64)
        for a in range(3):
            ax = 2 - a
            F = np.fft.fft(f, axis=ax)
            ac = np.fft.ifft(F * np.conj(F), axis=ax).real
            ac = np.moveaxis(ac, ax, 0).reshape(L, -1).sum(axis=1)
            assert np.array_equal(S[a], np.rint(ac[: L // 2 + 1]).astype(np.int64))
            # fold identity: full cyclic sum of S equals the sum of squared line sums
            full = S[a, 0] + 2 * S[a, 1: L // 2].sum() + S[a, L // 2]
            lines = f.sum(axis=ax)
            assert full == int((lines ** 2).sum())


@pytest.mark.parametrize("L", [4, 6])
def test_corr_bruteforce_pairs(orc, L):
    s = orc.init(L, 99)
    S, M = orc.corr(s)
    N = L ** 3
    coords = np.argwhere(np.ones((L, L, L)))
    flat = s.ravel().astype(np.int64)
    want = np.zeros_like(S)
    for i, (z, y, x) in enumerate(coords):
        for j, (z2, y2, x2) in enumerate(coords):
            d = ((x2 - x) % L, (y2 - y) % L, (z2 - z) % L)
            for a in range(3):
                others = [d[b] for b in range(3) if b != a]
                if others == [0, 0] and d[a] <= L // 2:
                    want[a, d[a]] += flat[i] * flat[j]
    assert np.array_equal(S, want)
    assert M == int(flat.sum())
    assert N == L ** 3


# --------------------------------------------------------------------------
# window replay, host derivations, schedules
# --------------------------------------------------------------------------
def test_window_replay_matches_full_run(orc):
    L = 16
    seed = 31
    rng = np.random.default_rng(2)
    s = orc.init(L, seed)
    orc.run(s, seed, 0, 4)
    for T in (1, 2, 3):
        for _ in range(3):
            W = 4 + 4 * T + int(rng.integers(0, 3))
            o = [int(v) for v in rng.integers(0, L, size=3)]
            z, y, x = np.ix_([(o[2] + k) % L for k in range(W)], [(o[1] + k) % L for k in range(W)],
                             [(o[0] + k) % L for k in range(W)])
            w = np.ascontiguousarray(s[z, y, x])
            full = s.copy()
            orc.run(full, seed, 4, T)
            orc.window_advance(L, seed, o, w, 4, T)
            m = 2 * T
            got = w[m:W - m, m:W - m, m:W - m]
            want = full[z, y, x][m:W - m, m:W - m, m:W - m]
            assert np.array_equal(got, want)


def test_window_replay_mixed_matches_full_run(orc):
    """The mixed-cycle replay against full mixed-cycle runs; the 01-cycle
    replay of the same cube differs wherever a sweep draws colour 1 first."""
    L = 16
    seed = 77
    rng = np.random.default_rng(5)
    s = orc.init(L, seed)
    orc.run(s, seed, 0, 6, mixed=True)
    t0 = 6
    # the cycle must draw both orders within the replayed sweeps
    assert {orc.first_colour(seed, t0 + k) for k in range(3)} == {0, 1}
    differs = False
    for T in (1, 2, 3):
        for _ in range(3):
            W = 4 + 4 * T + int(rng.integers(0, 3))
            o = [int(v) for v in rng.integers(0, L, size=3)]
            z, y, x = np.ix_([(o[2] + k) % L for k in range(W)], [(o[1] + k) % L for k in range(W)],
                             [(o[0] + k) % L for k in range(W)])
            w = np.ascontiguousarray(s[z, y, x])
            w01 = w.copy()
            full = s.copy()
            orc.run(full, seed, t0, T, mixed=True)
            orc.window_advance(L, seed, o, w, t0, T, mixed=True)
            orc.window_advance(L, seed, o, w01, t0, T)
            m = 2 * T
            got = w[m:W - m, m:W - m, m:W - m]
            want = full[z, y, x][m:W - m, m:W - m, m:W - m]
            assert np.array_equal(got, want)
            differs |= not np.array_equal(w01[m:W - m, m:W - m, m:W - m], want)
    assert differs


def test_init_window_is_a_slice_of_init(orc):
    L = 12
    s = orc.init(L, 8)
    for o, W in (((0, 0, 0), 12), ((5, 11, 3), 7), ((11, 11, 11), 4)):
        z, y, x = np.ix_([(o[2] + k) % L for k in range(W)], [(o[1] + k) % L for k in range(W)],
                         [(o[0] + k) % L for k in range(W)])
        assert np.array_equal(orc.init_window(L, 8, o, W), s[z, y, x])


def test_host_derivations(orc):
    L = 32
    N = L ** 3
    assert orc.ell_energy(0, N) == float("inf")
    assert orc.ell_energy(3 * N // 8, N) == 8.0
    r = np.arange(L // 2 + 1)
    M = 0
    # C(r) linear in r crosses 1/2 exactly at ell; linear interpolation is exact there
    for ell in (1.5, 7.3, 11.0):
        S = np.tile(np.rint(N * (1.0 - r / (2.0 * ell))).astype(np.int64), (3, 1))
        assert abs(orc.ell_intercept(S, M, N) - ell) < 1e-3
    # exponential decay exp(-r/xi) crosses at xi*ln 2, up to the chord error of
    # linear interpolation (bounded by 1/(8 xi) for unit spacing)
    for xi in (5.0, 9.0):
        S = np.tile(np.rint(N * np.exp(-r / xi)).astype(np.int64), (3, 1))
        assert abs(orc.ell_intercept(S, M, N) - xi * np.log(2.0)) < 1.0 / (8 * xi) + 1e-3
    # a magnetised lattice is handled through the connected part:
    # C(r) = (1 - m^2)(1 - r/14) crosses 1/2 at r = 14 (1 - 0.5/(1 - m^2))
    m = 0.25
    S = np.tile(np.rint(N * (m * m + (1 - m * m) * (1.0 - r / 14.0))).astype(np.int64), (3, 1))
    assert abs(orc.ell_intercept(S, int(m * N), N) - 14.0 * (1 - 0.5 / (1 - m * m))) < 1e-3
    S2 = np.full((3, L // 2 + 1), N, dtype=np.int64)
    assert orc.ell_intercept(S2, 0, N) == float("inf")


def test_log_times_schedule():
    ts = wl.log_times(10_000)
    assert len(ts) == 40 and ts[0] == 1 and ts[-1] == 10_000
    assert all(b > a for a, b in zip(ts, ts[1:]))
    assert ts[:10] == list(range(1, 11))
    ts5 = wl.log_times(100_000)
    assert ts5[-1] == 100_000 and len(ts5) == 40


def test_physics_bands_file_parses():
    with open(os.path.join(GOLDEN, "paper_physics_bands.json")) as f:
        d = json.load(f)
    assert d["ell_L256_t4000_rescaled"]["checkerboard_time_factor"] == 1.75


# --------------------------------------------------------------------------
# mixed cycle (Supplementary Methods I B): colour order drawn per sweep
# --------------------------------------------------------------------------
def test_mixed_cycle_order_keying_and_balance(orc, torch_philox):
    rows = [[0, t, 2, 0, 77, 0] for t in range(400)]
    want = [w[0] & 1 for w in torch_philox(rows)]
    got = [orc.first_colour(77, t) for t in range(400)]
    assert got == want
    assert 150 < sum(got) < 250


@pytest.mark.parametrize("L", [4, 6])
def test_mixed_cycle_bruteforce(orc, torch_philox, L):
    """Each sweep: the drawn colour first, every proposal judged by full energies."""
    col = colour(L)
    jj = colour_index(L)
    seed = 5
    s_or = orc.init(L, seed)
    s_bf = s_or.copy()
    firsts = [w[0] & 1 for w in torch_philox([[0, t, 2, 0, seed, 0] for t in range(16)])]
    assert 0 < sum(firsts) < 16
    for t in range(16):
        for p in (firsts[t], 1 - firsts[t]):
            bits = bits_from_blocks(torch_philox, seed, jj.ravel(), t, p, 0).reshape(L, L, L)
            for (z, y, x) in np.argwhere(col == p):
                e0 = energy(s_bf)
                s_bf[z, y, x] = -s_bf[z, y, x]
                dE = energy(s_bf) - e0
                if not (dE < 0 or (dE == 0 and bits[z, y, x] == 1)):
                    s_bf[z, y, x] = -s_bf[z, y, x]
    orc.run(s_or, seed, 0, 16, mixed=True)
    assert np.array_equal(s_bf, s_or)


def test_mixed_cycle_keeps_invariants(orc):
    L = 12
    s = orc.init(L, 3)
    B_prev = int(orc.bonds(s).sum())
    for t in range(10):
        orc.sweep_mixed(s, 3, t)
        B = int(orc.bonds(s).sum())
        assert B <= B_prev
        B_prev = B
    u = np.ones((L, L, L), dtype=np.int8)
    orc.run(u, 3, 0, 5, mixed=True)
    assert np.all(u == 1)


# --------------------------------------------------------------------------
# Menger-sponge starts (Results, sponge test): the input generator itself
# --------------------------------------------------------------------------
def test_menger_tiles():
    L = 27
    s1 = wl.menger_state(L, 1, seed=4)
    # each 3^3 tile: 20 cells of the sponge's sign and 7 holes (centre + face centres)
    for tz in range(9):
        for ty in range(9):
            for tx in range(9):
                t = s1[3 * tz:3 * tz + 3, 3 * ty:3 * ty + 3, 3 * tx:3 * tx + 3]
                vals, counts = np.unique(t, return_counts=True)
                assert sorted(counts.tolist()) == [7, 20]
                maj = vals[np.argmax(counts)]
                assert t[1, 1, 1] == -maj and t[0, 0, 0] == maj
    s3 = wl.menger_state(L, 3, seed=4)
    # one tile: the sponge's cells are (20/27)^3 of it, the holes the rest
    fracs = sorted([(s3 == 1).mean(), (s3 == -1).mean()])
    assert fracs[0] == pytest.approx((20 / 27) ** 3)
    s0 = wl.menger_state(16, 0, seed=4)
    assert abs(float(s0.mean())) < 0.1            # k = 0: independent fair spins
    # tiles that do not fit at the upper end are cut off there
    s = wl.menger_state(32, 2, seed=1)
    assert s.shape == (32, 32, 32)
    assert np.array_equal(s[:9, :9, :9] != 0, np.ones((9, 9, 9), dtype=bool))


# --------------------------------------------------------------------------
# FFT correlation (eq:sisik) with the radial average and S(k)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L", [4, 6])
def test_fft_corr_bruteforce(orc, L):
    s = orc.init(L, 3 + L)
    orc.run(s, 3 + L, 0, 1)
    N = L ** 3
    f = s.astype(np.float64)
    # O(N^2): G(d) = (1/N) sum_i s_i s_{i+d} for every d by direct sums
    G = np.zeros((L, L, L))
    for dz in range(L):
        for dy in range(L):
            for dx in range(L):
                G[dz, dy, dx] = (f * np.roll(f, (-dz, -dy, -dx), axis=(0, 1, 2))).sum() / N
    m = f.mean()
    sh = orc.oracle.shell_index(L).ravel()
    C, Sk, nr, nk, mm = orc.fft_corr(s)
    assert mm == pytest.approx(m)
    for b in range(len(C)):
        sel = sh == b
        if sel.any():
            assert C[b] == pytest.approx(G.ravel()[sel].mean() - m * m, abs=1e-12)
    # structure factor by a direct discrete Fourier sum
    k = 2 * np.pi * orc.oracle._signed(L) / L
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    S_direct = np.zeros(L ** 3)
    idx = 0
    for kz in k:
        for ky in k:
            for kx in k:
                amp = (f * np.exp(-1j * (kx * x + ky * y + kz * z))).sum()
                S_direct[idx] = abs(amp) ** 2 / N
                idx += 1
    sh_k = orc.oracle.shell_index(L).ravel()
    for b in range(len(Sk)):
        sel = sh_k == b
        if sel.any():
            assert Sk[b] == pytest.approx(S_direct[sel].mean(), rel=1e-10, abs=1e-10)


def test_fft_corr_axis_points_and_sum_rules(orc):
    L = 16
    s = orc.init(L, 8)
    orc.run(s, 8, 0, 6)
    N = L ** 3
    C, Sk, nr, nk, m = orc.fft_corr(s)
    S, M = orc.corr(s)
    assert m * N == pytest.approx(M)
    # shell 0 is d = 0 alone: C(0) = 1 - m^2
    assert nr[0] == 1 and C[0] == pytest.approx(1 - m * m)
    # shell 1 holds |d| = 1 (6) and |d| = sqrt(2) (12)
    assert nr[1] == 18
    # along the axes G equals the exact integer sums S_a(r) / N
    G = orc.oracle.fft_G(s)
    for r in range(L // 2 + 1):
        assert G[0, 0, r] == pytest.approx(S[0, r] / N, abs=1e-12)
        assert G[0, r, 0] == pytest.approx(S[1, r] / N, abs=1e-12)
        assert G[r, 0, 0] == pytest.approx(S[2, r] / N, abs=1e-12)
    # Parseval: sum over all k of |F|^2 / N = sum_i s_i^2 = N; S(k = 0) = M^2 / N
    assert (Sk * nk).sum() == pytest.approx(N)
    assert Sk[0] == pytest.approx(M * M / N)
    assert nr.sum() == N


# --------------------------------------------------------------------------
# double checkerboard (Supplementary Methods I A)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L,B", [(4, 1), (8, 2), (8, 4)])
def test_double_checkerboard_bruteforce(orc, torch_philox, L, B):
    """Phases (coarse, fine) = (0,0), (0,1), (1,0), (1,1); every proposal judged
    by full energies, sites of a phase in random order."""
    rng = np.random.default_rng(B)
    z, y, x = np.indices((L, L, L))
    fine = (x + y + z) % 2
    coarse = (x // B + y // B + z // B) % 2
    jj = colour_index(L)
    seed = 21
    s_or = orc.init(L, seed)
    s_bf = s_or.copy()
    for t in range(4):
        for cc in (0, 1):
            for p in (0, 1):
                bits = bits_from_blocks(torch_philox, seed, jj.ravel(), t, p, 0).reshape(L, L, L)
                sites = np.argwhere((fine == p) & (coarse == cc))
                rng.shuffle(sites)
                for (zz, yy, xx) in sites:
                    e0 = energy(s_bf)
                    s_bf[zz, yy, xx] = -s_bf[zz, yy, xx]
                    dE = energy(s_bf) - e0
                    if not (dE < 0 or (dE == 0 and bits[zz, yy, xx] == 1)):
                        s_bf[zz, yy, xx] = -s_bf[zz, yy, xx]
        orc.sweep_double(s_or, B, seed, t)
        assert np.array_equal(s_bf, s_or), t


@pytest.mark.parametrize("L,B", [(4, 2), (8, 2), (8, 4)])
def test_double_checkerboard_mixed_bruteforce(orc, torch_philox, L, B):
    """Mixed cycle (Supplementary Methods I B): the coarse order drawn per
    sweep, each cube's fine order drawn per sweep; draws and tie bits from
    torch's Philox, every proposal judged by full energies, the sites of a
    step in random order."""
    rng = np.random.default_rng(100 + B)
    z, y, x = np.indices((L, L, L))
    fine = (x + y + z) % 2
    coarse = (x // B + y // B + z // B) % 2
    nb = L // B
    cube = (x // B) + nb * ((y // B) + nb * (z // B))
    jj = colour_index(L)
    seed = 0x1234_0000_0021
    s_or = orc.init(L, seed)
    s_bf = s_or.copy()
    for t in range(5):
        c0 = torch_philox([[0, t, 3, 0, seed & 0xFFFFFFFF, seed >> 32]])[0][0] & 1
        first = bits_from_blocks(torch_philox, seed, np.arange(nb ** 3), t, 4, 0)
        for m in (0, 1):
            cc = c0 ^ m
            for k in (0, 1):
                p_site = first[cube] ^ k
                sel = (coarse == cc) & (fine == p_site)
                sites = np.argwhere(sel)
                rng.shuffle(sites)
                bits = {p: bits_from_blocks(torch_philox, seed, jj.ravel(), t, p, 0).reshape(L, L, L)
                        for p in (0, 1)}
                for (zz, yy, xx) in sites:
                    e0 = energy(s_bf)
                    s_bf[zz, yy, xx] = -s_bf[zz, yy, xx]
                    dE = energy(s_bf) - e0
                    tie = bits[fine[zz, yy, xx]][zz, yy, xx]
                    if not (dE < 0 or (dE == 0 and tie == 1)):
                        s_bf[zz, yy, xx] = -s_bf[zz, yy, xx]
        orc.sweep_double(s_or, B, seed, t, mixed=True)
        assert np.array_equal(s_bf, s_or), t


def test_double_checkerboard_mixed_draws(orc, torch_philox):
    """Keying of the two draws against torch's Philox, and their balance."""
    seed = 91
    rows = [[0, t, 3, 0, seed, 0] for t in range(400)]
    want = [w[0] & 1 for w in torch_philox(rows)]
    got = [orc.coarse_first(seed, t) for t in range(400)]
    assert got == want
    assert 150 < sum(got) < 250
    b = np.arange(0, 4096, 7)
    want_f = bits_from_blocks(torch_philox, seed, b, 9, 4, 0)
    got_f = np.array([orc.fine_first(seed, 9, int(k)) for k in b])
    assert np.array_equal(got_f, want_f)
    assert abs(got_f.mean() - 0.5) < 5 * 0.5 / np.sqrt(len(b))
    # the coarse draw is not the plain checkerboard's colour draw
    assert got != [orc.first_colour(seed, t) for t in range(400)]


def test_double_checkerboard_mixed_invariants(orc):
    """Energy never rises, uniform states absorb, and an isolated flipped
    spin (a = 6) heals in one sweep whatever the drawn orders."""
    L, B = 16, 4
    s = orc.init(L, 8)
    Bprev = int(orc.bonds(s).sum())
    for t in range(10):
        orc.sweep_double(s, B, 8, t, mixed=True)
        Bn = int(orc.bonds(s).sum())
        assert Bn <= Bprev
        Bprev = Bn
    u = np.full((L, L, L), -1, dtype=np.int8)
    orc.sweep_double(u, B, 8, 0, mixed=True)
    assert np.all(u == -1)
    for t in range(4):
        w = np.full((L, L, L), 1, dtype=np.int8)
        w[5, 6, 7] = -1
        orc.sweep_double(w, B, 8, t, mixed=True)
        assert np.all(w == 1)


def test_double_checkerboard_reduces_to_plain_when_blocks_cover(orc):
    """With B = L/2 the coarse colours split the lattice into 8 cubes; the
    trajectory differs from the plain 01 cycle in general, but uniform states
    stay absorbing and the energy never rises."""
    L = 8
    s = orc.init(L, 2)
    Bprev = int(orc.bonds(s).sum())
    for t in range(8):
        orc.sweep_double(s, 4, 2, t)
        B = int(orc.bonds(s).sum())
        assert B <= Bprev
        Bprev = B
    u = np.ones((L, L, L), dtype=np.int8)
    orc.sweep_double(u, 2, 2, 0)
    assert np.all(u == 1)


# --------------------------------------------------------------------------
# accepted flips per sweep (the physics output beside the attempts)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("mixed,double_B", [(False, 0), (True, 0), (False, 2), (True, 4)])
def test_flip_counts_are_hamming_distances(orc, mixed, double_B):
    """Each site is proposed once per sweep, so the flips of a sweep equal the
    number of sites that differ before and after it; the bond trace equals the
    plain run's."""
    L, seed = 16, 12
    s = orc.init(L, seed)
    ref = s.copy()
    B, F = orc.run_traced(s, seed, 0, 9, 1, mixed=mixed, double_B=double_B)
    for k in range(9):
        before = ref.copy()
        if double_B:
            orc.sweep_double(ref, double_B, seed, k, mixed)
        else:
            orc.run(ref, seed, k, 1, mixed=mixed)
        assert F[k] == int((before != ref).sum())
        assert B[k] == int(orc.bonds(before).sum())
    assert np.array_equal(s, ref)
    assert F[0] > 0
