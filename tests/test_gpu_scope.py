"""Parity at the full sizes of the L = 256 int8 and L = 2048 1-bit workloads.

* L = 256 int8 (seed 2, 1e4 MCS): the whole trajectory against the oracle's
  run of the same schedule, with B, S_a(r) and M equal at all 40 log-spaced
  times and the final lattices equal.
* L = 2048 1-bit (seed 3, two sweeps per pass, the configuration bench.py
  times): windows replayed by the oracle at t0 = 1e3, 1e4 and 1e5 - 8; the
  whole lattice downloaded at 1e4 and 1e5 and its bonds recounted on the host
  against qz_bonds and the fused trace; the correlation sums at 1e5 against
  host line sums (fold identity) and direct sums at chosen separations.  The
  mixed cycle (both orders of a pair in one pass) replayed at t0 = 1e4.
* L = 1024: every S_a(r) of a late state against per-line FFT
  autocorrelations computed on the host.

(Methods, "Checkerboard update"; Results, the correlation function and the
c = 0.5 intercept.)
"""
import os

import numpy as np
import pytest

from paper_2305_12161_amd import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def qz():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_12161_amd import binding
    return binding


@pytest.fixture(scope="module", autouse=True)
def _threads(orc):
    n = min(16, len(os.sched_getaffinity(0)))
    orc.set_threads(n)
    import torch
    torch.set_num_threads(n)


def replay(orc, lat, seed, origin, W, T, mixed=False):
    """Advance a W^3 window of the GPU state T sweeps with the oracle and compare
    its core (2T sites in from every face) with the GPU's window T sweeps later.
    The GPU's T sweeps trace the bond count entering the first one, returned."""
    L = lat.L
    t0 = lat.t
    w = lat.window(origin, W)
    orc.window_advance(L, seed, origin, w, t0, T, mixed=mixed)
    B, _ = lat.run_at(T, [0])
    got = lat.window(origin, W)
    m = 2 * T
    core = (slice(m, W - m),) * 3
    assert np.array_equal(w[core], got[core]), (t0, origin)
    return int(B[0])


def host_line_square_sums(t):
    """Sum over the lines along each axis of (line magnetisation)^2, for x, y, z
    (array dims 2, 1, 0 of a (z, y, x) int8 tensor)."""
    import torch
    out = []
    for dim in (2, 1, 0):
        ls = t.sum(dim=dim, dtype=torch.int64)
        out.append(int((ls * ls).sum()))
    return out


def host_axis_sum(t, axis, r, slab=128):
    """S_axis(r) = sum_i s_i s_{i + r e_axis} by direct products, in slabs."""
    import torch
    L = t.shape[0]
    dim = {0: 2, 1: 1, 2: 0}[axis]
    cut = 0 if dim != 0 else 1          # slab along a dimension the shift does not use
    acc = 0
    for a in range(0, L, slab):
        part = t.narrow(cut, a, slab)
        acc += int((part * torch.roll(part, -r, dims=dim)).sum(dtype=torch.int64))
    return acc


# --------------------------------------------------------------------------
# L = 256, int8, seed 2, 1e4 MCS: the whole trajectory against the oracle
# --------------------------------------------------------------------------
def test_i8_L256_trajectory_matches_oracle(qz, orc):
    c = wl.RUN_I8_L256
    N = c.L ** 3
    lat = qz.Lattice(c.L, c.seed, "i8")
    s = orc.init(c.L, c.seed)
    t = 0
    for k, tc in enumerate(c.corr_times):
        lat.run(tc - lat.t)
        orc.run(s, c.seed, t, tc - t)
        t = tc
        B = lat.bonds()
        Bo = orc.bonds(s)
        S, M = lat.corr()
        So, Mo = orc.corr(s)
        say("i8 L=256 t =", tc, "B =", int(B.sum()), "M =", M)
        assert np.array_equal(B, Bo), tc
        assert M == Mo, tc
        assert np.array_equal(S, So), tc
        assert np.all(S[:, 0] == N) and np.array_equal(S[:, 1], N - 2 * B)
    assert lat.t == c.t_max == t
    assert np.array_equal(lat.download(), s)


# --------------------------------------------------------------------------
# L = 2048, 1-bit, seed 3, two sweeps per pass: late windows, recounts
# --------------------------------------------------------------------------
def test_L2048_late_replays_and_recounts(qz, orc):
    import torch
    c = wl.RUN_BIT_L2048
    L, seed, N = c.L, c.seed, c.L ** 3
    lat = qz.Lattice(L, seed, "bit")
    assert lat.pass_config()[0] == 2
    say("L=2048 late: pass", lat.pass_config())
    rng = np.random.default_rng(2048)
    W, T = 160, 8
    for t0 in (1_000, 10_000, c.t_max - T):
        lat.run(t0 - lat.t)
        o = [int(v) for v in rng.integers(0, L, size=3)]
        say("L=2048 replay at", t0, o)
        full = t0 == 10_000
        if full:
            s = lat.download()
            Bh = np.zeros(3, dtype=np.int64)
            Bh[:] = orc.bonds(s)
            del s
            assert np.array_equal(lat.bonds(), Bh)
        B_entering = replay(orc, lat, seed, o, W, T)
        if full:
            assert B_entering == int(Bh.sum())
    assert lat.t == c.t_max
    # the final state: host recount, and the correlation sums
    say("L=2048 final download")
    s = lat.download()
    Bh = orc.bonds(s)
    assert np.array_equal(lat.bonds(), Bh)
    S, M = lat.corr()
    ts = torch.from_numpy(s)
    del s
    assert M == int(ts.sum(dtype=torch.int64))
    assert np.all(S[:, 0] == N)
    assert np.array_equal(S[:, 1], N - 2 * Bh)
    sq = host_line_square_sums(ts)
    for a in range(3):
        fold = int(S[a, 0]) + 2 * int(S[a, 1:L // 2].sum()) + int(S[a, L // 2])
        assert fold == sq[a], a
    for a in range(3):
        for r in (2, 257, L // 2):
            say("L=2048 direct S", a, r)
            assert int(S[a, r]) == host_axis_sum(ts, a, r), (a, r)


def test_L2048_mixed_cycle_replay_t1e4(qz, orc):
    """The mixed cycle at L = 2048 (pairs of sweeps of either order share a
    pass) replayed by the oracle's mixed-cycle window at t0 = 1e4."""
    c = wl.RUN_BIT_L2048
    L, seed = c.L, c.seed
    lat = qz.Lattice(L, seed, "bit")
    lat.set_cycle(True)
    assert lat.pass_config()[0] == 2
    orders = [orc.first_colour(seed, t) for t in range(10_000, 10_008)]
    # the window covers pairs of equal and of different orders
    assert any(orders[i] != orders[i + 1] for i in range(0, 8, 2))
    lat.run(10_000)
    rng = np.random.default_rng(4096)
    for _ in range(2):
        o = [int(v) for v in rng.integers(0, L, size=3)]
        say("L=2048 mixed replay at", lat.t, o)
        replay(orc, lat, seed, o, 160, 8, mixed=True)


def test_L2048_tile_full_run_L256(qz, orc):
    """The two-sweep tile of the L = 2048 default, read from an L = 2048 handle,
    on a full L = 256 run against the oracle."""
    big = qz.Lattice(2048, 3, "bit")
    sweeps, V, Ty, Tz = big.pass_config()
    del big
    assert sweeps == 2
    L, seed, n = 256, 3, 60
    lat = qz.Lattice(L, seed, "bit")
    lat.set_pass(2, V, Ty, Tz)
    say("L256 with the L2048 tile", lat.pass_config())
    tr = lat.run(n, 5)
    s = orc.init(L, seed)
    want = orc.run(s, seed, 0, n, 5)
    assert np.array_equal(tr.astype(np.int64), want)
    assert np.array_equal(lat.download(), s)


# --------------------------------------------------------------------------
# L = 1024: every S_a(r) against per-line FFT autocorrelations on the host
# --------------------------------------------------------------------------
def test_corr_matches_per_line_fft_L1024(qz):
    import torch
    L, seed = 1024, 77
    lat = qz.Lattice(L, seed, "bit")
    lat.run(300)
    S, M = lat.corr()
    t = torch.from_numpy(lat.download())
    assert M == int(t.sum(dtype=torch.int64))
    R = L // 2 + 1
    # lines along x, y, z as the last dimension of a permuted view, in chunks
    for a, perm in enumerate(((0, 1, 2), (0, 2, 1), (1, 2, 0))):
        v = t.permute(*perm)
        power = torch.zeros(L // 2 + 1, dtype=torch.float64)
        for k in range(0, L, 64):
            chunk = v[k:k + 64].reshape(-1, L).to(torch.float64)
            f = torch.fft.rfft(chunk, dim=1)
            power += (f.real ** 2 + f.imag ** 2).sum(dim=0)
        ac = torch.fft.irfft(power, n=L)
        want = np.rint(ac[:R].numpy()).astype(np.int64)
        say("L1024 axis", a, "max |diff|", int(np.abs(S[a] - want).max()))
        assert np.array_equal(S[a], want), a
