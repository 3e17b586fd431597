"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

The dynamics are exact integer work, so every comparison is bit-exact:
lattices, bond traces, per-axis bond counts and correlation sums.
"""
import os

import numpy as np
import pytest

from paper_2305_12161_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qz():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_12161_amd import binding
    return binding


@pytest.fixture(scope="module", autouse=True)
def _threads(orc):
    orc.set_threads(min(16, os.cpu_count() or 1))


def say(*a):
    print(*a, flush=True)


def oracle_run(orc, L, seed, n, every=0, s=None, t0=0):
    if s is None:
        s = orc.init(L, seed)
    tr = orc.run(s, seed, t0, n, every)
    return s, tr


# --------------------------------------------------------------------------
# initial state
# --------------------------------------------------------------------------
@pytest.mark.parametrize("layout,L", [("i8", 4), ("i8", 6), ("i8", 10), ("i8", 32),
                                      ("bit", 64), ("bit", 128), ("bit", 192), ("bit", 256)])
def test_init_matches_oracle(qz, orc, layout, L):
    say("init", layout, L)
    for seed in (1, 2**63 + 12345):
        lat = qz.Lattice(L, seed, layout)
        assert np.array_equal(lat.download(), orc.init(L, seed))


# --------------------------------------------------------------------------
# dynamics: the L=32 int8 run in full, small and ragged sizes, both layouts
# --------------------------------------------------------------------------
def test_i8_L32_full_run(qz, orc):
    c = wl.RUN_I8_L32
    say("i8 L=32", c)
    lat = qz.Lattice(c.L, c.seed, "i8")
    tr = lat.run(c.t_max, c.trace_every)
    s, want = oracle_run(orc, c.L, c.seed, c.t_max, c.trace_every)
    assert np.array_equal(tr.astype(np.int64), want)
    assert np.array_equal(lat.download(), s)
    assert np.array_equal(lat.bonds(), orc.bonds(s))
    assert lat.t == c.t_max


@pytest.mark.parametrize("L", [4, 6, 8, 10, 16, 18])
def test_i8_small_sizes(qz, orc, L):
    for seed in (3, 2**40 + 7):
        say("i8 small", L, seed)
        lat = qz.Lattice(L, seed, "i8")
        s = orc.init(L, seed)
        for chunk in (1, 4, 15):
            tr = lat.run(chunk, 1)
            want = orc.run(s, seed, lat.t - chunk, chunk, 1)
            assert np.array_equal(tr.astype(np.int64), want)
            assert np.array_equal(lat.download(), s)


@pytest.mark.parametrize("L", [272, 320])
def test_i8_chunked_sizes_above_256(qz, orc, L):
    """The int8 half-sweep of 16-byte chunks at sides above 256 that are not
    multiples of 64 (L = 272: 17 chunks per row, 320: 20), whose planes do not
    fill whole workgroups of chunks.  Traces, the full lattice and its bonds
    equal the oracle's, in both cycles."""
    for mixed in (False, True):
        seed = 7000 + L + (1 if mixed else 0)
        say("i8 chunked", L, "mixed" if mixed else "01")
        lat = qz.Lattice(L, seed, "i8")
        lat.set_cycle(mixed)
        s = orc.init(L, seed)
        for chunk in (1, 5):
            tr = lat.run(chunk, 1)
            want = orc.run(s, seed, lat.t - chunk, chunk, 1, mixed=mixed)
            assert np.array_equal(tr.astype(np.int64), want), (L, mixed, chunk)
        assert np.array_equal(lat.download(), s)
        assert np.array_equal(lat.bonds(), orc.bonds(s))
        del lat


@pytest.mark.parametrize("L", [64, 128, 192, 256])
def test_bit_default_tuning(qz, orc, L):
    seed = 1000 + L
    say("bit default", L)
    lat = qz.Lattice(L, seed, "bit")
    n = 20 if L <= 128 else 8
    tr = lat.run(n, 2)
    s, want = oracle_run(orc, L, seed, n, 2)
    assert np.array_equal(tr.astype(np.int64), want)
    assert np.array_equal(lat.download(), s)


def test_default_tunings_run_at_every_size(qz):
    """Every L % 64 == 0 up to 1024 gets a default one-sweep and two-sweep
    configuration that launches, and the two agree on the trajectory."""
    for L in range(64, 1025, 64):
        say("default tuning", L)
        a = qz.Lattice(L, 7, "bit")
        a.set_pass(1)
        b = qz.Lattice(L, 7, "bit")
        b.set_pass(2)
        ta = a.run(4, 2)
        tb = b.run(4, 2)
        assert np.array_equal(ta, tb), (L, a.tuning(), b.pass_config())
        assert np.array_equal(a.window((1, 2, 3), 16), b.window((1, 2, 3), 16)), L
        del a, b


# (V, Ty, Tz) triples covering whole planes, halo tiles, ragged y and z tiles
TUNINGS = {
    64: [(1, 64, 64), (1, 64, 5), (1, 28, 7), (1, 12, 64), (1, 60, 3)],
    128: [(2, 128, 8), (1, 128, 13), (2, 28, 11), (1, 60, 128), (2, 124, 6)],
    192: [(1, 192, 16), (1, 28, 20), (1, 60, 7)],
    256: [(4, 256, 16), (2, 60, 32), (4, 28, 10), (1, 28, 256), (4, 124, 9)],
}


@pytest.mark.parametrize("L", sorted(TUNINGS))
def test_bit_tunings_match_oracle(qz, orc, L):
    seed = 77 + L
    n = 6
    s, want = oracle_run(orc, L, seed, n, 1)
    for V, Ty, Tz in TUNINGS[L]:
        say("bit tuning", L, (V, Ty, Tz))
        lat = qz.Lattice(L, seed, "bit")
        lat.set_tuning(V, Ty, Tz)
        tr = lat.run(n, 1)
        assert np.array_equal(tr.astype(np.int64), want), (V, Ty, Tz)
        assert np.array_equal(lat.download(), s), (V, Ty, Tz)


# (V, Ty, Tz) of the two-sweep pass: ragged y and z tiles, one-plane tiles,
# tiles whose held rows wrap past L, and the paired row mapping
TUNINGS2 = {
    64: [(1, 24, 64), (1, 8, 5), (1, 56, 7), (1, 64, 3)],
    128: [(2, 24, 11), (1, 56, 128), (2, 120, 6), (2, 8, 1)],
    192: [(1, 24, 20), (1, 56, 7)],
    256: [(4, 24, 32), (2, 56, 10), (4, 24, 256), (4, 8, 9), (4, 120, 5)],
    # paired row mapping (wave-uniform x parity): V = 4 with E a multiple of 128 / R
    512: [(4, 56, 7), (4, 120, 32)],
}


@pytest.mark.parametrize("L", sorted(TUNINGS2))
def test_two_sweep_pass_matches_oracle(qz, orc, L):
    """Two sweeps per pass: same trajectory and bond trace (every sweep traced,
    so both counters of a pass are used; an odd count ends with one sweep)."""
    seed = 500 + L
    n = 7
    s, want = oracle_run(orc, L, seed, n, 1)
    for V, Ty, Tz in [(0, 0, 0)] + TUNINGS2[L]:
        say("two-sweep pass", L, (V, Ty, Tz))
        lat = qz.Lattice(L, seed, "bit")
        lat.set_pass(2, V, Ty, Tz)
        assert lat.pass_config()[0] == 2
        tr = lat.run(n, 1)
        assert np.array_equal(tr.astype(np.int64), want), (V, Ty, Tz)
        assert np.array_equal(lat.download(), s), (V, Ty, Tz)


@pytest.mark.parametrize("tuning", [(4, 24, 32), (4, 120, 5), (4, 56, 8)])
def test_two_sweep_pass_late_times(qz, orc, tuning):
    """3000 sweeps at L = 256 with V = 4 tunings (paired and unpaired rows),
    traced every 100: the late regime, where ties are sparse, against the
    oracle."""
    L, seed, n, every = 256, 77, 3000, 100
    key = ("late", L, seed, n, every)
    if key not in _LATE:
        s = orc.init(L, seed)
        _LATE[key] = (orc.run(s, seed, 0, n, every), s)
    want, s = _LATE[key]
    say("two-sweep late times", L, tuning)
    lat = qz.Lattice(L, seed, "bit")
    lat.set_pass(2, *tuning)
    tr = lat.run(n, every)
    assert np.array_equal(tr.astype(np.int64), want), tuning
    assert np.array_equal(lat.download(), s), tuning


_LATE = {}


@pytest.mark.parametrize("every,n", [(2, 8), (3, 9), (5, 10)])
def test_two_sweep_pass_trace_alignment(qz, orc, every, n):
    """Start at an odd time from an uploaded state: pairs straddle the traced
    sweeps, so a pass carries the count in its first sweep, its second, or none."""
    L, seed, t0 = 128, 61, 5
    s = wl.random_state(L, 9)
    lat = qz.Lattice(L, seed, "bit")
    lat.upload(s, t0)
    lat.set_pass(2)
    say("two-sweep alignment", every, n)
    tr = lat.run(n, every)
    want = orc.run(s, seed, t0, n, every)
    assert np.array_equal(tr.astype(np.int64), want)
    assert np.array_equal(lat.download(), s)
    assert lat.t == t0 + n


@pytest.mark.parametrize("L,tuning", [(64, (1, 24, 5)), (128, (2, 56, 8)), (256, (4, 120, 5)),
                                      (256, (4, 24, 32))])
def test_two_sweep_pass_mixed_cycle(qz, orc, L, tuning):
    """The mixed cycle with two sweeps per pass: every two consecutive sweeps
    share a pass, whichever first colours they draw (planes exchanged when
    sweep t draws colour 1; the second sweep's stages the other way round
    when it draws the other colour); every sweep traced, against the oracle."""
    n = 21

    def pair_orders(seed):     # (first colour of t, of t+1) of each shared pass
        fc = [orc.first_colour(seed, t) for t in range(n)]
        return {(fc[t], fc[t + 1]) for t in range(0, n - 1, 2)}

    seed = 700 + L
    while len(pair_orders(seed)) < 4:      # passes of all four order pairs
        seed += 1
    s = orc.init(L, seed)
    want = orc.run(s, seed, 0, n, 1, mixed=True)
    lat = qz.Lattice(L, seed, "bit")
    lat.set_cycle(True)
    lat.set_pass(2, *tuning)
    say("two-sweep mixed", L, tuning, seed)
    tr = lat.run(n, 1)
    assert np.array_equal(tr.astype(np.int64), want)
    assert np.array_equal(lat.download(), s)


def test_two_sweep_pass_mixed_cycle_large(qz):
    """L = 1024, the paired tile of the large lattices: the mixed cycle with two
    sweeps per pass (all four order pairs occur in 12 sweeps of this seed)
    gives the same bond and flip traces and lattice as one sweep per pass."""
    L, seed = 1024, 91
    say("two-sweep mixed vs one-sweep", L, seed)
    two = qz.Lattice(L, seed, "bit")
    two.set_cycle(True)
    two.set_pass(2, 4, 56, 64)
    B2, F2 = two.run_traced(12, 1)
    one = qz.Lattice(L, seed, "bit")
    one.set_cycle(True)
    one.set_pass(1)
    B1, F1 = one.run_traced(12, 1)
    assert np.array_equal(B2, B1)
    assert np.array_equal(F2, F1)
    assert np.array_equal(two.download(), one.download())


def test_two_sweep_pass_falls_back_and_rejects(qz, orc):
    L, seed = 64, 8
    lat = qz.Lattice(L, seed, "bit")
    lat.set_pass(2)
    lat.set_cycle(True)        # the mixed cycle pairs only sweeps of equal order
    tr = lat.run(5, 1)
    s = orc.init(L, seed)
    want = orc.run(s, seed, 0, 5, 1, mixed=True)
    assert np.array_equal(tr.astype(np.int64), want)
    assert np.array_equal(lat.download(), s)
    for bad in ((3, 0, 0, 0), (0, 0, 0, 0), (2, 3, 24, 8), (2, 1, 2000, 8), (2, 1, 24, 0)):
        with pytest.raises(qz.QuenchError):
            lat.set_pass(*bad)
    with pytest.raises(qz.QuenchError):
        qz.Lattice(16, 1, "i8").set_pass(2)


@pytest.mark.parametrize("L", [64, 128])
def test_bit_equals_i8(qz, L):
    seed = 5 + L
    say("bit==i8", L)
    a = qz.Lattice(L, seed, "i8")
    b = qz.Lattice(L, seed, "bit")
    ta = a.run(60, 3)
    tb = b.run(60, 3)
    assert np.array_equal(ta, tb)
    assert np.array_equal(a.download(), b.download())
    assert np.array_equal(a.bonds(), b.bonds())
    Sa, Ma = a.corr()
    Sb, Mb = b.corr()
    assert np.array_equal(Sa, Sb) and Ma == Mb


# --------------------------------------------------------------------------
# measurements
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L", [512, 768, 1024])
def test_corr_closed_forms_large(qz, L):
    """Axis sums of states with a closed form, at sizes where y and z run on
    the matrix cores: uniform (S = N), Neel (S = N (-1)^r) and slabs normal
    to y and to z (S = N - 4 r L^2 along the normal, N along the others)."""
    N = L ** 3
    R = L // 2 + 1
    r = np.arange(R, dtype=np.int64)
    flat = np.full(R, N, dtype=np.int64)
    ar = np.arange(L)
    half = np.where(ar < L // 2, -1, 1).astype(np.int8)

    def state(name):   # int8 throughout: at L = 1024 a state is 1 GiB
        s = np.empty((L, L, L), dtype=np.int8)
        if name == "up":
            s[...] = 1
        elif name == "neel":
            pyz = ((ar[:, None] + ar[None, :]) % 2).astype(np.int8)[:, :, None]
            px = (ar % 2).astype(np.int8)[None, None, :]
            np.bitwise_xor(pyz, px, out=s)
            np.multiply(s, -2, out=s)
            np.add(s, 1, out=s)
        elif name == "slab_z":
            s[...] = half[:, None, None]
        else:
            s[...] = half[None, :, None]
        return s

    cases = {
        "up": (np.stack([flat, flat, flat]), N),
        "neel": (np.tile(N * (-1) ** r, (3, 1)), 0),
        "slab_z": (np.stack([flat, flat, N - 4 * r * L * L]), 0),
        "slab_y": (np.stack([flat, N - 4 * r * L * L, flat]), 0),
    }
    lat = qz.Lattice(L, 1, "bit")
    for name, (want, want_M) in cases.items():
        say("corr closed form", L, name)
        lat.upload(state(name), 0)
        S, M = lat.corr()
        assert M == want_M, name
        assert np.array_equal(S, want), name


@pytest.mark.parametrize("sweeps", [1, 2])
def test_corr_leaves_the_dynamics_unchanged(qz, sweeps):
    """The correlation uses the lattice's idle copy as scratch (for the x
    axis on the matrix cores): measuring between runs must not change the
    trajectory."""
    L, seed = 256, 23
    a = qz.Lattice(L, seed, "bit")
    b = qz.Lattice(L, seed, "bit")
    a.set_pass(sweeps)
    b.set_pass(sweeps)
    ta = [a.run(10, 5)]
    for _ in range(3):
        S1, M1 = a.corr()
        S2, M2 = a.corr()
        assert np.array_equal(S1, S2) and M1 == M2
        ta.append(a.run(11, 1))
    tb = [b.run(10, 5)] + [b.run(11, 1) for _ in range(3)]
    for x, y in zip(ta, tb):
        assert np.array_equal(x, y)
    assert np.array_equal(a.download(), b.download())


def test_corr_matches_fft_L512(qz):
    """A random state after 40 sweeps at L = 512 against the axis
    autocorrelation computed with numpy's FFT (rounded; exact in double)."""
    L, seed = 512, 91
    lat = qz.Lattice(L, seed, "bit")
    lat.run(40)
    S, M = lat.corr()
    s = lat.download().astype(np.float64)
    assert M == int(s.sum())
    R = L // 2 + 1
    for a, ax in enumerate((2, 1, 0)):   # x, y, z are array axes 2, 1, 0
        f = np.fft.rfft(s, axis=ax)
        ac = np.fft.irfft(f * np.conj(f), n=L, axis=ax)
        del f
        want = np.rint(ac.sum(axis=tuple(k for k in range(3) if k != ax))[:R]).astype(np.int64)
        del ac
        assert np.array_equal(S[a], want), a


@pytest.mark.parametrize("L", [4, 6, 10, 18, 34, 66, 130, 256])
def test_i8_corr_random_states(qz, L):
    """The int8 layout's correlation sums on uploaded random states (biased,
    so that M is far from 0) against numpy's FFT autocorrelation per axis
    (exact in double at these sizes): sizes with L % 4 == 2 end their lines
    in a half word, and L = 256 runs the full block geometry."""
    R = L // 2 + 1
    for p_up, seed in ((0.5, 3), (0.8, 4)):
        say("i8 corr", L, p_up)
        st = wl.random_state(L, seed + L, p_up)
        lat = qz.Lattice(L, 1, "i8")
        lat.upload(st, 0)
        S, M = lat.corr()
        s = st.astype(np.float64)
        assert M == int(s.sum())
        for a, ax in enumerate((2, 1, 0)):   # x, y, z are array axes 2, 1, 0
            f = np.fft.rfft(s, axis=ax)
            ac = np.fft.irfft(f * np.conj(f), n=L, axis=ax)
            want = np.rint(ac.sum(axis=tuple(k for k in range(3) if k != ax))[:R]).astype(np.int64)
            assert np.array_equal(S[a], want), (a, L, p_up)


@pytest.mark.parametrize("layout,L", [("i8", 6), ("i8", 16), ("i8", 34), ("bit", 64),
                                      ("bit", 128), ("bit", 192), ("bit", 256)])
def test_bonds_and_corr_match_oracle(qz, orc, layout, L):
    seed = 11 + L
    say("measure", layout, L)
    lat = qz.Lattice(L, seed, layout)
    s = orc.init(L, seed)
    for n in (0, 3, 10):
        if n:
            lat.run(n)
            orc.run(s, seed, lat.t - n, n)
        assert np.array_equal(lat.download(), s)
        assert np.array_equal(lat.bonds(), orc.bonds(s))
        # the asynchronous form, into device memory after a stale fill
        import torch
        dev = torch.full((5,), -1, dtype=torch.int64, device="cuda")
        lat.bonds_device(dev[1:])
        torch.cuda.synchronize()
        got = dev.cpu().numpy()
        assert got[0] == -1 and got[4] == -1
        assert np.array_equal(got[1:4], orc.bonds(s))
        S, M = lat.corr()
        So, Mo = orc.corr(s)
        assert M == Mo
        assert np.array_equal(S, So)


# --------------------------------------------------------------------------
# special states, upload/download, windows
# --------------------------------------------------------------------------
SPECIAL = {
    "uniform_up": lambda L: wl.uniform_state(L, 1),
    "uniform_down": lambda L: wl.uniform_state(L, -1),
    "isolated": lambda L: wl.isolated_flip(L, (5, 3, 1)),
    "slab_z": lambda L: wl.slab(L, 2),
    "slab_x": lambda L: wl.slab(L, 0),
    "plane": lambda L: wl.flipped_plane(L, 1, 2),
    "line": lambda L: wl.flipped_line_x(L, 2, 3),
    "neel": lambda L: wl.neel(L),
    "cube": lambda L: wl.flipped_cube(L, (L - 1, 0, 7)),
    "random": lambda L: wl.random_state(L, 3, 0.3),
}


@pytest.mark.parametrize("layout,L", [("i8", 8), ("i8", 64), ("bit", 64), ("bit", 128)])
@pytest.mark.parametrize("name", sorted(SPECIAL))
def test_special_states(qz, orc, layout, L, name):
    say("special", name, layout, L)
    s = SPECIAL[name](L)
    lat = qz.Lattice(L, 9, layout)
    lat.upload(s, 40)
    assert lat.t == 40
    assert np.array_equal(lat.download(), s)
    tr = lat.run(4, 1)
    want = orc.run(s, 9, 40, 4, 1)
    assert np.array_equal(tr.astype(np.int64), want)
    assert np.array_equal(lat.download(), s)


def test_upload_rejects_non_spin_values(qz):
    for layout, L in (("i8", 8), ("bit", 64)):
        lat = qz.Lattice(L, 1, layout)
        bad = np.ones((L, L, L), dtype=np.int8)
        bad[1, 2, 3] = 0
        with pytest.raises(qz.QuenchError) as ei:
            lat.upload(bad, 0)
        assert ei.value.status == qz.QZ_EINVAL


@pytest.mark.parametrize("layout,L", [("i8", 16), ("bit", 64), ("bit", 128)])
def test_window_download(qz, layout, L):
    lat = qz.Lattice(L, 21, layout)
    lat.run(5)
    full = lat.download()
    rng = np.random.default_rng(L)
    for _ in range(4):
        W = int(rng.integers(1, L + 1))
        o = [int(v) for v in rng.integers(0, L, size=3)]
        w = lat.window(o, W)
        z, y, x = np.ix_([(o[2] + k) % L for k in range(W)], [(o[1] + k) % L for k in range(W)],
                         [(o[0] + k) % L for k in range(W)])
        assert np.array_equal(w, full[z, y, x])


def test_checkpoint_resume_is_exact(qz):
    for layout, L in (("i8", 32), ("bit", 64)):
        a = qz.Lattice(L, 44, layout)
        a.run(30)
        snap, t = a.download(), a.t
        ta = a.run(30, 5)
        b = qz.Lattice(L, 44, layout)
        b.upload(snap, t)
        tb = b.run(30, 5)
        assert np.array_equal(ta, tb)
        assert np.array_equal(a.download(), b.download())


def test_run_device_trace_matches_host_trace(qz):
    import torch
    a = qz.Lattice(128, 8, "bit")
    b = qz.Lattice(128, 8, "bit")
    dev = torch.zeros(10, dtype=torch.int64, device="cuda")
    a.run_device(50, 5, dev)
    tb = b.run(50, 5)
    torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy().astype(np.uint64), tb)


def test_bad_arguments_raise(qz):
    with pytest.raises(qz.QuenchError):
        qz.Lattice(96, 1, "bit")
    with pytest.raises(qz.QuenchError):
        qz.Lattice(7, 1, "i8")
    lat = qz.Lattice(64, 1, "bit")
    with pytest.raises(qz.QuenchError):
        lat.set_tuning(3, 64, 8)
    with pytest.raises(qz.QuenchError):
        lat.run(10, 3)
    i8 = qz.Lattice(8, 1, "i8")
    with pytest.raises(qz.QuenchError):
        i8.set_tuning(1, 8, 8)


# --------------------------------------------------------------------------
# mixed cycle: the colour updated first is drawn per sweep
# --------------------------------------------------------------------------
@pytest.mark.parametrize("layout,L,tuning", [("i8", 6, None), ("i8", 16, None), ("bit", 64, None),
                                             ("bit", 128, (2, 28, 11)), ("bit", 256, (4, 28, 10))])
def test_mixed_cycle_matches_oracle(qz, orc, layout, L, tuning):
    seed = 31 + L
    say("mixed", layout, L, tuning)
    lat = qz.Lattice(L, seed, layout)
    if tuning:
        lat.set_tuning(*tuning)
    lat.set_cycle(True)
    n = 12
    tr = lat.run(n, 1)
    s = orc.init(L, seed)
    want = orc.run(s, seed, 0, n, 1, mixed=True)
    assert np.array_equal(tr.astype(np.int64), want)
    assert np.array_equal(lat.download(), s)


def test_mixed_differs_from_01(qz):
    a = qz.Lattice(64, 3, "bit")
    b = qz.Lattice(64, 3, "bit")
    b.set_cycle(True)
    a.run(20)
    b.run(20)
    assert not np.array_equal(a.download(), b.download())


@pytest.mark.parametrize("layout,L,k", [("i8", 54, 3), ("bit", 64, 2), ("bit", 128, 3)])
def test_menger_start_matches_oracle(qz, orc, layout, L, k):
    """Quench from a Menger-sponge start (Results, sponge test) on both paths."""
    s = wl.menger_state(L, k, seed=L + k)
    say("menger", layout, L, k)
    lat = qz.Lattice(L, 5, layout)
    lat.upload(s, 0)
    tr = lat.run(10, 2)
    want = orc.run(s, 5, 0, 10, 2)
    assert np.array_equal(tr.astype(np.int64), want)
    assert np.array_equal(lat.download(), s)


# --------------------------------------------------------------------------
# FFT route to C(r) and S(k) (eq:sisik, radial average).  Both sides sum in
# double precision in different orders: the shell means agree to ~1e-12 at
# these sizes (eps * log2 N * sqrt N); 1e-9 is used.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("layout,L,n", [("i8", 16, 3), ("i8", 32, 20), ("bit", 64, 10),
                                        ("bit", 128, 40)])
def test_fft_corr_matches_oracle(qz, orc, layout, L, n):
    say("fft corr", layout, L)
    lat = qz.Lattice(L, 70 + L, layout)
    lat.run(n)
    s = lat.download()
    C, Sk, nr, nk, m = lat.fft_corr()
    Co, Sko, nro, nko, mo = orc.fft_corr(s)
    assert np.array_equal(nr, nro) and np.array_equal(nk, nko)
    assert m == pytest.approx(mo, abs=1e-12)
    assert np.allclose(C, Co, rtol=0, atol=1e-9)
    assert np.allclose(Sk, Sko, rtol=1e-9, atol=1e-9)


# --------------------------------------------------------------------------
# double checkerboard (coarse cubes of side B)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("mixed", [False, True], ids=["01", "mixed"])
@pytest.mark.parametrize("L,B", [(64, 2), (64, 8), (64, 32), (128, 4), (128, 64), (256, 16),
                                 (256, 2), (256, 4), (256, 64), (256, 128), (512, 8)])
def test_double_checkerboard_matches_oracle(qz, orc, L, B, mixed):
    seed = 90 + L + B + (1000 if mixed else 0)
    say("double checkerboard", L, B, "mixed" if mixed else "01")
    lat = qz.Lattice(L, seed, "bit")
    lat.set_double_checkerboard(B)
    if mixed:
        lat.set_cycle(True)
    n = 6 if L < 256 else 3
    tr = lat.run(n, 1)
    s = orc.init(L, seed)
    want = orc.run_double(s, B, seed, 0, n, 1, mixed=mixed)
    assert np.array_equal(tr.astype(np.int64), want)
    assert np.array_equal(lat.download(), s)


# a sweep in one pass of the four-stage kernel (two sweeps per pass selected;
# the mixed cycle adds one in-place phase); tile = (V, Ty, Tz) or None for the
# default tile
@pytest.mark.parametrize("mixed", [False, True], ids=["01", "mixed"])
@pytest.mark.parametrize("L,B,tile", [(64, 2, None), (64, 8, None), (64, 32, None),
                                      (128, 4, None), (128, 64, None), (192, 16, None),
                                      (192, 32, None), (256, 2, None), (256, 4, (4, 24, 8)),
                                      (256, 16, None), (256, 64, None), (256, 128, (4, 120, 40)),
                                      (512, 8, (4, 56, 16)), (512, 256, (4, 56, 64)),
                                      # 1024 lanes (the mixed cycle cuts the rows to 56)
                                      (512, 16, (2, 248, 16))])
def test_double_checkerboard_one_pass_matches_oracle(qz, orc, L, B, tile, mixed):
    seed = 190 + L + B + (500 if mixed else 0)
    say("double checkerboard one pass", L, B, tile, "mixed" if mixed else "01")
    lat = qz.Lattice(L, seed, "bit")
    lat.set_double_checkerboard(B)
    if mixed:
        lat.set_cycle(True)
    if tile is None:
        lat.set_pass(2)
    else:
        lat.set_pass(2, *tile)
    n = 5 if L < 256 else 3
    tr = lat.run(n, 1)
    s = orc.init(L, seed)
    want = orc.run_double(s, B, seed, 0, n, 1, mixed=mixed)
    assert np.array_equal(tr.astype(np.int64), want)
    assert np.array_equal(lat.download(), s)


@pytest.mark.parametrize("mixed", [False, True], ids=["01", "mixed"])
@pytest.mark.parametrize("B", [8, 16])
def test_double_checkerboard_one_pass_large(qz, B, mixed):
    """L = 1024, the paired tile of the large lattices: the one-pass sweep and
    the in-place phases (checked against the oracle above) give the same bond
    and flip traces and the same lattice."""
    L, seed = 1024, 77 + B
    say("double checkerboard one pass vs phases", L, B, "mixed" if mixed else "01")
    one = qz.Lattice(L, seed, "bit")
    one.set_double_checkerboard(B)
    one.set_cycle(mixed)
    one.set_pass(2, 4, 56, 64)
    Bo, Fo = one.run_traced(4, 1)
    ph = qz.Lattice(L, seed, "bit")
    ph.set_double_checkerboard(B)
    ph.set_cycle(mixed)
    ph.set_pass(1)
    Bp, Fp = ph.run_traced(4, 1)
    assert np.array_equal(Bo, Bp)
    assert np.array_equal(Fo, Fp)
    assert np.array_equal(one.download(), ph.download())


def test_double_checkerboard_rejects(qz):
    lat = qz.Lattice(64, 1, "bit")
    for B in (3, 64, 1):
        with pytest.raises(qz.QuenchError):
            lat.set_double_checkerboard(B)
    i8 = qz.Lattice(16, 1, "i8")
    with pytest.raises(qz.QuenchError):
        i8.set_double_checkerboard(4)


# --------------------------------------------------------------------------
# accepted flips traced beside the bond count
# --------------------------------------------------------------------------
@pytest.mark.parametrize("layout,L,mode", [("i8", 16, "01"), ("i8", 34, "mixed"),
                                           ("bit", 64, "01"), ("bit", 128, "mixed"),
                                           ("bit", 128, "pass2"), ("bit", 192, "pass2"),
                                           ("bit", 64, "dcb"), ("bit", 128, "dcb-mixed"),
                                           ("bit", 256, "dcb"), ("bit", 256, "dcb-mixed"),
                                           ("bit", 128, "dcb-pass2"), ("bit", 256, "dcb-pass2"),
                                           ("bit", 128, "mixed-pass2"), ("bit", 256, "mixed-pass2"),
                                           ("bit", 128, "dcb-mixed-pass2"),
                                           ("bit", 256, "dcb-mixed-pass2")])
def test_flip_trace_matches_oracle(qz, orc, layout, L, mode):
    seed = 300 + L
    say("flips", layout, L, mode)
    lat = qz.Lattice(L, seed, layout)
    mixed = mode in ("mixed", "mixed-pass2", "dcb-mixed", "dcb-mixed-pass2")
    double_B = 4 if mode.startswith("dcb") else 0
    if mixed:
        lat.set_cycle(True)
    if double_B:
        lat.set_double_checkerboard(double_B)
    if mode in ("pass2", "mixed-pass2", "dcb-pass2", "dcb-mixed-pass2"):
        lat.set_pass(2)
    for every, n in ((1, 5), (3, 9)):
        B, F = lat.run_traced(n, every)
        s = lat.download()
        t0 = lat.t - n
        # replay the same sweeps with the oracle from the state before them
        lat2 = qz.Lattice(L, seed, layout)
        if mixed:
            lat2.set_cycle(True)
        if double_B:
            lat2.set_double_checkerboard(double_B)
        lat2.run(t0)
        s0 = lat2.download()
        wantB, wantF = orc.run_traced(s0, seed, t0, n, every, mixed=mixed, double_B=double_B)
        assert np.array_equal(B, wantB), (every, n)
        assert np.array_equal(F, wantF), (every, n)
        assert np.array_equal(s0, s)


def test_run_device_traced_matches_host(qz):
    import torch
    L, seed = 128, 17
    a = qz.Lattice(L, seed, "bit")
    b = qz.Lattice(L, seed, "bit")
    b.set_pass(2)
    B, F = a.run_traced(20, 2)
    dB = torch.zeros(10, dtype=torch.int64, device="cuda")
    dF = torch.zeros(10, dtype=torch.int64, device="cuda")
    b.run_device_traced(20, 2, dB, dF)
    torch.cuda.synchronize()
    assert np.array_equal(dB.cpu().numpy(), B)
    assert np.array_equal(dF.cpu().numpy(), F)
    assert np.array_equal(a.download(), b.download())


@pytest.mark.parametrize("layout,L", [("i8", 4), ("i8", 6), ("bit", 64)])
def test_zero_sweep_calls_change_nothing(qz, layout, L):
    """Empty runs: zero sweeps with and without traces, an empty list of
    traced sweeps, and an asynchronous zero-sweep run leave the state and
    the time as they were and return empty traces."""
    import torch
    say("zero sweeps", layout, L)
    lat = qz.Lattice(L, 5, layout)
    lat.run(3)
    s0, t0 = lat.download(), lat.t
    assert lat.run(0).size == 0
    assert lat.run(0, 1).size == 0
    B, F = lat.run_at(0, [])
    assert B.size == 0 and F.size == 0
    dev = torch.full((2,), -7, dtype=torch.int64, device="cuda")
    lat.run_device(0, 1, dev)
    torch.cuda.synchronize()
    assert dev.cpu().tolist() == [-7, -7]
    assert lat.t == t0 and np.array_equal(lat.download(), s0)
    # and the trajectory goes on as if nothing had been called
    ref = qz.Lattice(L, 5, layout)
    ref.run(3)
    assert np.array_equal(lat.run(4, 2), ref.run(4, 2))
    assert np.array_equal(lat.download(), ref.download())


def test_batch_zero_sweeps_and_all_parked(qz):
    """A batch advanced zero sweeps, or with every slot parked, keeps its
    states and times; unparked, each slot goes on exactly as a lone run."""
    specs = [(64, 71), (128, 72)]
    b = qz.Batch(specs, trace_every=5, trace_cap=16)
    b.run(10)
    b.sync()
    states = [b.download(i) for i in range(len(specs))]
    b.run(0)
    for i in range(len(specs)):
        b.set_active(i, False)
    b.run(20)
    b.sync()
    for i, (L, seed) in enumerate(specs):
        assert b.time(i) == 10
        assert np.array_equal(b.download(i), states[i])
        b.set_active(i, True)
    b.run(10)
    b.sync()
    for i, (L, seed) in enumerate(specs):
        lone = qz.Lattice(L, seed, "bit")
        tr = lone.run(20, 5)
        assert b.time(i) == 20
        assert np.array_equal(b.download(i), lone.download())
        assert np.array_equal(b.trace(i, 10, 2), tr[2:4])


@pytest.mark.parametrize("L,mixed", [(16, False), (32, True)])
def test_i8_onchip_long_run_in_pieces(qz, orc, L, mixed):
    """Small int8 lattices run on chip in launches of up to 65536 sweeps (whole
    multiples of the trace cadence): a run across a launch boundary, traced
    and untraced, equals the oracle's."""
    say("i8 on chip", L, mixed)
    seed = 70 + L
    lat = qz.Lattice(L, seed, "i8")
    lat.set_cycle(mixed)
    n, every = 70_000, 7_000
    tr = lat.run(n, every)
    s = orc.init(L, seed)
    want = orc.run(s, seed, 0, n, every, mixed=mixed)
    assert np.array_equal(tr.astype(np.int64), want)
    assert np.array_equal(lat.download(), s)
    lat.run(3)
    orc.run(s, seed, n, 3, mixed=mixed)
    assert np.array_equal(lat.download(), s)
