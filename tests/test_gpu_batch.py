"""Batched replicas: every replica equals the same (L, seed) run alone, and the
oracle, bit for bit, whatever the batch composition, tuning or graph use."""
import os

import numpy as np
import pytest

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


MIX = [(64, 11), (128, 12), (64, 13), (192, 14), (256, 15), (64, 2**63 + 5), (128, 17), (192, 18)]


def alone(qz, L, seed, n, every):
    lat = qz.Lattice(L, seed, "bit")
    tr = lat.run(n, every)
    return tr, lat.download()


@pytest.mark.parametrize("graph_sweeps", [0, 4, 7])
def test_batch_matches_single_lattices(qz, graph_sweeps):
    n, every = 30, 3
    print("batch mix graph", graph_sweeps, flush=True)
    b = qz.Batch(MIX, trace_every=every, trace_cap=64)
    b.set_tuning(64, 0, graph_sweeps)
    b.run(n)
    b.sync()
    for slot, (L, seed) in enumerate(MIX):
        tr, s = alone(qz, L, seed, n, every)
        assert b.time(slot) == n
        assert np.array_equal(b.trace(slot, 0, n // every), tr), (slot, L)
        assert np.array_equal(b.download(slot), s), (slot, L)


def test_batch_tunings_agree(qz):
    n = 12
    ref = qz.Batch(MIX[:5], trace_every=2, trace_cap=16)
    ref.run(n)
    ref.sync()
    for tz in ((64, 8), (128, 32), (256, 64), (192, 16), (64, 2), (128, 4), (256, 1), (192, 3)):
        b = qz.Batch(MIX[:5], trace_every=2, trace_cap=16)
        b.set_tuning(tz[0], tz[1], 5)
        b.run(n)
        b.sync()
        for slot in range(5):
            assert np.array_equal(b.trace(slot, 0, n // 2), ref.trace(slot, 0, n // 2))
            assert np.array_equal(b.download(slot), ref.download(slot))


def test_batch_matches_oracle(qz, orc):
    specs = [(64, 101), (64, 102), (128, 103)]
    n, every = 16, 4
    b = qz.Batch(specs, trace_every=every, trace_cap=8)
    b.run(n)
    b.sync()
    for slot, (L, seed) in enumerate(specs):
        s = orc.init(L, seed)
        want = orc.run(s, seed, 0, n, every)
        assert np.array_equal(b.trace(slot, 0, n // every).astype(np.int64), want)
        assert np.array_equal(b.download(slot), s)
        assert np.array_equal(b.bonds(slot), orc.bonds(s))
        S, M = b.corr(slot)
        So, Mo = orc.corr(s)
        assert M == Mo and np.array_equal(S, So)


def test_batch_corr_on_matrix_cores(qz, orc):
    """An L = 256 replica (all three axes on the matrix cores, the x axis
    through the replica's idle copy) against the oracle, measured between
    runs without changing the trajectory of it or of its neighbour."""
    specs = [(256, 211), (64, 212)]
    b = qz.Batch(specs, trace_every=3, trace_cap=16)
    ref = qz.Batch(specs, trace_every=3, trace_cap=16)
    s = orc.init(256, 211)
    t = 0
    for n in (6, 9):
        b.run(n)
        ref.run(n)
        b.sync()
        orc.run(s, 211, t, n)
        t += n
        S, M = b.corr(0)
        So, Mo = orc.corr(s)
        assert M == Mo and np.array_equal(S, So), t
    b.sync()
    ref.sync()
    for slot in range(2):
        assert np.array_equal(b.trace(slot, 0, 5), ref.trace(slot, 0, 5))
        assert np.array_equal(b.download(slot), ref.download(slot))


def test_slot_reset_and_parking(qz):
    specs = [(64, 1), (64, 2), (128, 3)]
    b = qz.Batch(specs, trace_every=5, trace_cap=32)
    b.run(10)
    b.set_active(1, False)          # slot 1 parked at t = 10
    b.run(7)
    b.reset(0, 999)                 # slot 0 restarted from seed 999 at t = 0
    b.run(13)
    b.set_active(1, True)
    b.run(5)
    b.sync()
    # slot 0: seed 999 for 18 sweeps
    tr, s = alone(qz, 64, 999, 15, 5)
    assert b.time(0) == 18
    assert np.array_equal(b.trace(0, 0, 3), tr)
    lat = qz.Lattice(64, 999, "bit")
    lat.run(18)
    assert np.array_equal(b.download(0), lat.download())
    # slot 1: seed 2, 15 sweeps in total (parked for 20 of them)
    lat = qz.Lattice(64, 2, "bit")
    tr = lat.run(15, 5)
    assert b.time(1) == 15
    assert np.array_equal(b.trace(1, 0, 3), tr)
    assert np.array_equal(b.download(1), lat.download())
    # slot 2 ran all 35
    lat = qz.Lattice(128, 3, "bit")
    tr = lat.run(35, 5)
    assert np.array_equal(b.trace(2, 0, 7), tr)
    assert np.array_equal(b.download(2), lat.download())


def test_trace_ring_limits(qz):
    b = qz.Batch([(64, 1)], trace_every=2, trace_cap=4)
    b.run(20)
    b.sync()
    with pytest.raises(qz.QuenchError):
        b.trace(0, 0, 3)            # overwritten
    with pytest.raises(qz.QuenchError):
        b.trace(0, 18, 2)           # t = 20 not yet recorded
    with pytest.raises(qz.QuenchError):
        b.trace(0, 3, 1)            # not a multiple of trace_every
    lat = qz.Lattice(64, 1, "bit")
    tr = lat.run(20, 2)
    assert np.array_equal(b.trace(0, 12, 4), tr[6:10])


def test_batch_rejects_bad_sizes(qz):
    with pytest.raises(qz.QuenchError):
        qz.Batch([(96, 1)])
    with pytest.raises(qz.QuenchError):
        qz.Batch([(320, 1)])
    b = qz.Batch([(64, 1)])
    with pytest.raises(qz.QuenchError):
        b.set_tuning(64, 3, 5)       # Tz must divide L


# --------------------------------------------------------------------------
# the batch boundary: traces returned by the run, t_max, slot replacement,
# the tuning text and the library's own autotune
# --------------------------------------------------------------------------
def test_batch_run_returns_traces_and_stops_at_t_max(qz):
    """qz_batch_run's host trace: entry i of a slot is B(tau + i * every); a
    slot with t_max stops there on the device (even inside a graph), and
    its later entries read -1."""
    every = 3
    specs = [(64, 31, 0), (128, 32, 20), (192, 33, 9), (256, 34, 0), (64, 35, 1)]
    b = qz.Batch(specs, trace_every=every, trace_cap=8, tuning={"graph_sweeps": 6})
    print("batch trace run, tuning", b.tuning(), flush=True)
    n1, n2 = 12, 17
    tr1 = b.run(n1, every)
    tr2 = b.run(n2, every)
    assert tr1.shape == (5, 4) and tr2.shape == (5, 6)
    for slot, (L, seed, t_max) in enumerate(specs):
        end = t_max if t_max else n1 + n2
        assert b.time(slot) == end, slot
        ref = qz.Lattice(L, seed, "bit")
        full = ref.run(30, 1)                     # B(0) .. B(29)
        # the first run starts at t = 0, the second at t = 12
        for tr, t0, n in ((tr1, 0, n1), (tr2, n1, n2)):
            tau = -(-t0 // every) * every
            for i in range(tr.shape[1]):
                t = tau + i * every
                want = int(full[t]) if (t < t0 + n and t < end) else -1
                assert int(tr[slot, i]) == want, (slot, t)
        lat = qz.Lattice(L, seed, "bit")
        lat.run(end)
        assert np.array_equal(b.download(slot), lat.download()), slot


def test_batch_slot_replace(qz):
    """A slot takes a new replica of any side up to the one it was created
    with; the new replica follows its lone trajectory, and the others are
    unaffected (the launch's tiles are rebuilt when a side changes)."""
    specs = [(256, 41), (128, 42), (64, 43)]
    b = qz.Batch(specs, trace_every=2, trace_cap=16, tuning={"graph_sweeps": 4})
    b.run(8)
    b.replace(0, 64, 77, 10)           # a 256 slot now holds an L = 64 replica, t_max 10
    b.replace(2, 64, 78)               # same side, new seed
    with pytest.raises(qz.QuenchError):
        b.replace(1, 256, 79)          # larger than the slot was sized for
    with pytest.raises(qz.QuenchError):
        b.replace(1, 96, 79)           # not a batch size
    b.run(12)
    b.sync()
    assert [b.time(k) for k in range(3)] == [10, 20, 12]
    for slot, (L, seed, n) in enumerate(((64, 77, 10), (128, 42, 20), (64, 78, 12))):
        lat = qz.Lattice(L, seed, "bit")
        tr = lat.run(n, 2)
        first = 8 if slot == 1 else 0
        assert np.array_equal(b.trace(slot, first, (n - first) // 2), tr[first // 2:]), slot
        assert np.array_equal(b.download(slot), lat.download()), slot
    # back to the full side
    b.replace(0, 256, 80)
    b.run(4)
    lat = qz.Lattice(256, 80, "bit")
    lat.run(4)
    assert np.array_equal(b.download(0), lat.download())


def test_batch_autotune_and_tuning_text(qz):
    """Without a tuning the library times candidate plane counts at creation
    and draws the starts again; with a tuning text it uses the text.  Both
    follow the lone trajectories."""
    specs = [(64, 51), (128, 52), (256, 53), (192, 54)]
    auto = qz.Batch(specs, trace_every=2, trace_cap=16, tuning=None)
    given = qz.Batch(specs, trace_every=2, trace_cap=16,
                     tuning='{"graph_sweeps": 5, "tz": {"64": 4, "256": 16}}')
    ta, tg = auto.tuning(), given.tuning()
    print("autotuned", ta, "given", tg, flush=True)
    assert ta["source"] == "autotune" and tg["source"] == "json"
    assert tg["graph_sweeps"] == 5
    assert tg["tz"] == {"64": 4, "128": 8, "192": 8, "256": 16}
    for L, tz in ta["tz"].items():
        assert int(L) % tz == 0
    for b in (auto, given):
        assert [b.time(k) for k in range(4)] == [0, 0, 0, 0]
        b.run(10)
        b.sync()
    for slot, (L, seed) in enumerate(specs):
        lat = qz.Lattice(L, seed, "bit")
        tr = lat.run(10, 2)
        for b in (auto, given):
            assert np.array_equal(b.trace(slot, 0, 5), tr), slot
            assert np.array_equal(b.download(slot), lat.download()), slot


@pytest.mark.parametrize("graph_sweeps", [0, 5, 12])
def test_batch_onchip_side64(qz, orc, graph_sweeps):
    """Side-64 replicas held on chip (all sweeps of a group in one launch)
    against the same batch run as sub-tiles, against lone runs, and against
    the oracle: traces at every sweep, a t_max inside a group, parking."""
    specs = [(64, 61, 0), (128, 62, 0), (64, 63, 17), (192, 64, 0), (64, 2**63 + 65, 0),
             (64, 66, 3)]
    n, every = 30, 1
    runs = {}
    for onchip in (1, 0):
        b = qz.Batch(specs, trace_every=every, trace_cap=64,
                     tuning={"onchip": onchip, "graph_sweeps": graph_sweeps})
        assert b.tuning()["onchip"] == onchip
        b.run(10)
        b.set_active(4, False)          # parked for 10 sweeps
        b.run(10)
        b.set_active(4, True)
        b.run(10)
        b.sync()
        runs[onchip] = [(b.time(k), b.trace(k, 0, min(b.time(k), 30)), b.download(k))
                        for k in range(len(specs))]
    for k, (L, seed, t_max) in enumerate(specs):
        t_end = 20 if k == 4 else (t_max or n)
        (t1, tr1, s1), (t0, tr0, s0) = runs[1][k], runs[0][k]
        assert t1 == t0 == t_end, (k, t1, t0)
        assert np.array_equal(tr1, tr0) and np.array_equal(s1, s0), k
        lat = qz.Lattice(L, seed, "bit")
        tr = lat.run(t_end, 1)
        assert np.array_equal(tr1, tr), k
        assert np.array_equal(s1, lat.download()), k
        if L == 64 and k < 3:
            s = orc.init(L, seed)
            want = orc.run(s, seed, 0, t_end, 1)
            assert np.array_equal(tr1.astype(np.int64), want), k
            assert np.array_equal(s1, s), k
