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
