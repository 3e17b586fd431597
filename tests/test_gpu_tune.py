"""The autotuner on small configurations: it times the candidate tilings on
the device, keeps the fastest, and the kept tilings reproduce the same
trajectory as the defaults (the tuning changes speed, never results)."""
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


@pytest.fixture()
def tune(tmp_path, monkeypatch):
    from paper_2305_12161_amd import tune as t
    monkeypatch.setattr(t, "CACHE", str(tmp_path / "tuned.json"))
    return t


def test_tune_single_lattice(qz, tune):
    L, seed = 256, 41
    best1, ms1 = tune.tune_single(L, sweeps=4, verbose=False)
    best2, ms2 = tune.tune_pass2(L, sweeps=4, verbose=False)
    assert best1 in tune.single_candidates(L) and ms1 > 0
    assert best2 in tune.pass2_candidates(L) and ms2 > 0
    assert tune.best_single(L) == best1 and tune.best_pass2(L) == best2
    ref = qz.Lattice(L, seed, "bit")
    ref.set_pass(1)
    a = qz.Lattice(L, seed, "bit")
    a.set_pass(1)
    a.set_tuning(*best1)
    b = qz.Lattice(L, seed, "bit")
    b.set_pass(2, *best2)
    tr = ref.run(12, 3)
    assert np.array_equal(a.run(12, 3), tr)
    assert np.array_equal(b.run(12, 3), tr)
    s = ref.download()
    assert np.array_equal(a.download(), s) and np.array_equal(b.download(), s)


def test_tune_batch(qz, tune):
    specs = [(64, 1), (64, 2), (128, 3)]
    chosen, (graph, ms) = tune.tune_batch(specs, sweeps=20, verbose=False)
    assert set(chosen) == {64, 128} and ms > 0
    for L, Tz in chosen.items():
        assert L % Tz == 0 and tune.best_batch(L) == (Tz, graph)
    # the stored winners reach the library through the batch's tuning text
    text = tune.batch_tuning_json(sorted(chosen))
    assert text is not None
    ref = qz.Batch(specs, trace_every=4, trace_cap=8, tuning=None)     # library autotune
    b = qz.Batch(specs, trace_every=4, trace_cap=8, tuning=text)
    got = b.tuning()
    assert got["source"] == "json" and got["graph_sweeps"] == min(graph, 8 * 4)
    assert {int(k): v for k, v in got["tz"].items()} == chosen
    assert ref.tuning()["source"] == "autotune"
    ref.run(16)
    b.run(16)
    ref.sync()
    b.sync()
    for slot in range(len(specs)):
        assert np.array_equal(b.trace(slot, 0, 4), ref.trace(slot, 0, 4))
        assert np.array_equal(b.download(slot), ref.download(slot))
