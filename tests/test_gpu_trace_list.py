"""Listed traced sweeps (qz_run_at, qz_run_device_at): the bond count entering
each listed sweep and the spins it flips, against the oracle's sweep-by-sweep
trace, for every pass layout -- one sweep per pass, two sweeps per pass with
the listed sweep in either position of a pair, the mixed cycle (pairs of equal
and of different first colours), the double checkerboard and int8.  The
lattice after the run equals the oracle's too.  (Methods, "Checkerboard
update"; Supplementary Methods I A, I B.)"""
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


# offsets chosen so that two-sweep passes see listed sweeps at the first
# position only, the second only, both, and neither
AT = [0, 1, 2, 5, 6, 9, 10, 11, 14, 19, 22, 23]
N_SWEEPS = 25


def _oracle(orc, L, seed, t0, n, mixed=False, double_B=0):
    s = orc.init(L, seed)
    if t0:
        if double_B:
            orc.run_double(s, double_B, seed, 0, t0, mixed=mixed)
        else:
            orc.run(s, seed, 0, t0, mixed=mixed)
    B, F = orc.run_traced(s, seed, t0, n, 1, mixed=mixed, double_B=double_B)
    return s, B[AT], F[AT]


@pytest.mark.parametrize("layout,L,sweeps,mixed,dcb", [
    ("bit", 64, 1, False, 0), ("bit", 64, 2, False, 0), ("bit", 128, 2, False, 0),
    ("bit", 256, 2, False, 0), ("bit", 64, 2, True, 0), ("bit", 192, 2, True, 0),
    ("bit", 64, 1, True, 0), ("bit", 128, 2, False, 8), ("bit", 64, 1, True, 4),
    ("i8", 32, 1, False, 0), ("i8", 18, 1, True, 0)])
def test_run_at_matches_oracle(qz, orc, layout, L, sweeps, mixed, dcb):
    seed, t0 = 900 + L, 3
    print("run_at", layout, L, sweeps, mixed, dcb, flush=True)
    lat = qz.Lattice(L, seed, layout)
    if layout == "bit":
        lat.set_pass(sweeps)
    lat.set_cycle(mixed)
    if dcb:
        lat.set_double_checkerboard(dcb)
    lat.run(t0)
    B, F = lat.run_at(N_SWEEPS, AT)
    s, wB, wF = _oracle(orc, L, seed, t0, N_SWEEPS, mixed, dcb)
    assert np.array_equal(B, wB)
    assert np.array_equal(F, wF)
    assert lat.t == t0 + N_SWEEPS
    assert np.array_equal(lat.download(), s)


def test_run_device_at_two_sweep_default_L1024(qz):
    """At a size whose default is two sweeps per pass: the device trace at
    listed sweeps equals the host trace of a one-sweep-per-pass lattice."""
    import torch
    L, seed = 1024, 5
    two = qz.Lattice(L, seed, "bit")
    assert two.pass_config()[0] == 2
    one = qz.Lattice(L, seed, "bit")
    one.set_pass(1)
    dB = torch.full((len(AT),), -1, dtype=torch.int64, device="cuda")
    dF = torch.full((len(AT),), -1, dtype=torch.int64, device="cuda")
    two.run_device_at(N_SWEEPS, AT, dB, dF)
    torch.cuda.synchronize()
    B1, F1 = one.run_traced(N_SWEEPS, 1)
    assert np.array_equal(dB.cpu().numpy(), B1[AT])
    assert np.array_equal(dF.cpu().numpy(), F1[AT])
    for o in ((0, 0, 0), (1000, 17, 511)):
        assert np.array_equal(one.window(o, 40), two.window(o, 40))


def test_run_at_long_lists_and_errors(qz, orc):
    """More listed sweeps than the handle's trace ring holds, and bad lists."""
    L, seed = 64, 77
    lat = qz.Lattice(L, seed, "bit")
    lat.set_pass(2)
    n = 9000
    at = list(range(0, n, 2)) + [n - 1]          # 4501 entries: two pieces
    B, F = lat.run_at(n, at)
    one = qz.Lattice(L, seed, "bit")
    one.set_pass(1)
    B1, F1 = one.run_traced(n, 1)
    assert np.array_equal(B, B1[at]) and np.array_equal(F, F1[at])
    assert np.array_equal(lat.download(), one.download())
    t = lat.t
    for bad in ([3, 3], [5, 2], [0, n]):
        with pytest.raises(qz.QuenchError) as e:
            lat.run_at(n, bad)
        assert e.value.status == qz.QZ_EINVAL
    assert lat.t == t          # rejected before any sweep
    B, F = lat.run_at(4, [])
    assert B.size == 0 and lat.t == t + 4
