"""The product's host derivations (paper_2305_12161_amd.measure) against the
oracle's own: energy-excess length 3N/B, the connected C_a(r) (Results,
eq:correlation function) and the c = 0.5 intercept (Results), including the
cases with no length (C(0) <= 1/2: nan) and a saturated one (no crossing up to
L/2: inf).  Inputs are oracle lattices and synthetic profiles."""
import math

import numpy as np
import pytest

from paper_2305_12161_amd import measure


def _same(a, b):
    if math.isnan(b):
        return math.isnan(a)
    if math.isinf(b):
        return a == b
    return abs(a - b) <= 1e-12 * max(1.0, abs(b))


def test_energy_length_matches_oracle(orc):
    for L in (4, 32, 2048):
        N = L ** 3
        for B in (0, 1, 7, 3 * N // 8, 3 * N):
            assert _same(measure.energy_length(B, N), orc.ell_energy(B, N)), (L, B)
    assert measure.energy_length(0, 64) == math.inf


@pytest.mark.parametrize("L,seed,times", [(16, 3, (0, 1, 5, 40)), (32, 9, (0, 2, 30, 300))])
def test_connected_and_crossing_on_oracle_runs(orc, L, seed, times):
    N = L ** 3
    s = orc.init(L, seed)
    t = 0
    for tt in times:
        orc.run(s, seed, t, tt - t)
        t = tt
        S, M = orc.corr(s)
        assert np.allclose(measure.connected(S, M, N), orc.connected_corr(S, M, N),
                           rtol=0, atol=1e-15)
        assert _same(measure.crossing_length(S, M, N), orc.ell_intercept(S, M, N)), (L, tt)
        B = int(orc.bonds(s).sum())
        assert _same(measure.energy_length(B, N), orc.ell_energy(B, N))


def test_crossing_special_cases(orc):
    L = 32
    N = L ** 3
    r = np.arange(L // 2 + 1)
    # fully magnetised: C = 0 everywhere, so C(0) <= 1/2 and no length exists
    S = np.full((3, L // 2 + 1), N, dtype=np.int64)
    assert math.isnan(measure.crossing_length(S, N, N))
    assert math.isnan(orc.ell_intercept(S, N, N))
    # m = 0 and perfect order along every axis: C stays 1, saturated
    assert measure.crossing_length(S, 0, N) == math.inf == orc.ell_intercept(S, 0, N)
    # C(0) exactly 1/2 (|m| = 1/sqrt 2 is not an integer state; use S(0) = N/2 instead)
    S_half = np.tile(np.full(L // 2 + 1, N // 2, dtype=np.int64), (3, 1))
    assert math.isnan(measure.crossing_length(S_half, 0, N))
    assert math.isnan(orc.ell_intercept(S_half, 0, N))
    # crossing exactly on a lattice point, and between points, for uneven axes
    for ell in (1.0, 2.5, 6.25, 15.5):
        prof = np.stack([np.rint(N * np.clip(1.0 - r / (2.0 * ell * f), -1, 1)).astype(np.int64)
                         for f in (0.8, 1.0, 1.2)])
        assert _same(measure.crossing_length(prof, 0, N), orc.ell_intercept(prof, 0, N)), ell
    # a magnetised state: the connected part removes m^2
    m = 0.375
    prof = np.tile(np.rint(N * (m * m + (1 - m * m) * np.exp(-r / 4.0))).astype(np.int64), (3, 1))
    assert _same(measure.crossing_length(prof, int(m * N), N),
                 orc.ell_intercept(prof, int(m * N), N))
