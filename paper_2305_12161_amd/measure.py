"""Host-side derivations from the library's integer measurements (double precision).

  ell_E = 3N / B             energy-excess length: the mean distance between
                             unsatisfied bonds along an axis (+inf when B = 0)
  C_a(r) = S_a(r)/N - (M/N)^2  connected two-point function along axis a
                             (Results, eq:correlation function), per lattice
  ell_C                      where the axis mean of C first drops below c = 1/2,
                             linearly interpolated (Results: ell from C = 0.5)
"""
import math

import numpy as np


def energy_length(B: int, N: int) -> float:
    return math.inf if B == 0 else 3.0 * N / B


def connected(S: np.ndarray, M: int, N: int) -> np.ndarray:
    m = M / N
    return np.asarray(S, dtype=np.float64) / N - m * m


def crossing_length(S: np.ndarray, M: int, N: int, c: float = 0.5) -> float:
    """First r where mean_a C_a(r) < c, linearly interpolated from r - 1.

    nan if C(0) <= c (no correlated domains to measure); inf if C never drops
    below c up to r = L/2 (the length has saturated at the box size).
    """
    cm = connected(S, M, N).mean(axis=0)
    if cm[0] <= c:
        return math.nan
    below = np.nonzero(cm < c)[0]
    if below.size == 0:
        return math.inf
    r = int(below[0])
    return (r - 1) + (cm[r - 1] - c) / (cm[r - 1] - cm[r])
