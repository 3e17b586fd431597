"""ctypes binding of the C oracle plus the oracle's own host-side derivations.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product package.

Every function follows the definitions of arXiv:2305.12161:
  * update rule: T -> 0 Glauber acceptance (Methods, equation
    equ:glauberAcceptance); one MCS = N proposals (Methods, rsf update);
  * sweep order: checkerboard colour 0 then colour 1 every sweep (Methods,
    "Checkerboard update"; Supplementary Methods I B, "01 cycle");
  * C(r,t) = <s_i s_j> - <s_i><s_j> (Results, eq:correlation function),
    here per lattice along the three axes, and ell from the intercept of C
    with c = 0.5 (Results, dynamical-scaling paragraph).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i8p = ctypes.POINTER(ctypes.c_int8)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build_oracle
        build_oracle.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.or_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    lib.or_philox4x32_10.restype = None
    lib.or_tie_bit.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint64]
    lib.or_tie_bit.restype = ctypes.c_int
    lib.or_init_bit.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.or_init_bit.restype = ctypes.c_int
    lib.or_init.argtypes = [ctypes.c_int, ctypes.c_uint64, _i8p]
    lib.or_init.restype = None
    lib.or_half_sweep.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, _i8p]
    lib.or_half_sweep.restype = ctypes.c_int64
    lib.or_sweep.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, _i8p]
    lib.or_sweep.restype = ctypes.c_int64
    lib.or_bonds.argtypes = [ctypes.c_int, _i8p, _i64p]
    lib.or_bonds.restype = None
    lib.or_corr.argtypes = [ctypes.c_int, _i8p, _i64p, _i64p]
    lib.or_corr.restype = None
    lib.or_run.argtypes = [ctypes.c_int, ctypes.c_uint64, _i8p, ctypes.c_uint64, ctypes.c_uint64,
                           ctypes.c_uint64, _i64p]
    lib.or_run.restype = None
    lib.or_window_advance.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, _i8p, ctypes.c_uint64,
                                      ctypes.c_uint64]
    lib.or_window_advance.restype = None
    lib.or_window_advance_cycle.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int, ctypes.c_int, _i8p,
                                            ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
    lib.or_window_advance_cycle.restype = None
    lib.or_first_colour.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
    lib.or_first_colour.restype = ctypes.c_int
    lib.or_sweep_mixed.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, _i8p]
    lib.or_sweep_mixed.restype = ctypes.c_int64
    lib.or_run_cycle.argtypes = [ctypes.c_int, ctypes.c_uint64, _i8p, ctypes.c_uint64,
                                 ctypes.c_uint64, ctypes.c_uint64, _i64p, ctypes.c_int]
    lib.or_run_cycle.restype = None
    lib.or_sweep_double.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                    _i8p]
    lib.or_sweep_double.restype = ctypes.c_int64
    lib.or_sweep_double_mixed.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                          ctypes.c_uint32, _i8p]
    lib.or_sweep_double_mixed.restype = ctypes.c_int64
    lib.or_coarse_first.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
    lib.or_coarse_first.restype = ctypes.c_int
    lib.or_fine_first.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64]
    lib.or_fine_first.restype = ctypes.c_int
    lib.or_init_window.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, _i8p]
    lib.or_init_window.restype = None
    lib.or_set_threads.argtypes = [ctypes.c_int]
    lib.or_set_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _i8(a):
    assert a.dtype == np.int8 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_i8p)


def _check_L(L):
    if L < 4 or L % 2:
        raise ValueError("the checkerboard needs an even L >= 4 under periodic boundaries")


def set_threads(n: int = 0) -> int:
    """Set the OpenMP thread count (0 keeps the current one); returns the count in use."""
    return int(_load().or_set_threads(int(n)))


def philox4x32_10(ctr, key):
    """Raw Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib.or_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def tie_bit(seed: int, t: int, p: int, j: int) -> int:
    return int(_load().or_tie_bit(seed, t, p, j))


def init_bit(seed: int, i: int) -> int:
    return int(_load().or_init_bit(seed, i))


def init(L: int, seed: int) -> np.ndarray:
    """Infinite-temperature start: i.i.d. fair +-1 spins, shape (L, L, L) indexed [z, y, x]."""
    _check_L(L)
    s = np.empty((L, L, L), dtype=np.int8)
    _load().or_init(L, seed, _i8(s))
    return s


def init_window(L: int, seed: int, origin, W: int) -> np.ndarray:
    """The infinite-temperature start of the L^3 lattice restricted to a W^3 window."""
    _check_L(L)
    w = np.empty((W, W, W), dtype=np.int8)
    ox, oy, oz = (int(v) % L for v in origin)
    _load().or_init_window(L, seed, ox, oy, oz, W, _i8(w))
    return w


def half_sweep(s: np.ndarray, seed: int, t: int, p: int) -> int:
    """In-place half-sweep of colour p during sweep t; returns the number of flips."""
    L = s.shape[0]
    _check_L(L)
    return int(_load().or_half_sweep(L, seed, t, p, _i8(s)))


def sweep(s: np.ndarray, seed: int, t: int) -> int:
    L = s.shape[0]
    _check_L(L)
    return int(_load().or_sweep(L, seed, t, _i8(s)))


def bonds(s: np.ndarray) -> np.ndarray:
    """Per-axis unsatisfied-bond counts [B_x, B_y, B_z]."""
    L = s.shape[0]
    B = np.zeros(3, dtype=np.int64)
    _load().or_bonds(L, _i8(s), B.ctypes.data_as(_i64p))
    return B


def corr(s: np.ndarray):
    """Axis correlation sums S[a, r] for r = 0..L/2 and magnetisation M."""
    L = s.shape[0]
    S = np.zeros((3, L // 2 + 1), dtype=np.int64)
    M = np.zeros(1, dtype=np.int64)
    _load().or_corr(L, _i8(s), S.ctypes.data_as(_i64p), M.ctypes.data_as(_i64p))
    return S, int(M[0])


def run(s: np.ndarray, seed: int, t0: int, n: int, every: int = 0,
        mixed: bool = False) -> np.ndarray:
    """Advance n sweeps in place from time t0; returns B(t0 + k*every) for k < n/every.

    mixed=True uses the mixed cycle (colour order drawn per sweep), else the 01 cycle.
    """
    L = s.shape[0]
    _check_L(L)
    if every > 0:
        tr = np.zeros((n + every - 1) // every, dtype=np.int64)
        ptr = tr.ctypes.data_as(_i64p)
    else:
        tr = np.zeros(0, dtype=np.int64)
        ptr = None
    _load().or_run_cycle(L, seed, _i8(s), t0, n, every, ptr, 1 if mixed else 0)
    return tr


def run_traced(s: np.ndarray, seed: int, t0: int, n: int, every: int, mixed: bool = False,
               double_B: int = 0):
    """n sweeps in place from t0; at every `every`-th sweep record the bond count
    of the state entering it and the number of sites it flips.  double_B > 0
    runs the double checkerboard with cubes of that side."""
    L = s.shape[0]
    _check_L(L)
    lib = _load()
    B, F = [], []
    for k in range(n):
        t = t0 + k
        traced = every > 0 and k % every == 0
        if traced:
            B.append(int(bonds(s).sum()))
        if double_B:
            f = sweep_double(s, double_B, seed, t, mixed)
        elif mixed:
            f = int(lib.or_sweep_mixed(L, seed, t, _i8(s)))
        else:
            f = int(lib.or_sweep(L, seed, t, _i8(s)))
        if traced:
            F.append(f)
    return np.array(B, dtype=np.int64), np.array(F, dtype=np.int64)


def first_colour(seed: int, t: int) -> int:
    """Mixed cycle: the colour updated first in sweep t."""
    return int(_load().or_first_colour(seed, t))


def sweep_double(s: np.ndarray, B: int, seed: int, t: int, mixed: bool = False) -> int:
    """Double-checkerboard sweep with coarse cubes of side B (needs L % 2B == 0).

    mixed=False: the 01 order (coarse 0, then 1; fine 0 then 1 in each cube).
    mixed=True: coarse order drawn per sweep, fine order per cube and sweep.
    """
    L = s.shape[0]
    _check_L(L)
    if B < 1 or L % (2 * B):
        raise ValueError("need L % (2B) == 0")
    if mixed:
        f = int(_load().or_sweep_double_mixed(L, B, seed, t, _i8(s)))
        if f < 0:
            raise MemoryError("order table")
        return f
    return int(_load().or_sweep_double(L, B, seed, t, _i8(s)))


def run_double(s: np.ndarray, B: int, seed: int, t0: int, n: int, every: int = 0,
               mixed: bool = False) -> np.ndarray:
    """n double-checkerboard sweeps from t0; B(t0 + k*every) traced at sweep starts."""
    tr = []
    for k in range(n):
        if every and k % every == 0:
            tr.append(int(bonds(s).sum()))
        sweep_double(s, B, seed, t0 + k, mixed)
    return np.array(tr, dtype=np.int64)


def coarse_first(seed: int, t: int) -> int:
    """Mixed double checkerboard: the coarse colour updated first in sweep t."""
    return int(_load().or_coarse_first(seed, t))


def fine_first(seed: int, t: int, b: int) -> int:
    """Mixed double checkerboard: the fine colour cube b updates first in sweep t."""
    return int(_load().or_fine_first(seed, t, b))


def sweep_mixed(s: np.ndarray, seed: int, t: int) -> int:
    L = s.shape[0]
    _check_L(L)
    return int(_load().or_sweep_mixed(L, seed, t, _i8(s)))


def window_advance(L: int, seed: int, origin, w: np.ndarray, t0: int, T: int,
                   mixed: bool = False) -> None:
    """Advance a W^3 window (global corner `origin` = (ox, oy, oz)) by T sweeps in place.

    Sites within local distance 2T of a face are not trustworthy afterwards.
    mixed=True follows the mixed cycle (colour order drawn per sweep).
    """
    W = w.shape[0]
    ox, oy, oz = (int(v) for v in origin)
    if mixed:
        _load().or_window_advance_cycle(L, seed, ox, oy, oz, W, _i8(w), t0, T, 1)
    else:
        _load().or_window_advance(L, seed, ox, oy, oz, W, _i8(w), t0, T)


# --------------------------------------------------------------------------
# Host-side derivations (double precision), written for the oracle only.
# --------------------------------------------------------------------------
def ell_energy(B: int, N: int) -> float:
    """Energy-excess length 3N/B (mean chord between walls along an axis); +inf if B = 0."""
    return float("inf") if B == 0 else 3.0 * N / float(B)


def connected_corr(S: np.ndarray, M: int, N: int) -> np.ndarray:
    """C_a(r) = S_a(r)/N - (M/N)^2, shape (3, L/2+1)."""
    m = M / float(N)
    return S.astype(np.float64) / float(N) - m * m


def ell_intercept(S: np.ndarray, M: int, N: int, c: float = 0.5) -> float:
    """Linear-interpolated first crossing of the axis-averaged C(r) with c.

    Returns nan when C(0) <= c (no length defined) and inf when C stays >= c
    up to r = L/2 (saturated).
    """
    Cbar = connected_corr(S, M, N).mean(axis=0)
    if not Cbar[0] > c:
        return float("nan")
    for r in range(1, Cbar.shape[0]):
        if Cbar[r] < c:
            return (r - 1) + (Cbar[r - 1] - c) / (Cbar[r - 1] - Cbar[r])
    return float("inf")


# --------------------------------------------------------------------------
# The paper's FFT route to C(r,t) (Methods, "Calculating the correlation
# function", eq:sisik), with numpy's FFT as the library primitive, followed by
# the radial (spherical-shell) average, and the structure factor.
# --------------------------------------------------------------------------
def _signed(L):
    v = np.arange(L)
    return np.where(v < L // 2, v, v - L)


def shell_index(L):
    """round(|d|) for every displacement / wavevector, components in [-L/2, L/2)."""
    c = _signed(L).astype(np.float64)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return np.rint(np.sqrt(x * x + y * y + z * z)).astype(np.int64)


def fft_G(s: np.ndarray) -> np.ndarray:
    """G(d) = <s_i s_{i+d}> over i for every displacement d, indexed [dz, dy, dx]."""
    f = s.astype(np.float64)
    F = np.fft.fftn(f)
    return np.fft.ifftn((F * np.conj(F)).real).real / f.size


def fft_corr(s: np.ndarray):
    """Shell means of C(d) = <s_i s_{i+d}> - m^2 and of S(k) = |F s(k)|^2 / N.

    Returns (C, Sk, n_r, n_k, m) with shells b = 0 .. round(sqrt(3) L/2) + 1.
    """
    L = s.shape[0]
    N = L ** 3
    f = s.astype(np.float64)
    F = np.fft.fftn(f)
    P = (F * np.conj(F)).real
    G = np.fft.ifftn(P).real / N            # sum_i s_i s_{i+d} = (1/N) sum_k |F|^2 e^{ikd}
    m = float(f.sum()) / N
    nb = int(0.8660254037844386 * L + 0.5) + 2
    sh = shell_index(L).ravel()
    n = np.bincount(sh, minlength=nb)[:nb]
    gs = np.bincount(sh, weights=G.ravel(), minlength=nb)[:nb]
    ps = np.bincount(sh, weights=P.ravel() / N, minlength=nb)[:nb]
    with np.errstate(invalid="ignore", divide="ignore"):
        C = np.where(n > 0, gs / np.maximum(n, 1) - m * m, 0.0)
        Sk = np.where(n > 0, ps / np.maximum(n, 1), 0.0)
    return C, Sk, n.astype(np.int64), n.astype(np.int64), m
