"""Seeded synthetic workloads: lattice sizes, schedules, special initial states
and served request streams.

This module holds input generators only -- none of the dynamics or the
measurement arithmetic -- so that the product path and the CPU oracle can be
fed identical inputs without sharing any of the method's code.

The workloads stand in for the paper's runs (Results: L = 128 ... 2048 from
random starts, 40 realisations each, up to a few 1e5 MCS); no dataset is
involved, every input is drawn from a seed.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


def log_times(t_max: int, n: int = 40) -> List[int]:
    """n log-spaced integer measurement times from 1 to t_max, strictly increasing.

    t_k = max(round(t_max^(k/(n-1))), t_{k-1} + 1), so t_0 = 1 and t_{n-1} = t_max.
    """
    if t_max < n:
        raise ValueError("t_max must be >= n")
    out: List[int] = []
    for k in range(n):
        v = int(np.floor(t_max ** (k / (n - 1)) + 0.5))
        if out:
            v = max(v, out[-1] + 1)
        out.append(v)
    out[-1] = t_max
    if out[-2] >= t_max:
        raise ValueError("schedule collided with t_max")
    return out


@dataclass(frozen=True)
class LatticeRun:
    """One quench: lattice size, layout, seed, length and what is measured."""
    name: str
    L: int
    layout: str            # "i8" or "bit"
    seed: int
    t_max: int
    trace_every: int = 0   # B(t) every this many MCS (0 = none)
    corr_times: tuple = ()  # times at which the axis correlation is taken


RUN_I8_L32 = LatticeRun("L32_i8_1e3", 32, "i8", 1, 1000, trace_every=10)
RUN_I8_L256 = LatticeRun("L256_i8_1e4", 256, "i8", 2, 10_000, trace_every=0,
                         corr_times=tuple(log_times(10_000)))
RUN_BIT_L2048 = LatticeRun("L2048_bit_1e5", 2048, "bit", 3, 100_000, trace_every=0,
                           corr_times=tuple(log_times(100_000)))


@dataclass(frozen=True)
class ReplicaSpec:
    L: int
    seed: int
    t_max: int


def batch_mix_584() -> List[ReplicaSpec]:
    """512 replicas at L=64, 64 at L=128 and 8 at L=256, seeds 0x40000000 + r, 1e4 MCS."""
    specs: List[ReplicaSpec] = []
    r = 0
    for L, count in ((64, 512), (128, 64), (256, 8)):
        for _ in range(count):
            specs.append(ReplicaSpec(L, 0x4000_0000 + r, 10_000))
            r += 1
    return specs


@dataclass(frozen=True)
class Request:
    idx: int
    L: int
    t_max: int
    seed: int
    arrival_s: float


SERVE_SIZES = (64, 96, 128, 192, 256, 384, 512)
SERVE_TMAX = (1_000, 10_000)
# Device memory for lattice state held at once by the server (admission binds
# on it), the batch slots per size, and the arrival rate: 0.8 of the rate one
# MI355X sustained on this stream, measured once and frozen here.
SERVE_BUDGET_BYTES = 512 << 20
SERVE_BATCH_SLOTS = {64: 8, 128: 8, 192: 8, 256: 8}
SERVE_RATE_PER_S = 52.5   # 0.8 x 65.7 requests/s, the first 300 requests all queued at t = 0


def request_stream(n: int = 2000, rate_per_s: float = 100.0, master_seed: int = 5,
                   sizes=SERVE_SIZES, t_maxes=SERVE_TMAX) -> List[Request]:
    """Served quench stream: L ~ U(sizes), t_max ~ U(t_maxes), Poisson arrivals.

    Request seeds are 0x50000000 + idx; arrivals are exponential gaps at
    rate_per_s, all drawn from numpy's PCG64 with master_seed.
    """
    rng = np.random.Generator(np.random.PCG64(master_seed))
    Ls = rng.choice(np.asarray(sizes), size=n)
    ts = rng.choice(np.asarray(t_maxes), size=n)
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    arr = np.cumsum(gaps) - gaps[0]
    return [Request(i, int(Ls[i]), int(ts[i]), 0x5000_0000 + i, float(arr[i])) for i in range(n)]


# --------------------------------------------------------------------------
# Special initial states, int8 arrays indexed [z, y, x].
# --------------------------------------------------------------------------
def uniform_state(L: int, sign: int = 1) -> np.ndarray:
    return np.full((L, L, L), 1 if sign > 0 else -1, dtype=np.int8)


def isolated_flip(L: int, pos, sign: int = 1) -> np.ndarray:
    s = uniform_state(L, sign)
    x, y, z = pos
    s[z, y, x] = -s[z, y, x]
    return s


def slab(L: int, axis: int = 2) -> np.ndarray:
    """Half the lattice -1 and half +1 along `axis` (two flat walls under periodic BC)."""
    s = uniform_state(L, 1)
    idx = [slice(None)] * 3
    idx[2 - axis] = slice(0, L // 2)
    s[tuple(idx)] = -1
    return s


def flipped_plane(L: int, axis: int = 2, at: int = 0) -> np.ndarray:
    s = uniform_state(L, 1)
    idx = [slice(None)] * 3
    idx[2 - axis] = at
    s[tuple(idx)] = -1
    return s


def flipped_line_x(L: int, y: int, z: int) -> np.ndarray:
    s = uniform_state(L, 1)
    s[z, y, :] = -1
    return s


def neel(L: int) -> np.ndarray:
    """s = (-1)^(x+y+z): +1 on colour 0, -1 on colour 1."""
    z, y, x = np.indices((L, L, L))
    return np.where((x + y + z) % 2 == 0, 1, -1).astype(np.int8)


def flipped_cube(L: int, origin, size: int = 2) -> np.ndarray:
    s = uniform_state(L, 1)
    ox, oy, oz = origin
    for dz in range(size):
        for dy in range(size):
            for dx in range(size):
                s[(oz + dz) % L, (oy + dy) % L, (ox + dx) % L] = -1
    return s


def random_state(L: int, seed: int, p_up: float = 0.5) -> np.ndarray:
    """Arbitrary seeded +-1 state (numpy PCG64), for upload paths and invariants."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.where(rng.random((L, L, L)) < p_up, 1, -1).astype(np.int8)


def menger_state(L: int, k: int, seed: int) -> np.ndarray:
    """Menger-sponge start (Results, sponge test): tiles of (3^k)^3, each tile's
    sponge drawn as up or down spins with probability 1/2 (numpy PCG64).

    Tiles that do not fit wholly at the upper end of an axis are cut off there.
    """
    n = 3 ** k
    cube = np.ones((n, n, n), dtype=bool)
    if k > 0:
        idx = np.arange(n)
        holes = np.zeros((n, n, n), dtype=bool)
        for level in range(k):
            digit = (idx // (3 ** level)) % 3 == 1
            dz, dy, dx = np.meshgrid(digit, digit, digit, indexing="ij")
            holes |= (dx.astype(int) + dy.astype(int) + dz.astype(int)) >= 2
        cube = ~holes
    rng = np.random.Generator(np.random.PCG64(seed))
    nt = (L + n - 1) // n
    signs = rng.choice(np.array([-1, 1], dtype=np.int8), size=(nt, nt, nt))
    s = np.empty((L, L, L), dtype=np.int8)
    for tz in range(nt):
        for ty in range(nt):
            for tx in range(nt):
                sg = signs[tz, ty, tx]
                block = np.where(cube, sg, -sg).astype(np.int8)
                z0, y0, x0 = tz * n, ty * n, tx * n
                z1, y1, x1 = min(z0 + n, L), min(y0 + n, L), min(x0 + n, L)
                s[z0:z1, y0:y1, x0:x1] = block[: z1 - z0, : y1 - y0, : x1 - x0]
    return s
