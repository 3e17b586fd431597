import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-side test")


@pytest.fixture(scope="session")
def orc():
    """The CPU oracle (built on demand)."""
    import oracle
    oracle.oracle._load()
    return oracle


_PIN_DIR = os.path.join(ROOT, "tests", "_pinbin")


def _compile_pin(name, src, extra):
    os.makedirs(_PIN_DIR, exist_ok=True)
    exe = os.path.join(_PIN_DIR, name)
    srcp = os.path.join(_PIN_DIR, name + ".cpp")
    with open(srcp, "w") as f:
        f.write(src)
    subprocess.run(["g++", "-O1", "-std=c++17", *extra, srcp, "-o", exe], check=True)
    return exe


_TORCH_PIN = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>
int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = k0 | (k1 << 32), offset = c0 | (c1 << 32), subseq = c2 | (c3 << 32);
    at::Philox4_32 eng(seed, subseq, offset);
    uint32_t a = eng(), b = eng(), c = eng(), d = eng();
    printf("%u %u %u %u\n", a, b, c, d);
  }
}
"""

_ROCRAND_PIN = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
// Reach rocRAND's ten-round block function through a derived class.
struct Block : rocrand_device::philox4x32_10_engine {
  uint4 raw(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};
int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  Block b;
  while (scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 c; c.x = (unsigned)c0; c.y = (unsigned)c1; c.z = (unsigned)c2; c.w = (unsigned)c3;
    uint2 k; k.x = (unsigned)k0; k.y = (unsigned)k1;
    uint4 o = b.raw(c, k);
    printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
  }
}
"""


def _run_pin(exe, rows):
    inp = "".join(" ".join(str(int(v)) for v in r) + "\n" for r in rows)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [[int(v) for v in line.split()] for line in out.strip().splitlines()]


@pytest.fixture(scope="session")
def torch_philox():
    """Philox4x32-10 from torch's ATen header, used as an independent black box.

    torch's engine maps (seed, subsequence, offset) to key = seed,
    counter = (offset_lo, offset_hi, subseq_lo, subseq_hi).
    """
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    exe = _compile_pin("pin_torch_philox", _TORCH_PIN, ["-I" + inc])
    return lambda rows: _run_pin(exe, rows)


@pytest.fixture(scope="session")
def rocrand_philox():
    """Philox4x32-10 from rocRAND's header (host build), an independent black box.

    Its ten-round block function is called directly on (counter, key).
    """
    if not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers not present")
    exe = _compile_pin("pin_rocrand_philox", _ROCRAND_PIN,
                       ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"])
    return lambda rows: _run_pin(exe, rows)


def rng_rows(n, seed=1234):
    r = np.random.default_rng(seed)
    return [[int(v) for v in r.integers(0, 2**32, size=6, dtype=np.uint64)] for _ in range(n)]
