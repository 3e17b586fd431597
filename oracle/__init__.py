"""CPU oracle for the zero-temperature checkerboard quench (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The product library never imports, links or calls it.
"""
from .oracle import *  # noqa: F401,F403
