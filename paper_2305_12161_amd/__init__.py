"""Zero-temperature checkerboard quench of the d=3 Ising model on MI355X.

The compute path is the HIP library ``libquench.so`` (C ABI, ``include/quench.h``);
``paper_2305_12161_amd.binding`` is its thin ctypes binding.  Importing this
package does not load the library; ``binding`` raises if it is missing.
"""
__all__ = ["binding", "workloads"]
