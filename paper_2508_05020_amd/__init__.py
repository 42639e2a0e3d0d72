"""MI355X-native AMR compressible-Euler hot path (WENO5-JS + Rusanov + SSP-RK3).

The compute path lives in the HIP library ``libamr.so`` built from ``csrc/``;
``paper_2508_05020_amd.amr`` is a thin ctypes binding over its C ABI
(``include/amr.h``).  Importing this package does not load the library; only
``paper_2508_05020_amd.amr`` does, and it fails loudly when the library is
missing.
"""
__all__ = ["workloads"]
