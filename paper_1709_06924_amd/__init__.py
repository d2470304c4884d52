"""MI355X-native hot path of Lloyd-preconditioned LBFGS for spherical CVTs.

The work runs in the HIP library `libscvt.so` (built from csrc/); this package
holds its thin ctypes binding (`scvt`) and the seeded workload generators
(`inputs`).  Importing the package loads nothing; `paper_1709_06924_amd.scvt`
loads the library and raises if it is missing.
"""
__all__ = ["inputs", "scvt"]
