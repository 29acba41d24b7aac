"""MI355X-native line-of-sight projection library (gfx950 HIP kernels behind a C ABI).

Importing the package loads nothing; ``paper_2509_25110_amd.los`` binds the
compiled ``liblos.so`` and raises if it is missing.
"""
__all__ = ["inputs"]
