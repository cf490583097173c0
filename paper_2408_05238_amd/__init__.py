"""skf: skew-symmetric LTL^T factorization and Pfaffians on AMD MI355X (gfx950).

The compute path is the HIP library ``libskf.so`` (C ABI in ``include/skf.h``);
``skf`` is its thin ctypes binding and ``inputs`` the seeded input generator.
Importing the package does not load the GPU library.
"""
__all__ = ["skf", "inputs", "build"]
