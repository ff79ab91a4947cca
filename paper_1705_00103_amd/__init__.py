"""MI355X-native Chebyshev-Jacobi Poisson solver.

The solver lives in the C-ABI library libcj.so (HIP kernels for gfx950); its
Python binding is ``paper_1705_00103_amd.cj``.  Importing this package loads
nothing; ``cj`` loads the library on first use and raises if it is missing.
"""
