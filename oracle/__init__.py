"""CPU oracle for the Chebyshev-Jacobi method (CJM) on the 2D Poisson problem.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import anything here; the GPU library and its Python
binding never do, and the oracle never imports them.  Everything is plain FP64:

  cjm.py        the method as the paper states it (kappa bounds, Chebyshev
                weights, their ordering, the cycle loop and the stopping rule),
                driving the O(N^2) loops of cj_oracle.c;
  dense.py      plain definitions used to pin cjm.py: A = -Delta_h assembled
                from Kronecker products, the fast-sine-transform direct solve,
                the stencil symbol and the Chebyshev polynomial T_M;
  cj_oracle.c   the stencil, one weighted Jacobi sweep and the residual norm.
"""
