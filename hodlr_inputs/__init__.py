"""Seeded synthetic inputs for the HODLR matrix-vector product.

This package is shared by the oracle's tests and by the HIP library's
callers (tests, bench).  It generates inputs only -- point sets, kernel
matrix entries, right-hand sides and the compressed (eps-HODLR) operator
that the library's ``hodlr_create`` consumes -- and holds none of the
arithmetic of the product path: no tree construction (the caller passes the
partition in), no precision assignment, no rounding to storage formats and
no matrix-vector product.

* ``points``   -- point sets (sorted 1D, Morton-ordered 2D, clustered 1D,
                  uniform grids).
* ``kernels``  -- kernel functions and dense evaluation of A[I, J].
* ``compress`` -- truncated-SVD compression of every off-diagonal block of
                  a kernel matrix over a given partition (dense SVD for
                  small blocks, randomised range finder with an exact
                  residual certificate for large ones).
* ``configs``  -- the named workloads (sizes, kernels, eps, formats, X).
"""
