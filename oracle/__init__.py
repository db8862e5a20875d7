"""CPU float64 oracle for the low-rank Poisson solve -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the package smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU solver never calls it, links it or
falls back to it, and this package never imports the GPU solver: the two share
no code.  Inputs come from the seeded generators in
``paper_1306_2150_amd.inputs`` (random draws only), which the tests pass in.

Contents
--------
``poisson``  plain definitions: grid, 1D operator, its eigenvalues, the
             orthonormal sine transform, and the full-grid direct solvers
             (2D and 3D) of Section 4.1 (the "textbook" diagonalisation).
``lowrank``  the paper's low-rank 2D method written step by step in its
             order (transform of the factors, cross approximation of the
             divided spectrum with maxvol pivots, rounding, back transform),
             Sections 3 and 4.2, with the readings stated in each docstring.
``tucker``   the 3D Tucker variant (the paper only promises it; the reading
             is stated there).
``metrics``  blockwise relative Frobenius error of a factored result.
``expsum``   the exponential-sum comparator of Section 4.1 (sinc quadrature
             of 1/x, Hadamard product with the transformed right-hand side,
             rounding).
``stokes``   the discrete 2D Stokes problem of Section 2 (gradients from the
             shift matrices, the consistent Laplacian, the Schur complement)
             and its full-format Uzawa solve; the test problem of Section 6.

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
library routines or brute force; see each function's docstring for its pin.
"""
from . import poisson, lowrank, metrics, tucker, expsum, stokes  # noqa: F401
