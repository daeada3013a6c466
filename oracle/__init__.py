"""CPU float64 oracle for Golub-Kahan partial SVD and numerical rank.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import anything from this package; the product path (the
HIP library and its Python binding) never does, and this package imports
nothing from the product path either. The two share no code: the only common
ingredient is the seeded input generator, which holds none of the method's
arithmetic.

Arithmetic is plain numpy in float64. Library primitives used as single steps:
matrix-vector / matrix-matrix products, ``numpy.linalg.svd`` for the small
projected matrix, ``numpy.linalg.qr`` and ``numpy.linalg.eigh``. There is no
blocking, fusion or reordering beyond what the paper's algorithms state.

Modules
-------
gk        Golub-Kahan bidiagonalization (Bidiag 1, eq. 2.1-2.4), full
          reorthogonalization, Ritz extraction (eq. 2.13 and the left-vector
          formula after it), thick restart, convergence test, Algorithms 1-3.
rank      numerical rank: singular-value count and an independent Sylvester
          inertia (Sturm) count on the Golub-Kahan tridiagonal.
jacobi    brute-force one-sided Jacobi SVD used to pin the rest on tiny inputs.
checks    invariants of eq. 2.4 / orthonormality, triplet residuals, the error
          metrics of the experiments section and the sign-invariant triplet
          alignment metric of Figure 1.
bf16      round-to-nearest-even bfloat16 storage and the Rayleigh-Ritz
          refinement of eq. (5) on the float32 matrix.
mlp       the start-vector network (forward, backward, Adam) in float64.
philox    Philox4x32-10 counter-based generator and the Gaussian start vector
          drawn from it (for the device-generated start path).
"""
