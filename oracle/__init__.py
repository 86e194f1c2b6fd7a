"""Oracle: plain, slow CPU reference for the Gaussian-process likelihood engine.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package; only the tests, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the HIP library.

Modules
-------
kernels   covariance kernels K(x, y; theta) and their parameter derivatives
          (Matern nu = 1/2, 3/2, 5/2 closed forms and rational quadratic).
dense     the plain definitions: log-likelihood, log-determinant, solve and the
          score equations by dense FP64 Cholesky (eq. loglikelihood and
          eq. gradient of the paper).
rsf       the recursive skeletonization factorization written out step by step
          in the paper's order (Section 2): quadtree, modified proxy trick,
          interpolative decomposition by column-pivoted QR, block elimination,
          root Cholesky, sweeps, log-determinant, and the multiply-only form of
          the derivative operator.
peel      matrix peeling for weakly admissible matrices (Section 3.2) and the
          trace extraction at the leaves.
peel_strong  matrix peeling in the strongly admissible format (the form the
          remark after Theorem 2 points to): interaction blocks of separated
          boxes, coloured probes, near field never compressed.
philox    the Philox4x32-10 counter-based generator (Salmon et al., SC'11) and
          the Box-Muller transform, used to draw the Gaussian peeling probes.
"""
