"""FP64 CPU oracle for the ISDF-xTC hot path.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously-correct
NumPy/SciPy implementation of what the GPU library computes, written from the
paper (arXiv 2607.17314) and used to check it. Only the test-suite, the
package's smoke check and the benchmark's CPU-baseline leg may import it; the
product path never routes through it. It shares no code with the HIP library:
the only common dependency is the seeded workload generator (``workloads``),
which holds none of the method's arithmetic.

Modules, each citing the passage it follows:
  orbitals    orbital values and gradients on the grid (Alg. 2, grid step)
  pivots      weight-scaled fixed-rank pivoted Cholesky, both channels, and
              pivot fusion (ISDF section, Alg. 1; matrix-free pivot search)
  fit         ISDF least-squares fit of xi and xi~ with Tikhonov retry
              (ISDF section, auxiliary basis fitting; auxiliary-fit robustness)
  correlator  scaled-distance correlators and their analytic derivatives
              (Jastrow correlator section, eqs. bh-scaled and bh-u)
  contract    the grid-pair kernels u^(1), u^(3), the Laplacian kernel, the
              xTC D^(1), D^(4) terms, the field A_gamma and energy-scale sums
              (K-kernel section, eqs. K1-isdf and K3-isdf; xTC section,
              eqs. deltaU-fields, deltaU-isdf-map, Terms 1 and 4)
  adjoint     derivatives of those outputs with respect to the linear
              correlator coefficients
  mlp         the learned interpolation-point scorer (not in the paper)
  fourindex   four-index brute force of K^(1), K^(3) and Terms 1, 4 on tiny
              inputs (eqs. K1-isdf, K3-isdf, deltaU-preisdf)

Parity status of every function is stated in its docstring; all functions are
pinned by the tests in tests/test_oracle_*.py.
"""
