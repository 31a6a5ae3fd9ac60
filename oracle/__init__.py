"""Plain FP64 CPU oracle for the lattice core-Hamiltonian eigenproblem.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP library; the only
thing both sides read is the seeded instance description from ``synth``.

Modules
  model      grids, nodal Gaussian factors, 1D FEM matrices, sinc rule,
             potential collocation factors and lattice windows
  dense3d    the plain definition: full N x N Galerkin matrices H and S by
             direct quadrature on the 3D grid, dense generalized eigensolve
  separable  the paper's route: 1D Gram matrices, Hadamard combination into
             the generator blocks, Fourier blocks, per-block eigensolves
  toeplitz   dense block-Toeplitz operators and their circulant embedding
  toeplitz3  three-level block-Toeplitz operator of a lattice in a box
             (replicated central cell) and its three-level circulant embedding
  boxchain   the exact box case (B) of a Dirichlet chain: finite-lattice
             potential (eq. EwaldSumE), every block of the band computed
  backtransform  eigenvectors of the full lattice problem from the
             Fourier-block eigenvectors, U = (F^* x I) bdiag(Ubar_j)

Every floating-point step is float64.  Readings of passages where the paper
is silent or ambiguous are listed at the top of each module.
"""
