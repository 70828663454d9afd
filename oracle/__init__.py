"""CPU oracle for the layered-stencil thermal solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call, link or execute anything in this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark use it.

The oracle computes what the method must reach, from plain definitions:

* ``assembly``  - the finite-volume system of the paper's steady-state and
  backward-Euler equations (Section 3.2), assembled in FP64 CSR;
* ``direct``    - dense Cholesky, sparse LU and an exact separable (DCT x
  tridiagonal) solver for per-layer-uniform stacks, plus exact extreme
  eigenvalues;
* ``krylov``    - the paper's Chebyshev polynomial preconditioner (Section 4.3),
  its closed-form residual polynomial, Lanczos spectral estimation and the
  preconditioned CG of Algorithm 1, all in FP64 numpy;
* ``cpu_cg``    - a plain FP64 Jacobi-preconditioned CG in C with OpenMP, for
  large grids and as the timed CPU baseline;
* ``adjoint``   - the gradient of a scalar loss with respect to power and layer
  conductivities through one adjoint solve.

It shares no code, header, table or helper with the GPU path; inputs come from
the separate ``workloads`` package, which holds no solver arithmetic.
"""
