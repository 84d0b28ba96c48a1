"""CPU oracle for the Bidomain AMG-PCG solve path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, double-precision reference written from the paper's statement of the
method (Centofanti & Scacchi, "A comparison of Algebraic Multigrid Bidomain solvers on
hybrid CPU-GPU architectures"): Q1 assembly (Sec. 2.2), the smoothed-aggregation and
classical setups (Alg. 1, Sec. 4), the V-cycle (Alg. 2), PCG (Sec. 2.2) and the
decoupled IMEX step (eqs. (4)-(7)).

Only the test suite, the smoke entry point and the CPU-baseline leg of the benchmark may
import this package. The HIP library never links, imports or calls it, and the two share
no code; the oracle uses numpy/scipy as library primitives (sparse products, dense
eigen/Cholesky solves) and nothing else.

Modules:
  fem       -- mesh, fibers, conductivity tensors, Q1 stiffness and lumped mass
  amg       -- strength, MIS, aggregation, prolongators, Galerkin products, eigen estimate
  krylov    -- Chebyshev/Jacobi smoothers, V-cycle, coarse solve, PCG, FCG, exact dot
  bidomain  -- Aliev-Panfilov membrane update and the IMEX Bidomain step
"""
