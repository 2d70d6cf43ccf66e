"""CPU FP64 oracle for the preconditioned Krylov solve of the semi-implicit
Cahn-Hilliard / Allen-Cahn / Navier-Stokes time step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the tests, the package's smoke check
and the benchmark's CPU-baseline leg use it.  It shares no code with the HIP
path; the one common dependency is the seeded input generator module, which
holds none of the method's arithmetic.

What it computes (each module cites the passage it follows):

* ``fem``        exact-quadrature P1 and Taylor-Hood P2-P1 assembly on the
                 periodic right-diagonal triangulation, COO -> CSR with explicit
                 zeros kept.
* ``potential``  the double-well / mixing potential and the fitted quartic
                 potential, with their derivatives.
* ``systems``    the Cahn-Hilliard 2x2 block, the Allen-Cahn matrix and the
                 Oseen saddle point with their right-hand sides.
* ``solvers``    dense LU, SuperLU, and per-Fourier-mode solves for the
                 convection-free periodic systems.
* ``step``       one semi-implicit time step (binary CH, CH + AC, ternary
                 CH + AC + Oseen) by direct solves, plus diagnostics.
* ``multigrid``  the geometric V-cycle used inside the block preconditioners,
                 written out plainly as a reference for the GPU cycle.
* ``precond``    the block preconditioners (matching Schur approximation,
                 pressure convection-diffusion) applied with exact or
                 multigrid inner solves.
"""
