"""CPU oracle: plain, slow FP64 NumPy implementation of the P-multigrid FR/CPR stage solve.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this package; only
the tests, the smoke entry point and the benchmark's CPU baseline may use it.
It shares no code with the HIP library: the two sides meet only through the
seeded inputs of ``workloads``.

Every function follows a passage of Wang & Yu, "An implicit P-multigrid flux
reconstruction method for simulation of locally preconditioned unsteady
Navier-Stokes equations at low Mach numbers" (arXiv 1908.03972), cited by
section and equation number. Where the paper is silent the module says which
reading it takes.

Array conventions (oracle only): states are ``[Ne, Np, Nv]`` with the solution
point index ``p = i + (P+1)*j`` (xi index fastest) and variables last. Element
blocks are ``[Ne, n, n]`` with row/column index ``p*Nv + v``.

Modules
-------
basis     1-D Gauss points, Lagrange operators, Radau correction derivatives, transfers
gas       ideal-gas relations, M, Gamma, fluxes, eigenvalues, common flux (Sec. 2.1-2.3)
geometry  element mappings and metrics at solution and flux points
fr        FR/CPR residual R(q) and the stage residual F(q) (Sec. 2.3-2.4)
jacobian  element-diagonal blocks D of A (Sec. 2.4, eqs. (28)-(30)) by complex step
solver    element-Jacobi smoother, transfers, V-cycle, pseudo-time control, ESDIRK
"""
