"""Plain FP64 CPU oracle of the multigrid implicit UGKS (MIUGKS).

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
CPU-baseline leg of the benchmark may import this package.  The GPU library
never calls it and shares none of its code: the two meet only in the seeded
input recipes of ``workloads``.

Every routine is written from the paper (Zhu, Zhong & Xu, "Unified
gas-kinetic scheme with multigrid convergence for rarefied flow study",
arXiv:1704.03151) and cites the section or equation it follows.  Where the
paper is silent or garbled the oracle takes one stated reading; the readings
are listed in the design notes of the repository.  All arithmetic is float64
and vectorised with numpy over velocities and over the cells of one colour,
in the same red-black order the GPU path uses.

Modules
  quadrature  discrete velocity grids and weights
  gas         equilibrium states, moments, viscosity law
  mesh        structured levels, face tables, transfer operators
  flux        explicit UGKS interface flux and residuals (Step 1)
  fas         FAS V-cycle of the macroscopic prediction (Step 2)
  cs          CS V-cycle of the microscopic correction (Step 5)
  solver      the outer iteration, Steps 1-8
  sparse      direct assembly of the correction matrix (pins the CS cycle)
"""
