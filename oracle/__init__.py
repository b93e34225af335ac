"""Plain CPU FP64 oracle for the space-time multigrid method of Gander and
Neumueller (arXiv 1411.0519): DG-in-time / Q1-finite-elements-in-space heat
equation, damped block-Jacobi smoother, time semi-coarsening or full
space-time coarsening chosen by the mu >= mu* criterion.

TEST INFRASTRUCTURE ONLY.  This package is slow, obviously-correct reference
code.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path (the HIP library and its Python
binding) never does, and this package imports nothing from the product.

Modules
  dg_time    time matrices K_tau, M_tau, N_tau and the time transfers (Sec. 1, Sec. 3.2)
  fe_space   Q1 mass/stiffness matrices by element assembly (Sec. 1, Sec. 3)
  spacetime  block system L u = f and its right-hand side (Sec. 1)
  multigrid  hierarchy, coarsening rule, smoother, V-cycle, solve, adjoint (Sec. 2, Sec. 4)
  lfa        local Fourier analysis: symbols, smoothing and two-grid factors (Sec. 3)
  spatial_mg one spatial multigrid cycle per slab, the inexact smoother (Remark V-cycleApproxSpace)
  mesh       red refinement of triangles/tetrahedra, P1 matrices, nested interpolation (Sec. 4 examples)
  p1         the space-time hierarchy on P1 meshes (Sec. 4 examples)

Every function is pinned by a CPU test against something other than itself
(values printed in the paper, closed forms, textbook special cases, brute
force); no function here is "parity unpinned".
"""
