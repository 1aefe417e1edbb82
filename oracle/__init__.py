"""Plain FP64 CPU oracle of the directional diffusion splitting method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library; its inputs come
from the seeded generators in ``workloads`` and nothing else.

Paper: R. Drebotiy, H. Shynkarenko, "Directional diffusion splitting method
for advection-diffusion-reaction model" (arXiv 2411.11041).

Modules
  geometry   Sec. 3 fields b, p; eq. (12) inflow sets; eq. (13)-(14) curve families
  linefe     eq. (16)-(19): P1 line elements and tridiagonal solves
  transfer   Sec. 6 grid interpolation: scatter (crossing records) and eq. (21)-(23) gather
  method     one step Phi of eq. (10) (beta and gamma substeps, values handed on
             through the grid), the stationary fixed-point iteration and its
             relative update, eq. (11) initial guess, theta-scheme time marching
  dense      the affine map Phi(U) = T U + c assembled column by column, and the
             dense LU solve of (I - T) U = c (the iteration's limit)
  krylov     restarted GMRES(m) on (I - T) U = c: the same fixed point by a Krylov route
  direct     the interpolation-free transfer (Sec. 8): values handed from one curve
             family to the other at the intersections of their segments, and the
             stationary iteration on the gamma-curve values with it
  coarse     full-weighting restriction and bilinear interpolation between the
             solver grid and the warm-start network's coarse grid
  galerkin2d own 2D P1 Galerkin solve of eq. (5)-(6) (independent reference)
  cnn        FP64 conv-net forward/backward for the learned warm start

Functions whose result has no independent pin are marked "parity unpinned"
in their docstring (only galerkin2d.compare_data2d).
"""
