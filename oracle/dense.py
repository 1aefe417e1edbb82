"""Brute-force references for the method's own discrete problem.

Test infrastructure: plain FP64 NumPy.

The step Phi of eq. (10) (value transfer) is affine on the interior nodes:
Phi(U) = T U + c.  Its matrix is assembled column by column (Phi applied to
unit vectors, minus c) and the fixed point is obtained by a dense LU solve of
(I - T) U = c.  Only for small grids (N interior nodes <= ~4k).
"""
from __future__ import annotations

import numpy as np


def affine_map(orc, theta, dt):
    ii = orc.inner_idx
    N = len(ii)
    c = orc.step(orc.zero_field(), theta, dt)[ii]
    T = np.zeros((N, N))
    for col in range(N):
        e = orc.zero_field()
        e[ii[col]] = 1.0
        T[:, col] = orc.step(e, theta, dt)[ii] - c
    return T, c


def fixed_point(orc, theta, dt):
    """Dense LU solution of (I - T) U = c, embedded in a grid field."""
    T, c = affine_map(orc, theta, dt)
    u = np.linalg.solve(np.eye(len(c)) - T, c)
    U = orc.zero_field()
    U[orc.inner_idx] = u
    return U


def spectral_radius(orc, theta, dt):
    T, _ = affine_map(orc, theta, dt)
    return float(np.max(np.abs(np.linalg.eigvals(T))))
