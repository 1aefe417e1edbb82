"""Krylov acceleration of the stationary iteration (test infrastructure: plain
FP64 NumPy).

The stationary sweep is affine, Phi(U) = T U + c on the interior nodes, so its
fixed point solves the linear system (I - T) U = c, and the iteration's
residual rel = |Phi(U) - U| / |Phi(0)| is that system's relative residual
|c - (I - T) U| / |c|.  GMRES(m) (Saad and Schultz, 1986) minimises this
residual over a Krylov space built from applications of I - T, i.e. of one
sweep each, and restarts every m applications:
  r = c - A x;  beta = |r|;  v_1 = r / beta;
  Arnoldi, for j = 1..m:  w = A v_j;  h_{ij} = (w, v_i), w -= h_{ij} v_i for
      i = 1..j (modified Gram-Schmidt);  h_{j+1,j} = |w|;  v_{j+1} = w / h_{j+1,j};
  the small least-squares problem min |beta e_1 - H y| is kept triangular by
  Givens rotations, whose last entry is the residual norm;
  x += V y;  repeat until the residual reaches tol |c|.
The method and its tolerance do not change the fixed point; this module
computes it by a route independent of the plain iteration and of the dense
solve (oracle.dense), against which it is pinned.
"""
from __future__ import annotations

import numpy as np


def gmres(apply_A, b, x0, tol, restart, max_apply):
    """GMRES(restart) on A x = b from x0 until |b - A x| <= tol |b|.

    Returns (x, applications of A, relative residual history after each
    application)."""
    x = np.array(x0, float, copy=True)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), 0, [0.0]
    n_apply = 0
    hist = []
    while True:
        r = b - apply_A(x)
        n_apply += 1
        beta = np.linalg.norm(r)
        hist.append(beta / bn)
        if beta <= tol * bn or n_apply >= max_apply:
            return x, n_apply, hist
        m = restart
        V = np.zeros((m + 1, len(b)))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = apply_A(V[j])
            n_apply += 1
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):  # earlier rotations on the new column
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            hist.append(abs(g[j + 1]) / bn)
            if abs(g[j + 1]) <= tol * bn or n_apply >= max_apply:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):  # back substitution on the triangular H
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + V[:k].T @ y


def solve_fixed_point(orc, theta, dt, tol, restart=20, max_apply=2000, U0=None):
    """The stationary fixed point by GMRES(restart) on (I - T) U = c, T applied
    as Phi(z + v) - Phi(z) with z the field that is zero inside (g outside).
    Returns (U grid field, sweeps, residual history)."""
    ii = orc.inner_idx
    z = orc.zero_field()
    phi_z = orc.step(z, theta, dt)

    def apply_A(v):  # (I - T) v
        e = z.copy()
        e[ii] = v
        return v - (orc.step(e, theta, dt)[ii] - phi_z[ii])

    c = phi_z[ii]
    x0 = np.zeros(len(ii)) if U0 is None else orc.with_boundary(U0)[ii]
    x, n, hist = gmres(apply_A, c, x0, tol, restart, max_apply)
    U = z.copy()
    U[ii] = x
    return U, n, hist
