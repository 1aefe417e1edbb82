"""Own 2D P1 Galerkin solution of eq. (5)-(6) (an independent reference).

Test infrastructure: plain FP64 NumPy/SciPy.  The grid's cells are split into
two right triangles along the (i,j)-(i+1,j+1) diagonal; a(u,v) of eq. (6) is
assembled exactly for P1 functions with P1-interpolated beta (advection
integrated with the element-mean velocity is exact for P1 beta times constant
gradient times a P1 test function: int_T beta_q phi_q * phi_i = |T|(1+delta_qi)/12
summed), and the load uses the P1 interpolant of f.  Box domains only.

The paper compares its method with FEniCS P1 on 450 triangles (Sec. 7) and
reports 5 % (max norm) and 2 % (L1) relative differences.  FEniCS is not
available here; this assembly stands in for it.  compare_data2d is
"parity unpinned": the paper's mesh orientation and curve density are not
given, so only the order of magnitude of that comparison can be checked.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def solve(prob, transient=None):
    """Stationary P1 solution on the box grid of prob; returns a grid field."""
    nx, ny = prob.nx, prob.ny
    a, b, c, d = prob.box
    hx = (b - a) / (nx - 1)
    hy = (d - c) / (ny - 1)
    X = a + hx * np.arange(nx)
    Y = c + hy * np.arange(ny)
    idx = lambda i, j: j * nx + i  # noqa: E731
    tris = []
    for j in range(ny - 1):
        for i in range(nx - 1):
            tris.append((idx(i, j), idx(i + 1, j), idx(i + 1, j + 1)))
            tris.append((idx(i, j), idx(i + 1, j + 1), idx(i, j + 1)))
    tris = np.array(tris)
    px = np.tile(X, ny)
    py = np.repeat(Y, nx)
    B1 = prob.beta1.ravel()
    B2 = prob.beta2.ravel()
    F = prob.f.ravel()
    rows, cols, vals = [], [], []
    rhs = np.zeros(nx * ny)
    mu, sigma = prob.mu, prob.sigma
    for t in tris:
        xs, ys = px[t], py[t]
        Dm = np.array([[xs[1] - xs[0], xs[2] - xs[0]], [ys[1] - ys[0], ys[2] - ys[0]]])
        area = 0.5 * abs(np.linalg.det(Dm))
        # gradients of the barycentric basis
        Ginv = np.linalg.inv(Dm)
        grads = np.array([-Ginv[0] - Ginv[1], Ginv[0], Ginv[1]])  # (3, 2)
        mass = area / 12.0 * (np.ones((3, 3)) + np.eye(3))
        stiff = area * grads @ grads.T
        # int (beta . grad phi_j) phi_i, beta P1: sum_q beta_q int phi_q phi_i
        bq = np.stack([B1[t], B2[t]], 1)  # (3, 2)
        w = mass @ bq  # w[i] = int beta phi_i (vector)
        adv = w @ grads.T  # adv[i, j] = (int beta phi_i) . grad phi_j
        Ae = mu * stiff + adv + sigma * mass
        for ii in range(3):
            for jj in range(3):
                rows.append(t[ii]); cols.append(t[jj]); vals.append(Ae[ii, jj])
        rhs[t] += mass @ F[t]
    A = sp.csr_matrix((vals, (rows, cols)), shape=(nx * ny, nx * ny))
    inner = np.zeros((ny, nx), bool)
    inner[1:-1, 1:-1] = True
    ii = np.nonzero(inner.ravel())[0]
    Ai = A[ii][:, ii].tocsc()
    u = np.zeros(nx * ny)
    u[ii] = spla.spsolve(Ai, rhs[ii])
    return u


def compare_data2d(U_method, U_p1, mask):
    """Relative differences (max norm, L1) over interior nodes: parity unpinned."""
    d = (U_method - U_p1)[mask.ravel()]
    r = U_p1[mask.ravel()]
    return float(np.abs(d).max() / np.abs(r).max()), float(np.abs(d).sum() / np.abs(r).sum())
