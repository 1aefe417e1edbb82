"""P1 finite elements on the polylines and tridiagonal solves (eq. (16)-(19)).

Test infrastructure: plain FP64 NumPy/SciPy.

A line has nodes z_0..z_n; z_0 and z_n lie on Gamma and carry Dirichlet values.
Element e_k = [z_{k-1}, z_k] has length h_k = |z_k - z_{k-1}| (chords: the
elements are straight).  With hat functions phi_k:

  mass       (u, v) on the line                   eq. (16)/(18) first term
             row k: [h_k/6, (h_k + h_{k+1})/3, h_{k+1}/6]
  stiffness  int u' v' dl                          eq. (17), (19)
             row k: [-1/h_k, 1/h_k + 1/h_{k+1}, -1/h_{k+1}]
  advection  int |beta| u' v dl, |beta| taken as the P1 interpolant of its nodal
             values w_k and integrated exactly                    eq. (17)
             row k: [-(w_{k-1} + 2 w_k)/6, (w_{k-1} - w_{k+1})/6, (2 w_k + w_{k+1})/6]
  load       int f v dl, f taken as its P1 interpolant: L = M f   eq. (17)

s_i = mu K + C + sigma M on beta-lines (eq. (17)); m_i = mu K on gamma-lines (eq. (19)).

Stabilised beta-lines (exponential fitting, Il'in / Allen-Southwell; the
paper's first item of further work, singularly perturbed lines): on element
e the diffusion mu becomes mu phi(Pe_e), phi(Pe) = Pe coth(Pe), with the
element Peclet number Pe_e = |beta|_e h_e / (2 mu) and |beta|_e the mean of
the element's two nodal values.  phi -> 1 as Pe -> 0 (plain Galerkin) and
phi ~ Pe for large Pe (the upwind diffusion |beta| h / 2).  For constant
|beta| on a uniform line, -mu u'' + |beta| u' = 0 is then solved exactly at
the nodes.
The flow runs from z_0 to z_n (the tracing direction), which fixes the sign of C.

All arrays here are "full-node" arrays over the concatenated nodes of every line
of a family; the rows of the two end nodes of each line are not equations.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded


def chords(fam):
    """h[k] = |z_k - z_{k-1}| for every node that has a predecessor on its line, else 0."""
    h = np.zeros(fam.n_nodes)
    d = np.hypot(np.diff(fam.x), np.diff(fam.y))
    h[1:] = d
    h[fam.offsets[:-1]] = 0.0
    return h


class Tri:
    """Tridiagonal operator on full-node arrays; rows of end nodes are zero."""

    def __init__(self, lo, di, up):
        self.lo, self.di, self.up = lo, di, up

    def __add__(self, o):
        return Tri(self.lo + o.lo, self.di + o.di, self.up + o.up)

    def scale(self, s):
        return Tri(s * self.lo, s * self.di, s * self.up)

    def apply(self, u):
        """(A u)_k for interior rows; u includes the end values."""
        r = self.di * u
        r[1:] += self.lo[1:] * u[:-1]
        r[:-1] += self.up[:-1] * u[1:]
        return r


def line_operators(fam, wnode):
    """Mass M, stiffness K and advection C of every line of a family.

    wnode: nodal |beta| for the advection (ignored if None; C is then zero).
    """
    n = fam.n_nodes
    inner = fam.interior()
    h = chords(fam)
    hk = np.zeros(n)      # h_k (element to the left of node k)
    hk1 = np.zeros(n)     # h_{k+1} (element to the right)
    hk[inner] = h[inner]
    hk1[:-1][inner[:-1]] = h[1:][inner[:-1]]
    z = np.zeros(n)
    Mlo, Mdi, Mup = z.copy(), z.copy(), z.copy()
    Klo, Kdi, Kup = z.copy(), z.copy(), z.copy()
    Mlo[inner] = hk[inner] / 6.0
    Mdi[inner] = (hk[inner] + hk1[inner]) / 3.0
    Mup[inner] = hk1[inner] / 6.0
    Klo[inner] = -1.0 / hk[inner]
    Kdi[inner] = 1.0 / hk[inner] + 1.0 / hk1[inner]
    Kup[inner] = -1.0 / hk1[inner]
    M = Tri(Mlo, Mdi, Mup)
    K = Tri(Klo, Kdi, Kup)
    Clo, Cdi, Cup = z.copy(), z.copy(), z.copy()
    if wnode is not None:
        idx = np.nonzero(inner)[0]
        wm, w0, wp = wnode[idx - 1], wnode[idx], wnode[idx + 1]
        Clo[idx] = -(wm + 2.0 * w0) / 6.0
        Cdi[idx] = (wm - wp) / 6.0
        Cup[idx] = (2.0 * w0 + wp) / 6.0
    C = Tri(Clo, Cdi, Cup)
    return M, K, C


def solve_lines(A, rhs, inner, end_values=None):
    """Solve A u = rhs on the interior nodes of every line, u = end_values at the ends.

    The lines are decoupled: end rows are identity rows, so a banded LU over the
    concatenation is the set of independent per-line solves.
    """
    n = len(rhs)
    di = np.where(inner, A.di, 1.0)
    lo = np.where(inner, A.lo, 0.0)
    up = np.where(inner, A.up, 0.0)
    b = np.where(inner, rhs, 0.0 if end_values is None else end_values)
    ab = np.zeros((3, n))
    ab[0, 1:] = up[:-1]
    ab[1] = di
    ab[2, :-1] = lo[1:]
    u = solve_banded((1, 1), ab, b, check_finite=False)
    u[~inner] = b[~inner]  # the identity rows are exact
    return u


def thomas(lo, di, up, rhs):
    """Thomas algorithm for one tridiagonal system (no pivoting).

    Row k: lo[k] x[k-1] + di[k] x[k] + up[k] x[k+1] = rhs[k]; lo[0], up[-1] unused.
    """
    n = len(di)
    cp = np.zeros(n)
    dp = np.zeros(n)
    cp[0] = up[0] / di[0]
    dp[0] = rhs[0] / di[0]
    for k in range(1, n):
        den = di[k] - lo[k] * cp[k - 1]
        cp[k] = up[k] / den if k < n - 1 else 0.0
        dp[k] = (rhs[k] - lo[k] * dp[k - 1]) / den
    x = np.zeros(n)
    x[-1] = dp[-1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def fitted_stiffness(fam, wnode, mu):
    """Stiffness of the exponentially fitted beta-lines: element e scaled by
    phi(Pe_e) = Pe_e coth(Pe_e), Pe_e = |beta|_e h_e / (2 mu)."""
    n = fam.n_nodes
    inner = fam.interior()
    h = chords(fam)
    # per node k: phi of the element to its left, [z_{k-1}, z_k] (0 at line starts)
    wl = np.zeros(n)
    wl[1:] = 0.5 * (wnode[1:] + wnode[:-1])
    pe = np.where(h > 0, wl * h / (2.0 * mu), 1.0)
    phi = np.where(h > 0, pe / np.tanh(pe), 0.0)
    z = np.zeros(n)
    lo, di, up = z.copy(), z.copy(), z.copy()
    idx = np.nonzero(inner)[0]
    lo[idx] = -phi[idx] / h[idx]
    up[idx] = -phi[idx + 1] / h[idx + 1]
    di[idx] = -lo[idx] - up[idx]
    return Tri(lo, di, up)
