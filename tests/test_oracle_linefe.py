"""Pins of the oracle's 1D line elements (eq. (16)-(19)) and tridiagonal solves.

Each check compares the oracle with a closed form or an independent
computation, never with a retyped copy of its own formula.
"""
import math

import numpy as np
import pytest
from scipy.linalg import solve_banded

from oracle import geometry as geo
from oracle import linefe as lfe
import workloads as W


def straight_family(ls_list, direction=(0.6, 0.8), origin=(0.1, 0.2)):
    """Lines along a fixed direction with the given arc-length node positions."""
    xs, ys, offs = [], [], [0]
    for ls in ls_list:
        xs.append(origin[0] + direction[0] * ls)
        ys.append(origin[1] + direction[1] * ls)
        offs.append(offs[-1] + len(ls))
    return geo.Family(np.array(offs), np.concatenate(xs), np.concatenate(ys), 0)


def test_pure_diffusion_nodal_exactness():
    """-mu u'' = f with f linear: P1 nodal values are exact on any mesh (textbook
    superconvergence of 1D linear elements for the Laplacian with exact load)."""
    rng = np.random.default_rng(0)
    mu = 0.37
    a0, a1 = 1.3, -2.1            # f(l) = a0 + a1 l
    uL, uR = 0.4, -0.7            # Dirichlet values at l=0 and l=1
    ls = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, 40)]))
    fam = straight_family([ls])
    M, K, _ = lfe.line_operators(fam, None)

    def exact(l):
        # -mu u'' = a0 + a1 l  ->  u = -(a0 l^2/2 + a1 l^3/6)/mu + c1 l + c0
        p = lambda s: -(a0 * s ** 2 / 2 + a1 * s ** 3 / 6) / mu  # noqa: E731
        c0 = uL
        c1 = uR - c0 - p(1.0)
        return p(l) + c1 * l + c0

    f = a0 + a1 * ls
    rhs = M.apply(f)
    ends = np.zeros(len(ls)); ends[0] = uL; ends[-1] = uR
    u = lfe.solve_lines(K.scale(mu), rhs, fam.interior(), ends)
    assert np.max(np.abs(u - exact(ls))) < 1e-12


@pytest.mark.parametrize("pe", [0.3, 0.8, 1.7])
def test_galerkin_advection_recurrence(pe):
    """-mu u'' + c u' = 0, u(0)=0, u(1)=1, uniform mesh: Galerkin nodal values are
    (r^k - 1)/(r^N - 1) with r = (1+Pe)/(1-Pe), Pe = c h / (2 mu)."""
    N = 20
    h = 1.0 / N
    c = 1.0
    mu = c * h / (2 * pe)
    ls = np.linspace(0.0, 1.0, N + 1)
    fam = straight_family([ls])
    M, K, C = lfe.line_operators(fam, np.full(N + 1, c))
    A = K.scale(mu) + C
    ends = np.zeros(N + 1); ends[-1] = 1.0
    u = lfe.solve_lines(A, np.zeros(N + 1), fam.interior(), ends)
    r = (1 + pe) / (1 - pe)
    k = np.arange(N + 1)
    ref = (r ** k - 1) / (r ** N - 1)
    assert np.max(np.abs(u - ref)) < 1e-11 * max(1.0, np.abs(ref).max())


def test_reaction_diffusion_recurrence():
    """-mu u'' + sigma u = 0 with consistent mass on a uniform mesh: the Galerkin
    equations form a constant-coefficient 3-term recurrence whose roots give
    u_k = (r1^k - r2^k) / (r1^N - r2^N) for u_0 = 0, u_N = 1."""
    N, mu, sigma = 16, 0.02, 3.0
    h = 1.0 / N
    ls = np.linspace(0.0, 1.0, N + 1)
    fam = straight_family([ls])
    M, K, _ = lfe.line_operators(fam, None)
    A = K.scale(mu) + M.scale(sigma)
    ends = np.zeros(N + 1); ends[-1] = 1.0
    u = lfe.solve_lines(A, np.zeros(N + 1), fam.interior(), ends)
    al = -mu / h + sigma * h / 6
    be = 2 * mu / h + 2 * sigma * h / 3
    r1, r2 = np.roots([al, be, al])
    k = np.arange(N + 1)
    ref = (r1 ** k - r2 ** k) / (r1 ** N - r2 ** N)
    assert np.max(np.abs(u - ref.real)) < 1e-12


def test_advection_matrix_by_quadrature():
    """Rows of C equal int w phi_j' phi_k with w the P1 interpolant of nodal |beta|,
    integrated by 4-point Gauss quadrature element by element (exact: cubic)."""
    rng = np.random.default_rng(3)
    ls = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, 9)]))
    w = rng.uniform(0.5, 2.0, len(ls))
    fam = straight_family([ls])
    _, _, C = lfe.line_operators(fam, w)
    n = len(ls)
    Cq = np.zeros((n, n))
    gx, gw = np.polynomial.legendre.leggauss(4)
    for e in range(1, n):
        a, b = ls[e - 1], ls[e]
        he = b - a
        for x, wt in zip(gx, gw):
            s = 0.5 * (x + 1)
            phi = {e - 1: 1 - s, e: s}
            dphi = {e - 1: -1 / he, e: 1 / he}
            wl = (1 - s) * w[e - 1] + s * w[e]
            for k in phi:
                for j in dphi:
                    Cq[k, j] += 0.5 * he * wt * wl * dphi[j] * phi[k]
    for k in range(1, n - 1):
        assert abs(C.lo[k] - Cq[k, k - 1]) < 1e-14
        assert abs(C.di[k] - Cq[k, k]) < 1e-14
        assert abs(C.up[k] - Cq[k, k + 1]) < 1e-14


def test_mass_and_stiffness_by_quadrature():
    rng = np.random.default_rng(4)
    ls = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, 7)]))
    fam = straight_family([ls], direction=(-0.8, 0.6))
    M, K, _ = lfe.line_operators(fam, None)
    n = len(ls)
    Mq = np.zeros((n, n)); Kq = np.zeros((n, n))
    gx, gw = np.polynomial.legendre.leggauss(3)
    for e in range(1, n):
        he = ls[e] - ls[e - 1]
        for x, wt in zip(gx, gw):
            s = 0.5 * (x + 1)
            phi = {e - 1: 1 - s, e: s}
            dphi = {e - 1: -1 / he, e: 1 / he}
            for k in phi:
                for j in phi:
                    Mq[k, j] += 0.5 * he * wt * phi[k] * phi[j]
                    Kq[k, j] += 0.5 * he * wt * dphi[k] * dphi[j]
    for k in range(1, n - 1):
        for T, Q in ((M, Mq), (K, Kq)):
            assert abs(T.lo[k] - Q[k, k - 1]) < 1e-12
            assert abs(T.di[k] - Q[k, k]) < 1e-12
            assert abs(T.up[k] - Q[k, k + 1]) < 1e-12


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 200])
def test_thomas_against_dense_and_banded(n):
    rng = np.random.default_rng(n)
    lo = rng.uniform(-1, 1, n)
    up = rng.uniform(-1, 1, n)
    di = np.abs(lo) + np.abs(up) + rng.uniform(0.5, 2, n)
    b = rng.uniform(-1, 1, n)
    x = lfe.thomas(lo, di, up, b)
    A = np.diag(di) + np.diag(lo[1:], -1) + np.diag(up[:-1], 1)
    assert np.max(np.abs(x - np.linalg.solve(A, b))) < 1e-13
    ab = np.zeros((3, n)); ab[0, 1:] = up[:-1]; ab[1] = di; ab[2, :-1] = lo[1:]
    assert np.max(np.abs(x - solve_banded((1, 1), ab, b))) < 1e-13


def test_thomas_brute_force_tiny():
    """3x3 system solved by Cramer's rule."""
    lo = np.array([0.0, 0.5, -0.25]); di = np.array([2.0, 3.0, 1.5]); up = np.array([1.0, -1.0, 0.0])
    b = np.array([1.0, 2.0, 3.0])
    A = np.array([[2.0, 1.0, 0.0], [0.5, 3.0, -1.0], [0.0, -0.25, 1.5]])
    det = np.linalg.det(A)
    ref = []
    for c in range(3):
        Ac = A.copy(); Ac[:, c] = b
        ref.append(np.linalg.det(Ac) / det)
    assert np.max(np.abs(lfe.thomas(lo, di, up, b) - np.array(ref))) < 1e-14


def test_solve_lines_is_independent_per_line():
    rng = np.random.default_rng(9)
    lines = [np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0, 1, m)])) for m in (1, 5, 30)]
    fam = straight_family(lines)
    w = rng.uniform(0.5, 1.5, fam.n_nodes)
    M, K, C = lfe.line_operators(fam, w)
    A = M + K.scale(0.01) + C.scale(0.3)
    rhs = rng.uniform(-1, 1, fam.n_nodes)
    u = lfe.solve_lines(A, rhs, fam.interior())
    for l in range(fam.n_lines):
        a, b = fam.offsets[l], fam.offsets[l + 1]
        ref = lfe.thomas(A.lo[a + 1:b - 1], A.di[a + 1:b - 1], A.up[a + 1:b - 1], rhs[a + 1:b - 1])
        assert np.max(np.abs(u[a + 1:b - 1] - ref)) < 1e-13
        assert u[a] == 0.0 and u[b - 1] == 0.0


def test_exponential_fitting_is_nodally_exact():
    """Il'in / Allen-Southwell: with mu phi(Pe) on each element, -mu u'' + c u' = 0,
    u(0) = 0, u(1) = 1 on a uniform mesh has the nodal values of the exact
    solution (e^{c x / mu} - 1) / (e^{c / mu} - 1), at any mesh Peclet number
    (plain Galerkin oscillates for Pe > 1); as mu grows it tends to Galerkin."""
    N = 20
    ls = np.linspace(0.0, 1.0, N + 1)
    fam = straight_family([ls])
    for mu, c in ((0.05, 1.0), (0.004, 1.0), (0.3, 2.5)):
        w = np.full(N + 1, c)
        _, _, C = lfe.line_operators(fam, w)
        K = lfe.fitted_stiffness(fam, w, mu)
        ends = np.zeros(N + 1); ends[-1] = 1.0
        u = lfe.solve_lines(K.scale(mu) + C, np.zeros(N + 1), fam.interior(), ends)
        x = ls
        ref = np.expm1(c * x / mu) / np.expm1(c / mu)
        assert np.max(np.abs(u - ref)) < 1e-12, mu
    # small Peclet: the fitted stiffness approaches the plain one
    w = np.full(N + 1, 1e-6)
    _, K0, _ = lfe.line_operators(fam, None)
    Kf = lfe.fitted_stiffness(fam, w, 1.0)
    inner = fam.interior()
    assert np.max(np.abs(Kf.di[inner] - K0.di[inner])) < 1e-9 * np.max(np.abs(K0.di[inner]))


def test_fitted_lines_keep_the_solution_free_of_undershoot():
    """A coarse advection-dominated instance (mesh Peclet ~ 10^2) with a
    non-negative source and zero Dirichlet data: the eq. (11) s-solve, whose
    line systems carry no mass term, oscillates with plain Galerkin lines
    (negative values at the outflow layers), and stays non-negative and below
    the reaction bound f / sigma = 1 with the fitted ones."""
    from oracle.method import Oracle
    p = W.constant_beta(33, 2e-4, 1.0, (1.0, 0.4), f=1.0)
    s0 = Oracle(p).s_guess()
    o = Oracle(p, stabilize=True)
    s1 = o.s_guess()
    m = o.inner_idx
    assert s0[m].min() < -0.1
    assert s1[m].min() >= 0.0 and s1[m].max() < 1.0
