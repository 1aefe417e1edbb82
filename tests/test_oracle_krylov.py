"""Pins of the Krylov acceleration (oracle.krylov): GMRES against direct
solves, and the accelerated stationary solve against the dense fixed point."""
import numpy as np
import pytest

import workloads as W
from oracle import dense, krylov
from oracle.method import Oracle


def test_gmres_full_space_is_the_direct_solve():
    """Without restart, GMRES on an n x n system is exact after n steps
    (the Krylov space is the whole space); its residual never increases."""
    rng = np.random.default_rng(0)
    n = 30
    A = rng.standard_normal((n, n)) + 4.0 * np.eye(n)
    b = rng.standard_normal(n)
    x, k, hist = krylov.gmres(lambda v: A @ v, b, np.zeros(n), 1e-14, n, 10 * n)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-12 * np.linalg.norm(x)
    est = hist[:-1]  # the Givens estimates of the cycle (the last entry is the recomputed residual)
    assert all(h2 <= h1 * (1 + 1e-12) for h1, h2 in zip(est, est[1:]))


def test_gmres_restarted_nonsymmetric_with_start():
    """Restarted GMRES(5) from a non-zero start on a non-normal (advection-like)
    tridiagonal system reaches the direct solution."""
    n = 200
    A = np.diag(np.full(n, 2.3)) + np.diag(np.full(n - 1, -1.6), -1) + np.diag(np.full(n - 1, 0.2), 1)
    b = np.sin(np.arange(n))
    x, k, hist = krylov.gmres(lambda v: A @ v, b, np.ones(n), 1e-12, 5, 5000)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-10 * np.linalg.norm(x)
    assert hist[-1] <= 1e-12


@pytest.mark.parametrize("maker", [lambda: W.c1(9), lambda: W.c1(17), lambda: W.c2(17),
                                   lambda: W.c4_instance(1, n_max=33)])
def test_accelerated_solve_is_the_dense_fixed_point(maker):
    """The fixed point is the method's, whatever the solver: GMRES(10) on
    (I - T) U = c equals the dense LU solution, in fewer sweeps than the
    plain iteration needs for the same residual."""
    p = maker()
    X, Y = p.coords()
    p.g = 0.1 * np.cos(2 * X) * Y  # non-zero Dirichlet data too
    o = Oracle(p)
    Ud = dense.fixed_point(o, 1.0, 0.05)
    U, n, hist = krylov.solve_fixed_point(o, 1.0, 0.05, 1e-13, restart=10)
    m = o.inner_idx
    assert np.linalg.norm(U[m] - Ud[m]) / np.linalg.norm(Ud[m]) < 1e-11
    _, it, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 5000, 1e-8)
    _, n8, _ = krylov.solve_fixed_point(o, 1.0, 0.05, 1e-8, restart=10)
    assert n8 < it
