"""Seeded synthetic inputs for the directional diffusion splitting solver.

This module only *describes problems*: grids, domains, coefficients and
nodal fields given in closed form (stream functions, their exact
derivatives, Gaussian mixtures).  It holds none of the method's arithmetic
(no tracing, no line elements, no transfers, no solves), so the CPU oracle
and the HIP library can both take their inputs from here without sharing
any solver code.

Problem data follow the paper's problem statement (Sec. 2, eq. (1)-(2)):
constant mu > 0 and sigma > 0, a divergence-free advection field beta
given as nodal values of beta = (psi_y, -psi_x) for a stream function psi,
a nodal source f, Dirichlet data on Gamma (zero, the paper's case, unless a
nodal field g is given) and, for the parabolic problem, an initial value u0.  All nodal arrays are float64, shape
(ny, nx), row-major with index [j, i] for the node (x_i, y_j) of the grid
that covers the bounding box P of eq. (20).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

DOM_BOX = 0
DOM_DISC = 1
DOM_POLYGON = 2

L_SHAPE = ((0.0, 0.0), (1.0, 0.0), (1.0, 0.5), (0.5, 0.5), (0.5, 1.0), (0.0, 1.0))


@dataclass
class Problem:
    """One ADR instance on the grid of its bounding box."""

    name: str
    nx: int
    ny: int
    box: tuple  # (a, b, c, d): P = [a,b] x [c,d]
    domain: int  # DOM_BOX / DOM_DISC / DOM_POLYGON
    dom_params: tuple  # disc: (cx, cy, r); polygon: ((x0,y0), ...) CCW; box: ()
    mu: float
    sigma: float
    beta1: np.ndarray
    beta2: np.ndarray
    f: np.ndarray
    u0: np.ndarray | None = None
    psi: np.ndarray | None = None
    extra: dict = field(default_factory=dict)
    g: np.ndarray | None = None  # nodal Dirichlet data (used on and outside Gamma); None = 0

    @property
    def h(self) -> float:
        a, b, c, d = self.box
        return min((b - a) / (self.nx - 1), (d - c) / (self.ny - 1))

    def coords(self):
        a, b, c, d = self.box
        hx = (b - a) / (self.nx - 1)
        hy = (d - c) / (self.ny - 1)
        x = a + hx * np.arange(self.nx)
        y = c + hy * np.arange(self.ny)
        return np.meshgrid(x, y, indexing="xy")


def _grid(n, box=(0.0, 1.0, 0.0, 1.0)):
    a, b, c, d = box
    hx = (b - a) / (n - 1)
    hy = (d - c) / (n - 1)
    x = a + hx * np.arange(n)
    y = c + hy * np.arange(n)
    return np.meshgrid(x, y, indexing="xy")


def gaussian_mixture(X, Y, rng, k):
    """Sum of k Gaussians: centres U[0.1,0.9]^2, std U[0.02,0.08], amplitude U[0.5,2]."""
    cen = rng.uniform(0.1, 0.9, size=(k, 2))
    s = rng.uniform(0.02, 0.08, size=k)
    amp = rng.uniform(0.5, 2.0, size=k)
    f = np.zeros_like(X)
    for q in range(k):
        r2 = (X - cen[q, 0]) ** 2 + (Y - cen[q, 1]) ** 2
        f += amp[q] * np.exp(-r2 / (2.0 * s[q] ** 2))
    return f


def curved_stream(X, Y):
    """psi = x + 0.5 y + 0.1 sin(pi x) sin(pi y); returns psi, beta1=psi_y, beta2=-psi_x."""
    pi = math.pi
    psi = X + 0.5 * Y + 0.1 * np.sin(pi * X) * np.sin(pi * Y)
    b1 = 0.5 + 0.1 * pi * np.sin(pi * X) * np.cos(pi * Y)
    b2 = -(1.0 + 0.1 * pi * np.cos(pi * X) * np.sin(pi * Y))
    return psi, b1, b2


def manufactured_f(X, Y, mu, sigma, b1, b2):
    """f for u = sin(pi x) sin(pi y) under -mu Lap u + beta.grad u + sigma u (constant beta)."""
    pi = math.pi
    u = np.sin(pi * X) * np.sin(pi * Y)
    ux = pi * np.cos(pi * X) * np.sin(pi * Y)
    uy = pi * np.sin(pi * X) * np.cos(pi * Y)
    return (2.0 * pi * pi * mu + sigma) * u + b1 * ux + b2 * uy


def manufactured_u(X, Y):
    return np.sin(math.pi * X) * np.sin(math.pi * Y)


def constant_beta(n, mu, sigma, beta=(1.0, 0.5), f="manufactured", name="const"):
    X, Y = _grid(n)
    b1 = np.full_like(X, beta[0])
    b2 = np.full_like(X, beta[1])
    if isinstance(f, str) and f == "manufactured":
        fv = manufactured_f(X, Y, mu, sigma, beta[0], beta[1])
    elif callable(f):
        fv = f(X, Y)
    else:
        fv = np.full_like(X, float(f))
    psi = beta[0] * Y - beta[1] * X
    return Problem(name, n, n, (0.0, 1.0, 0.0, 1.0), DOM_BOX, (), mu, sigma,
                   b1, b2, fv, psi=psi)


def c1(n=65):
    """Stationary ADR, unit square, mu=0.1, sigma=1, beta=(1,0.5), manufactured source."""
    return constant_beta(n, 0.1, 1.0, (1.0, 0.5), "manufactured", name=f"c1_{n}")


def c2(n=2049, seed=2):
    """Stationary, advection dominated: mu=1e-3, sigma=1, curved stream, 8 seeded Gaussians."""
    X, Y = _grid(n)
    psi, b1, b2 = curved_stream(X, Y)
    f = gaussian_mixture(X, Y, np.random.default_rng(seed), 8)
    return Problem(f"c2_{n}", n, n, (0.0, 1.0, 0.0, 1.0), DOM_BOX, (), 1e-3, 1.0,
                   b1, b2, f, psi=psi)


def c3(n=2049):
    """Parabolic: mu=1e-2, sigma=0.5, curved stream, f=0, Gaussian bump u0 (zero on Gamma)."""
    X, Y = _grid(n)
    psi, b1, b2 = curved_stream(X, Y)
    u0 = np.exp(-((X - 0.3) ** 2 + (Y - 0.3) ** 2) / (2.0 * 0.05 ** 2))
    u0[0, :] = 0.0
    u0[-1, :] = 0.0
    u0[:, 0] = 0.0
    u0[:, -1] = 0.0
    return Problem(f"c3_{n}", n, n, (0.0, 1.0, 0.0, 1.0), DOM_BOX, (), 1e-2, 0.5,
                   b1, b2, np.zeros_like(X), u0=u0, psi=psi,
                   extra=dict(theta=1.0, dt=0.005, steps=200))


def data2d(n=16):
    """The paper's numerical experiment (Sec. 7, eq. (24)): circular flow about (-1,-1)."""
    X, Y = _grid(n)
    b1 = -5.0 * (Y + 1.0)
    b2 = 5.0 * (X + 1.0)
    psi = -2.5 * ((X + 1.0) ** 2 + (Y + 1.0) ** 2)
    return Problem(f"data2d_{n}", n, n, (0.0, 1.0, 0.0, 1.0), DOM_BOX, (), 1.0, 1.0,
                   b1, b2, np.full_like(X, 5.0), psi=psi,
                   extra=dict(theta=0.5, dt=0.001, steps=50))


def random_stream(X, Y, rng):
    """psi = a(cos(phi) x + sin(phi) y) + sum_{m,n<=3} c_mn sin(m pi x) sin(n pi y).

    Redrawn until |grad psi| >= 0.3 a at every node (no stagnation point, so no
    closed streamline).  Returns psi, beta1 = psi_y, beta2 = -psi_x, a.
    """
    pi = math.pi
    while True:
        a = rng.uniform(0.5, 2.0)
        phi = rng.uniform(0.0, 2.0 * pi)
        cmn = rng.uniform(-1.0, 1.0, size=(3, 3))
        psi = a * (math.cos(phi) * X + math.sin(phi) * Y)
        px = np.full_like(X, a * math.cos(phi))
        py = np.full_like(X, a * math.sin(phi))
        for m in range(1, 4):
            for q in range(1, 4):
                cc = cmn[m - 1, q - 1] * 0.04 * a / (m + q)
                sx, cx = np.sin(m * pi * X), np.cos(m * pi * X)
                sy, cy = np.sin(q * pi * Y), np.cos(q * pi * Y)
                psi = psi + cc * sx * sy
                px = px + cc * m * pi * cx * sy
                py = py + cc * q * pi * sx * cy
        if np.min(np.hypot(px, py)) >= 0.3 * a:
            return psi, py, -px, a


def c4_instance(i, base_seed=1234, n_min=33, n_max=1025):
    """Instance i of the batched workload: disc (even i) or L-shape (odd i)."""
    rng = np.random.default_rng(base_seed + i)
    n = int(rng.integers(n_min, n_max + 1))
    mu = float(10.0 ** rng.uniform(-4.0, -1.0))
    sigma = float(rng.uniform(0.1, 10.0))
    X, Y = _grid(n)
    psi, b1, b2, _ = random_stream(X, Y, rng)
    f = gaussian_mixture(X, Y, rng, 8)
    if i % 2 == 0:
        dom, par = DOM_DISC, (0.5, 0.5, 0.5)
    else:
        dom, par = DOM_POLYGON, L_SHAPE
    return Problem(f"c4_{i}", n, n, (0.0, 1.0, 0.0, 1.0), dom, par, mu, sigma,
                   b1, b2, f, psi=psi)


def c4(n_instances=512, base_seed=1234, n_min=33, n_max=1025):
    return [c4_instance(i, base_seed, n_min, n_max) for i in range(n_instances)]


def c5_sample(seed, n=257):
    """Warm-start dataset sample: unit square, sigma=1, curved stream, mu logU[1e-3,1e-1]."""
    rng = np.random.default_rng(seed)
    mu = float(10.0 ** rng.uniform(-3.0, -1.0))
    k = int(rng.integers(1, 9))
    X, Y = _grid(n)
    psi, b1, b2 = curved_stream(X, Y)
    f = gaussian_mixture(X, Y, rng, k)
    return Problem(f"c5_{seed}", n, n, (0.0, 1.0, 0.0, 1.0), DOM_BOX, (), mu, 1.0,
                   b1, b2, f, psi=psi)

