"""Pins of the oracle's geometry: fields b, p (Sec. 3, eq. (3)), inflow seeding
(eq. (12)) and the curve families (eq. (13)-(14))."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import geometry as geo


def test_identity_split_eq3():
    """b b^T + p p^T = I (eq. (3)) with p = gamma/|gamma|, gamma = (beta2, -beta1)."""
    p = W.c2(33)
    g = geo.Grid(p.box, p.nx, p.ny)
    fl = geo.Flow(g, p.beta1, p.beta2)
    rng = np.random.default_rng(0)
    x, y = rng.uniform(0, 1, 100), rng.uniform(0, 1, 100)
    b1, b2 = fl.unit(x, y, 0)
    p1, p2 = fl.unit(x, y, 1)
    be1, be2 = fl.beta(x, y)
    ga = np.stack([be2, -be1], 1)
    pn = ga / np.linalg.norm(ga, axis=1, keepdims=True)
    assert np.max(np.abs(pn[:, 0] - p1)) < 1e-15 and np.max(np.abs(pn[:, 1] - p2)) < 1e-15
    for k in range(100):
        bb = np.outer([b1[k], b2[k]], [b1[k], b2[k]])
        pp = np.outer([p1[k], p2[k]], [p1[k], p2[k]])
        assert np.max(np.abs(bb + pp - np.eye(2))) < 1e-15


def test_c1_seeds_closed_form():
    """beta = (1, 0.5) on the unit square: inflow set = left side (|n.b| = 2/sqrt5)
    then bottom side (|n.b| = 1/sqrt5); seeds at mid-increments of the measure."""
    p = W.c1(65)
    g = geo.Grid(p.box, p.nx, p.ny)
    dom = geo.make_domain(p.domain, p.dom_params, p.box)
    fl = geo.Flow(g, p.beta1, p.beta2)
    sx, sy = geo.seeds(fl, dom, 0, g.h)
    s5 = math.sqrt(5.0)
    lam = 3.0 / s5
    n = int(math.floor(lam / g.h + 0.5))
    assert len(sx) == n == 86
    for k in range(n):
        m = (k + 0.5) * lam / n
        if m <= 2.0 / s5:
            ex, ey = 0.0, 1.0 - m / (2.0 / s5)
        else:
            ex, ey = (m - 2.0 / s5) / (1.0 / s5), 0.0
        assert abs(sx[k] - ex) < 1e-12 and abs(sy[k] - ey) < 1e-12
    # gamma = (0.5, -1): inflow = top side (|n.p| = 2/sqrt5) and left side (1/sqrt5)
    gx, gy = geo.seeds(fl, dom, 1, g.h)
    assert len(gx) == n


def test_c1_lines_straight_and_spaced():
    p = W.c1(65)
    g = geo.Grid(p.box, p.nx, p.ny)
    dom = geo.make_domain(p.domain, p.dom_params, p.box)
    fl = geo.Flow(g, p.beta1, p.beta2)
    fams = geo.build_families(g, dom, fl)
    s5 = math.sqrt(5.0)
    for fam, d in zip(fams, [(2 / s5, 1 / s5), (1 / s5, -2 / s5)]):
        for l in range(fam.n_lines):
            a, b = fam.offsets[l], fam.offsets[l + 1]
            dx, dy = np.diff(fam.x[a:b]), np.diff(fam.y[a:b])
            ln = np.hypot(dx, dy)
            assert np.max(np.abs(dx / ln - d[0])) < 1e-12 and np.max(np.abs(dy / ln - d[1])) < 1e-12
            assert np.max(np.abs(ln[:-1] - g.h)) < 1e-13
            assert 0.1 * g.h - 1e-13 <= ln[-1] <= 1.1 * g.h + 1e-13
            # both ends on Gamma (the box boundary)
            for k in (a, b - 1):
                assert min(fam.x[k], 1 - fam.x[k], fam.y[k], 1 - fam.y[k]) < 1e-12
        # transverse spacing between consecutive lines is h (perpendicular distance)
        nrm = np.array([-d[1], d[0]])
        offs = [fam.x[fam.offsets[l]] * nrm[0] + fam.y[fam.offsets[l]] * nrm[1]
                for l in range(fam.n_lines)]
        gaps = np.abs(np.diff(offs))
        assert np.max(np.abs(gaps - 3 / s5 / 86)) < 1e-12


def test_data2d_circles_and_rays():
    """beta = (-5(y+1), 5(x+1)) is linear, so its bilinear interpolant is exact:
    beta-curves are circles about (-1,-1) and gamma-curves are rays from it."""
    p = W.data2d(16)
    g = geo.Grid(p.box, p.nx, p.ny)
    dom = geo.make_domain(p.domain, p.dom_params, p.box)
    fl = geo.Flow(g, p.beta1, p.beta2)
    fB, fG = geo.build_families(g, dom, fl)
    for l in range(fB.n_lines):
        a, b = fB.offsets[l], fB.offsets[l + 1]
        r = np.hypot(fB.x[a:b] + 1, fB.y[a:b] + 1)
        assert np.max(np.abs(r - r[0])) < 1e-7 * r[0]
        # counter-clockwise: angle increases along the curve
        th = np.arctan2(fB.y[a:b] + 1, fB.x[a:b] + 1)
        assert np.all(np.diff(th) > 0)
    for l in range(fG.n_lines):
        a, b = fG.offsets[l], fG.offsets[l + 1]
        th = np.arctan2(fG.y[a:b] + 1, fG.x[a:b] + 1)
        assert np.max(np.abs(th - th[0])) < 1e-12
        r = np.hypot(fG.x[a:b] + 1, fG.y[a:b] + 1)
        assert np.all(np.diff(r) > 0)  # gamma = -grad psi = 5(z+1) points away from the centre


def test_stream_function_constant_on_beta_curves():
    """psi is constant along streamlines; the bilinear interpolant of beta is
    divergence free only up to O(h^2), so the drift shrinks under refinement."""
    drift = []
    for n in (65, 129):
        p = W.c2(n)
        g = geo.Grid(p.box, p.nx, p.ny)
        dom = geo.make_domain(p.domain, p.dom_params, p.box)
        fl = geo.Flow(g, p.beta1, p.beta2)
        sx, sy = geo.seeds(fl, dom, 0, g.h)
        fam = geo.trace(fl, dom, sx, sy, 0, g.h)
        _, X2, Y2 = None, *np.meshgrid(g.x, g.y, indexing="xy")
        psi = lambda x, y: x + 0.5 * y + 0.1 * np.sin(np.pi * x) * np.sin(np.pi * y)  # noqa: E731
        d = 0.0
        for l in range(fam.n_lines):
            a, b = fam.offsets[l], fam.offsets[l + 1]
            v = psi(fam.x[a:b], fam.y[a:b])
            d = max(d, np.max(np.abs(v - v[0])))
        drift.append(d)
    assert drift[0] < 2e-3 and drift[1] < drift[0] / 3.0, drift


def test_domains():
    disc = geo.Disc(0.5, 0.5, 0.5)
    assert disc.inside(0.5, 0.9) and not disc.inside(0.9, 0.9)
    t = disc.first_hit(np.array([0.5]), np.array([0.5]), np.array([1.5]), np.array([0.5]))
    assert abs(t[0] - 0.5) < 1e-15
    L = geo.make_domain(2, W.L_SHAPE, (0, 1, 0, 1))
    assert not L.convex
    assert L.inside(0.25, 0.75) and not L.inside(0.75, 0.75) and L.inside(0.75, 0.25)
    # a chord across the notch leaves the domain even though both ends are inside
    assert L.exits(np.array([0.45]), np.array([0.9]), np.array([0.9]), np.array([0.45]))[0]
    px, py = L.project(np.array([0.6]), np.array([0.7]))
    assert abs(px[0] - 0.5) < 1e-15 and abs(py[0] - 0.7) < 1e-15
    g = geo.Grid((0, 1, 0, 1), 101, 101)
    frac = geo.interior_mask(g, disc).mean()
    assert abs(frac - math.pi / 4) < 0.02


@pytest.mark.parametrize("i", [0, 1, 2, 3])
def test_c4_instances_cover_the_grid(i):
    """Every interior node of a disc / L-shape instance is bracketed by records."""
    from oracle.method import Oracle
    p = W.c4_instance(i, n_max=90)
    o = Oracle(p)  # raises if a node has no bracketing record
    assert o.fams[0].n_lines > 0 and o.fams[1].n_lines > 0


def test_beta_from_psi_exact_on_quadratics_and_second_order():
    """Second-order differences (central inside, one-sided on the edges) are
    exact for quadratic stream functions, and their error falls by about 4
    per halving of h on a smooth one; beta = (psi_y, -psi_x) is divergence
    free in the sense that both components come from one psi."""
    g = geo.Grid((0.0, 2.0, -1.0, 1.0), 9, 7)
    X, Y = np.meshgrid(g.x, g.y, indexing="xy")
    psi = 0.3 + 1.1 * X - 0.7 * Y + 0.5 * X * X - 1.3 * X * Y + 0.9 * Y * Y
    b1, b2 = geo.beta_from_psi(g, psi)
    assert np.max(np.abs(b1 - (-0.7 - 1.3 * X + 1.8 * Y))) < 1e-12
    assert np.max(np.abs(b2 + (1.1 + X - 1.3 * Y))) < 1e-12
    errs = []
    for n in (17, 33, 65):
        g = geo.Grid((0.0, 1.0, 0.0, 1.0), n, n)
        X, Y = np.meshgrid(g.x, g.y, indexing="xy")
        psi, e1, e2 = W.curved_stream(X, Y)
        b1, b2 = geo.beta_from_psi(g, psi)
        errs.append(max(np.max(np.abs(b1 - e1)), np.max(np.abs(b2 - e2))))
    assert 3.2 < errs[0] / errs[1] < 4.8 and 3.2 < errs[1] / errs[2] < 4.8, errs
