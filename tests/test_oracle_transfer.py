"""Pins of the oracle's grid <-> curve transfers (Sec. 6, eq. (20)-(23))."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import geometry as geo
from oracle import transfer as tr


def bilinear(x, y):
    return 0.3 - 1.2 * x + 0.7 * y + 2.1 * x * y


def test_gather_exact_on_bilinear(c1_65):
    o = c1_65
    X, Y = np.meshgrid(o.grid.x, o.grid.y, indexing="xy")
    U = bilinear(X, Y).ravel()
    for fam in (0, 1):
        F = o.fams[fam]
        v = o.gather(fam, U)
        m = F.interior()
        assert np.max(np.abs(v[m] - bilinear(F.x[m], F.y[m]))) < 1e-14
        assert np.all(v[~m] == 0.0)  # ends are Dirichlet, never gathered


def test_cell_index_on_grid_lines():
    """eq. (21)/(23) read as 0-based floor: a point on grid line x_i uses cell i
    with lambda = 0 (the last line uses the last cell with lambda = 1)."""
    g = geo.Grid((0.0, 2.0, -1.0, 1.0), 5, 9)
    i, j, lx, ly = g.cell(np.array([0.0, 0.5, 2.0, 1.25]), np.array([-1.0, 0.0, 1.0, 0.125]))
    assert list(i) == [0, 1, 3, 2] and list(j) == [0, 4, 7, 4]
    assert np.allclose(lx, [0, 0, 1, 0.5]) and np.allclose(ly, [0, 0, 1, 0.5])
    F = np.arange(45.0).reshape(9, 5)
    # value at a node is the nodal value
    assert g.interp(F, 0.5, 0.0) == F[4, 1]


def _with_boundary(o, fam, v, fn):
    P, (rows, coef, xb, yb) = tr.scatter_matrix(o.grid, o.dom, o.fams[fam], o.mask)
    out = P @ v
    np.add.at(out, rows, coef * fn(xb, yb))
    return out


@pytest.mark.parametrize("maker", [lambda: W.c1(33), lambda: W.c2(65), lambda: W.c4_instance(0, n_max=80),
                                   lambda: W.c4_instance(1, n_max=80)])
def test_scatter_exact_on_bilinear(maker):
    """Every crossing value is exact for a field linear along the segment, and
    along a grid line an affine field is linear: each estimate, and so their
    average, reproduces the field at the node."""
    from oracle.method import Oracle
    o = Oracle(maker())
    X, Y = np.meshgrid(o.grid.x, o.grid.y, indexing="xy")
    ref = bilinear(X, Y).ravel()
    for fam in (0, 1):
        F = o.fams[fam]
        # P1 values on the polyline segments of a bilinear field are exact only at
        # the nodes; along a straight segment the field is quadratic, so use an
        # affine field for the curved families.
        lin = lambda x, y: 0.3 - 1.2 * x + 0.7 * y  # noqa: E731
        v = lin(F.x, F.y)
        out = _with_boundary(o, fam, v, lin)
        refl = lin(X, Y).ravel()
        assert np.max(np.abs(out - refl)[o.inner_idx]) < 1e-13


def test_round_trip_exact_on_affine_and_second_order():
    """P G u = u for affine u; for smooth u the round trip error is O(h^2)."""
    from oracle.method import Oracle
    errs = []
    fn = lambda x, y: np.sin(2 * x) * np.cos(3 * y)  # noqa: E731
    lin = lambda x, y: 0.5 + 0.25 * x - 0.75 * y  # noqa: E731
    for n in (33, 65, 129):
        o = Oracle(W.c1(n))
        X, Y = np.meshgrid(o.grid.x, o.grid.y, indexing="xy")
        e_fam = []
        for fam in (0, 1):
            F = o.fams[fam]
            ends = ~F.interior()
            for f, store in ((lin, None), (fn, e_fam)):
                U = f(X, Y).ravel()
                v = o.gather(fam, U)
                v[ends] = f(F.x[ends], F.y[ends])
                out = _with_boundary(o, fam, v, f)
                err = np.max(np.abs(out - U)[o.inner_idx])
                if store is None:
                    assert err < 1e-13
                else:
                    store.append(err)
        errs.append(max(e_fam))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, errs


def _brute_scatter(grid, dom, fam, mask, local_edges=4):
    """The scatter rule written out node by node: all crossings of all segments
    with the node's horizontal and vertical grid lines, the closest one on each
    side (the boundary point of the grid line if it comes first), lerp along
    the grid line; then the plain average of the two estimates (Sec. 6), except
    that an estimate with a bracket more than local_edges grid edges from the
    node is dropped when the other estimate is local."""
    nx, ny = grid.nx, grid.ny
    P = np.zeros((nx * ny, fam.n_nodes))
    segs = []
    for l in range(fam.n_lines):
        for k in range(fam.offsets[l], fam.offsets[l + 1] - 1):
            segs.append(k)
    for j in range(ny):
        for i in range(nx):
            if not mask[j, i]:
                continue
            est = []
            for axis in (0, 1):  # 0: horizontal grid line y = y_j, 1: vertical x = x_i
                org, hh, nE, me = (grid.a, grid.hx, nx - 1, i) if axis == 0 else (grid.c, grid.hy, ny - 1, j)
                cs = []
                for k in segs:
                    x0, y0, x1, y1 = fam.x[k], fam.y[k], fam.x[k + 1], fam.y[k + 1]
                    if axis == 0:
                        p0, p1, q0, q1, gl, pos = y0, y1, x0, x1, grid.y[j], grid.x[i]
                    else:
                        p0, p1, q0, q1, gl, pos = x0, x1, y0, y1, grid.x[i], grid.y[j]
                    if p0 == p1 or (gl - p0) * (gl - p1) > 0:
                        continue
                    t = (gl - p0) / (p1 - p0)
                    cs.append((q0 + t * (q1 - q0), k, t))

                # boundary points: walk node by node outward until a non-interior node
                def walk(step):
                    ii, jj = i, j
                    while True:
                        ni, nj = (ii + step, jj) if axis == 0 else (ii, jj + step)
                        if not mask[nj, ni]:
                            x0, y0 = grid.x[ii], grid.y[jj]
                            x1, y1 = grid.x[ni], grid.y[nj]
                            t = float(dom.first_hit(np.array([x0]), np.array([y0]),
                                                    np.array([x1]), np.array([y1]))[0])
                            crd = (x0 + t * (x1 - x0)) if axis == 0 else (y0 + t * (y1 - y0))
                            return crd, (ni if axis == 0 else nj)
                        ii, jj = ni, nj
                (bl, nl), (br, nr) = walk(-1), walk(+1)
                left = [c for c in cs if bl <= c[0] < pos]
                right = [c for c in cs if pos <= c[0] <= br]

                def edge(c):  # the grid edge [x_e, x_e+1] that holds coordinate c
                    return min(max(int(np.floor((c - org) / hh)), 0), nE - 1)
                if left:
                    L = max(left, key=lambda c: c[0])
                    dl = me - edge(L[0])
                else:
                    L, dl = (bl, -1, 0.0), me - nl
                if right:
                    R = min(right, key=lambda c: c[0])
                    dr = edge(R[0]) - me + 1
                else:
                    R, dr = (br, -1, 0.0), nr - me
                dL, dR = pos - L[0], R[0] - pos
                span = dL + dR
                cl, cr = (dR / span, dL / span) if span > 0 else (0.5, 0.5)
                est.append((dl <= local_edges and dr <= local_edges, [(L, cl), (R, cr)]))
            loc = [e[0] for e in est]
            share = [0.5, 0.5] if loc[0] == loc[1] else [float(loc[0]), float(loc[1])]
            for w, (_, parts) in zip(share, est):
                for (crd, k, t), c in parts:
                    if k >= 0:
                        P[j * nx + i, k] += w * c * (1 - t)
                        P[j * nx + i, k + 1] += w * c * t
    return P


@pytest.mark.parametrize("domain", ["box", "disc", "L"])
def test_scatter_matches_brute_force(domain):
    if domain == "box":
        prob = W.c2(13)
    elif domain == "disc":
        prob = W.c4_instance(0, n_max=40)
        prob = W.Problem("disc", 15, 15, prob.box, prob.domain, prob.dom_params, prob.mu, prob.sigma,
                         prob.beta1[:15, :15] * 0 + 1.0, prob.beta2[:15, :15] * 0 + 0.4,
                         np.ones((15, 15)))
    else:
        X, Y = np.meshgrid(np.linspace(0, 1, 13), np.linspace(0, 1, 13), indexing="xy")
        _, b1, b2 = W.curved_stream(X, Y)
        prob = W.Problem("L", 13, 13, (0.0, 1.0, 0.0, 1.0), W.DOM_POLYGON, W.L_SHAPE, 0.01, 1.0,
                         b1, b2, np.ones_like(X))
    from oracle.method import Oracle
    o = Oracle(prob)
    for fam in (0, 1):
        P = o.P[fam].toarray()
        Pb = _brute_scatter(o.grid, o.dom, o.fams[fam], o.mask)
        assert np.max(np.abs(P - Pb)) < 1e-12


def test_scatter_weights_partition_of_unity(c1_65):
    """Rows of P plus boundary weights sum to 1 (a convex combination)."""
    o = c1_65
    for fam in (0, 1):
        P, (rows, coef, _, _) = tr.scatter_matrix(o.grid, o.dom, o.fams[fam], o.mask)
        s = np.asarray(P.sum(axis=1)).ravel()
        np.add.at(s, rows, coef)
        assert np.max(np.abs(s[o.inner_idx] - 1.0)) < 1e-14
        assert P.data.min() >= -1e-15


def test_scatter_is_the_plain_average_where_local():
    """Sec. 6: the node value is the average of the horizontal and the vertical
    estimate.  On C1 (straight curves at an angle to the grid) every bracket is
    local, so the scatter equals the literal rule at every node; with C2's
    curved flow most nodes take the average and the rows of the others put all
    their weight on one grid line."""
    from oracle.method import Oracle
    o = Oracle(W.c1(65))
    for fam in (0, 1):
        P, _ = tr.scatter_matrix(o.grid, o.dom, o.fams[fam], o.mask)
        Pl, _ = tr.scatter_matrix(o.grid, o.dom, o.fams[fam], o.mask, literal=True)
        assert (P != Pl).nnz == 0
    o = Oracle(W.c2(65))
    for fam in (0, 1):
        P, _ = tr.scatter_matrix(o.grid, o.dom, o.fams[fam], o.mask)
        Pl, _ = tr.scatter_matrix(o.grid, o.dom, o.fams[fam], o.mask, literal=True)
        same = np.asarray((abs(P - Pl) > 0).sum(axis=1)).ravel()[o.inner_idx] == 0
        assert same.mean() > 0.75


def test_scatter_grid_aligned_curves_closed_form():
    """beta = (1, 0): the beta-curves are the horizontal lines y = (m + 1/2) h
    with nodes on the vertical grid lines, so no horizontal grid line is crossed
    and the horizontal estimate would interpolate between the two ends of the
    domain.  The vertical estimate alone is used: a line field phi(x) scatters
    to phi(x_i) at every interior node (the literal average gives phi(x_i) / 2,
    the zero boundary value taking the other half)."""
    from oracle.method import Oracle
    p = W.constant_beta(17, 0.1, 1.0, (1.0, 0.0), f=1.0)
    o = Oracle(p)
    F = o.fams[0]
    h = o.grid.h
    ys = np.sort([F.y[F.offsets[l]] for l in range(F.n_lines)])
    assert np.allclose(ys, (np.arange(F.n_lines) + 0.5) * h, atol=1e-13)
    assert np.allclose(F.x / h, np.round(F.x / h), atol=1e-9)
    phi = lambda x: np.cos(3.0 * x) + x ** 3  # noqa: E731
    v = phi(F.x)
    X, _ = np.meshgrid(o.grid.x, o.grid.y, indexing="xy")
    ref = phi(X).ravel()[o.inner_idx]
    got = (o.P[0] @ v)[o.inner_idx]
    assert np.max(np.abs(got - ref)) < 1e-12
    Pl, _ = tr.scatter_matrix(o.grid, o.dom, F, o.mask, literal=True)
    assert np.max(np.abs((Pl @ v)[o.inner_idx] - 0.5 * ref)) < 1e-12
