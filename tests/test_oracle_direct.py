"""Pins of the interpolation-free transfer (oracle.direct; the conclusions'
second improvement, values handed on at the intersections of the two curve
families)."""
import numpy as np
import pytest

import workloads as W
from oracle import direct as D
from oracle.method import Oracle

from test_oracle_method import _affine_problem


def _orient(ax, ay, bx, by, cx, cy):
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)


def _brute_pairs(tgt, src):
    """All (target segment, source segment) pairs that meet, by orientation
    tests (proper crossings and touching), over every pair of segments."""
    kt = D._segments(tgt)
    ks = D._segments(src)
    out = set()
    near = 0
    for a in kt:
        P0x, P0y, P1x, P1y = tgt.x[a], tgt.y[a], tgt.x[a + 1], tgt.y[a + 1]
        Q0x, Q0y, Q1x, Q1y = src.x[ks], src.y[ks], src.x[ks + 1], src.y[ks + 1]
        o1 = _orient(P0x, P0y, P1x, P1y, Q0x, Q0y)
        o2 = _orient(P0x, P0y, P1x, P1y, Q1x, Q1y)
        o3 = _orient(Q0x, Q0y, Q1x, Q1y, P0x, P0y)
        o4 = _orient(Q0x, Q0y, Q1x, Q1y, P1x, P1y)
        hit = (o1 * o2 <= 0) & (o3 * o4 <= 0) & ~((o1 == 0) & (o2 == 0))
        scale = 1e-12 * (abs(P1x - P0x) + abs(P1y - P0y)) ** 2
        near += int(np.sum(hit & ((np.abs(o1) < scale) | (np.abs(o2) < scale) | (np.abs(o3) < scale)
                                  | (np.abs(o4) < scale))))
        for b in ks[hit]:
            out.add((int(a), int(b)))
    return out, near


def _fams(p):
    o = Oracle(p)
    return o, o.fams[0], o.fams[1]


@pytest.mark.parametrize("maker", [lambda: W.c1(17), lambda: W.c2(21), lambda: W.c4_instance(1, n_max=40),
                                   lambda: W.data2d(17)])
def test_intersections_match_brute_force(maker):
    """The cell search finds exactly the pairs an all-pairs orientation test
    finds (both directions), and each reported point lies on both segments."""
    o, fB, fG = _fams(maker())
    for tgt, src in ((fB, fG), (fG, fB)):
        kt, s, ks, t = D.intersections(o.grid, tgt, src)
        got = set(zip(kt.tolist(), ks.tolist()))
        ref, near = _brute_pairs(tgt, src)
        sym = got ^ ref  # touching pairs (orientation at rounding level) may be decided either way
        assert len(sym) <= near, (len(sym), near)
        assert len(got) > 0
        px = tgt.x[kt] + s * (tgt.x[kt + 1] - tgt.x[kt])
        py = tgt.y[kt] + s * (tgt.y[kt + 1] - tgt.y[kt])
        qx = src.x[ks] + t * (src.x[ks + 1] - src.x[ks])
        qy = src.y[ks] + t * (src.y[ks + 1] - src.y[ks])
        assert np.max(np.hypot(px - qx, py - qy)) < 1e-12


@pytest.mark.parametrize("maker", [lambda: W.c1(33), lambda: W.c2(33), lambda: W.c4_instance(0, n_max=60)])
def test_transfer_rows_are_a_partition_of_unity(maker):
    o, fB, fG = _fams(maker())
    for tgt, src in ((fB, fG), (fG, fB)):
        X, e0, e1 = D.transfer(o.grid, tgt, src)
        inner = tgt.interior()
        rs = np.asarray(X.sum(axis=1)).ravel() + e0 + e1
        assert np.max(np.abs(rs[inner] - 1.0)) < 1e-13
        assert np.all(rs[~inner] == 0.0)
        assert X.data.min() >= -1e-15  # convex combinations


def test_transfer_brackets_brute_force():
    """Each target node's brackets restated node by node: the nearest
    intersection on its curve at or before it and at or after it (by arc
    length), else the curve's end."""
    o, fB, fG = _fams(W.c2(17))
    for tgt, src in ((fB, fG), (fG, fB)):
        X, e0, e1 = D.transfer(o.grid, tgt, src)
        kt, s, ks, t = D.intersections(o.grid, tgt, src)
        for l in range(tgt.n_lines):
            a, b = tgt.offsets[l], tgt.offsets[l + 1]
            # arc coordinates by plain Python sums
            sig = [0.0]
            for k in range(a + 1, b):
                sig.append(sig[-1] + float(np.hypot(tgt.x[k] - tgt.x[k - 1], tgt.y[k] - tgt.y[k - 1])))
            pts = []
            for i in range(len(kt)):
                if a <= kt[i] < b - 1:
                    j = kt[i] - a
                    pts.append((sig[j] + s[i] * (sig[j + 1] - sig[j]), ks[i], t[i]))
            for q in range(a + 1, b - 1):
                sq = sig[q - a]
                left = [p for p in pts if p[0] <= sq]
                right = [p for p in pts if p[0] >= sq]
                L = max(left, key=lambda p: p[0]) if left else (0.0, -1, 0.0)
                R = min(right, key=lambda p: p[0]) if right else (sig[-1], -1, 0.0)
                row = np.zeros(src.n_nodes)
                ee = [0.0, 0.0]
                wL = (R[0] - sq) / (R[0] - L[0]) if R[0] > L[0] else 1.0
                for w, p, side in ((wL, L, 0), (1.0 - wL, R, 1)):
                    if p[1] < 0:
                        ee[side] += w
                    else:
                        row[p[1]] += w * (1 - p[2])
                        row[p[1] + 1] += w * p[2]
                got = X[q].toarray().ravel()
                assert np.max(np.abs(got - row)) < 1e-12
                assert abs(e0[q] - ee[0]) < 1e-12 and abs(e1[q] - ee[1]) < 1e-12


@pytest.mark.parametrize("kind,beta", [("box", (1.0, 0.5)), ("disc", (0.6, -1.1)), ("L", (-0.8, 0.3))])
def test_transfer_exact_on_affine_data_for_straight_curves(kind, beta):
    """Constant beta: both families are straight lines, the P1 value on a
    segment and linear interpolation along a straight curve reproduce an
    affine field exactly, the ends carrying its values."""
    p, u = _affine_problem(kind, 25, beta)
    o, fB, fG = _fams(p)
    f = lambda x, y: 0.7 - 1.3 * x + 0.4 * y
    for tgt, src in ((fB, fG), (fG, fB)):
        X, e0, e1 = D.transfer(o.grid, tgt, src)
        first = np.repeat(f(tgt.x, tgt.y)[tgt.offsets[:-1]], np.diff(tgt.offsets))
        last = np.repeat(f(tgt.x, tgt.y)[tgt.offsets[1:] - 1], np.diff(tgt.offsets))
        v = X @ f(src.x, src.y) + e0 * first + e1 * last
        inner = tgt.interior()
        assert np.max(np.abs(v[inner] - f(tgt.x, tgt.y)[inner])) < 1e-12


def test_transfer_second_order_on_curved_families():
    """On the curved C2 families a smooth field is transferred with an error
    that falls about fourfold when h halves."""
    errs = []
    f = lambda x, y: np.sin(2 * x) * np.cos(3 * y) + x * y
    for n in (33, 65, 129):
        o, fB, fG = _fams(W.c2(n))
        X, e0, e1 = D.transfer(o.grid, fG, fB)
        first = np.repeat(f(fG.x, fG.y)[fG.offsets[:-1]], np.diff(fG.offsets))
        last = np.repeat(f(fG.x, fG.y)[fG.offsets[1:] - 1], np.diff(fG.offsets))
        v = X @ f(fB.x, fB.y) + e0 * first + e1 * last
        inner = fG.interior()
        errs.append(np.max(np.abs(v[inner] - f(fG.x, fG.y)[inner])))
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


@pytest.mark.parametrize("kind,beta", [("box", (1.0, 0.5)), ("disc", (0.6, -1.1)), ("L", (-0.8, 0.3))])
def test_direct_sweep_keeps_the_affine_stationary_solution(kind, beta):
    """The affine solution with g = u (constant beta) is a fixed point of the
    direct sweep, and the iteration from zero reaches it."""
    p, u = _affine_problem(kind, 25, beta)
    o = Oracle(p)
    ds = D.DirectSweeps(o)
    fG = o.fams[1]
    vG = 0.7 - 1.3 * fG.x + 0.4 * fG.y
    m = o.inner_idx
    for theta in (1.0, 0.5):
        assert np.max(np.abs(ds.sweep(vG, theta, 0.05) - vG)) < 1e-12
    U, it, rel, _, _ = ds.iterate(o.zero_field(), 1.0, 0.05, 3000, 1e-13)
    assert rel <= 1e-13 and np.max(np.abs(U[m] - u[m])) < 1e-10


@pytest.mark.parametrize("maker", [lambda: W.c1(9), lambda: W.c2(17), lambda: W.c4_instance(0, n_max=36)])
def test_direct_iteration_limit_is_the_dense_fixed_point(maker):
    """The direct sweep is affine, v -> T v + c on the interior gamma values;
    the iteration's limit solves (I - T) v = c (dense LU)."""
    p = maker()
    X, Y = p.coords()
    p.g = np.sin(3 * X) + Y ** 2
    o = Oracle(p)
    ds = D.DirectSweeps(o)
    inner = np.nonzero(o.inner[1])[0]
    z = ds.zero_state()
    c = ds.sweep(z, 1.0, 0.05)
    T = np.zeros((len(inner), len(inner)))
    for col, q in enumerate(inner):
        e = z.copy()
        e[q] += 1.0
        T[:, col] = (ds.sweep(e, 1.0, 0.05) - c)[inner]
    vd = np.linalg.solve(np.eye(len(inner)) - T, c[inner])
    assert np.max(np.abs(np.linalg.eigvals(T))) < 0.99
    _, it, rel, _, v = ds.iterate(o.zero_field(), 1.0, 0.05, 5000, 1e-14)
    assert np.linalg.norm(v[inner] - vd) / np.linalg.norm(vd) < 1e-11


def test_direct_transfer_is_closer_to_the_exact_solution_than_the_grid_route():
    """Measured finding on the manufactured problem (C1): at the same pseudo
    step the direct transfer's fixed point is nearer the exact solution than
    the grid route's (one interpolation per transfer instead of two)."""
    for n in (17, 33):
        p = W.c1(n)
        o = Oracle(p)
        U, *_ = D.DirectSweeps(o).iterate(o.zero_field(), 1.0, 0.05, 5000, 1e-12)
        Ug, *_ = o.iterate(o.zero_field(), 1.0, 0.05, 5000, 1e-12)
        X, Y = p.coords()
        ue = W.manufactured_u(X, Y).ravel()
        m = o.inner_idx
        assert np.max(np.abs(U[m] - ue[m])) < 0.75 * np.max(np.abs(Ug[m] - ue[m]))


@pytest.mark.parametrize("maker", [lambda: W.c1(17), lambda: W.c2(17), lambda: W.c4_instance(1, n_max=40)])
def test_linear_sweep_is_the_sweep_without_load_and_end_values(maker):
    """The direct sweep is affine in the interior gamma values: with z the
    state carrying the end values and zero inside, sweep(z + v) - sweep(z) is
    the linear part for every v with zero ends, and the linear part maps 0 to 0."""
    p = maker()
    X, Y = p.coords()
    p.g = np.sin(3 * X) + Y ** 2
    o = Oracle(p)
    ds = D.DirectSweeps(o)
    z = ds.zero_state()
    inner = o.inner[1]
    rng = np.random.default_rng(5)
    v = np.where(inner, rng.standard_normal(z.size), 0.0)
    ref = ds.sweep(z + v, 1.0, 0.05) - ds.sweep(z, 1.0, 0.05)
    got = ds.linear_sweep(v, 1.0, 0.05)
    assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))
    assert np.all(got[~inner] == 0.0)
    assert np.all(ds.linear_sweep(np.zeros_like(v), 1.0, 0.05) == 0.0)


def test_hybrid_without_direct_sweeps_is_the_grid_iteration():
    p = W.c2(17)
    o = Oracle(p)
    U, k, rel = D.hybrid_iterate(o, D.DirectSweeps(o), o.zero_field(), 1.0, 0.05, 0, 9, 0.0)
    Ug, it, relg, _ = o.iterate(o.zero_field(), 1.0, 0.05, 9, 0.0)
    assert k == it == 9 and rel == relg and np.array_equal(U, Ug)


@pytest.mark.parametrize("maker", [lambda: W.c1(13), lambda: W.c2(17), lambda: W.c4_instance(0, n_max=40)])
@pytest.mark.parametrize("m", [3, 8])
def test_hybrid_limit_is_the_dense_grid_fixed_point(maker, m):
    """The grid sweep is affine, U -> T U + c on the interior nodes; whatever
    the direct sweeps between two grid sweeps contribute, the hybrid
    iteration stops on a grid sweep whose update is below tol, so its limit
    solves (I - T) U = c (dense LU)."""
    p = maker()
    X, Y = p.coords()
    p.g = np.cos(2 * X) * (1 + Y)
    o = Oracle(p)
    idx = o.inner_idx
    z = o.zero_field()
    c = o.step(z, 1.0, 0.05)
    T = np.zeros((len(idx), len(idx)))
    for col, q in enumerate(idx):
        e = z.copy()
        e[q] += 1.0
        T[:, col] = (o.step(e, 1.0, 0.05) - c)[idx]
    Ud = np.linalg.solve(np.eye(len(idx)) - T, c[idx])
    U, k, rel = D.hybrid_iterate(o, D.DirectSweeps(o), z, 1.0, 0.05, m, 5000, 1e-13)
    assert rel <= 1e-13
    assert np.linalg.norm(U[idx] - Ud) / np.linalg.norm(Ud) < 1e-10
    assert (k - 1) % (m + 1) == 0  # ends on a grid sweep


def test_hybrid_excess_sweeps_fall_as_the_grid_is_refined():
    """Measured finding (C2, blocks of 12 direct sweeps): the direct sweeps
    approximate the grid sweep's linear part up to the difference of the two
    transfers, which shrinks with h, so the sweeps the hybrid needs beyond
    the grid iteration's fall as the grid is refined; on the straight C1
    families (where both transfers are exact on affine data) fewer than one
    block more."""
    excess = []
    for n in (33, 65, 129):
        o = Oracle(W.c2(n))
        _, k, rel = D.hybrid_iterate(o, D.DirectSweeps(o), o.zero_field(), 1.0, 0.05, 12, 3000, 1e-8)
        _, it, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 3000, 1e-8)
        assert rel <= 1e-8
        excess.append(k - it)
    assert excess[0] > excess[1] > excess[2] > 0, excess
    o = Oracle(W.c1(33))
    _, k, _ = D.hybrid_iterate(o, D.DirectSweeps(o), o.zero_field(), 1.0, 0.05, 12, 3000, 1e-8)
    _, it, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 3000, 1e-8)
    assert k <= it + 13
