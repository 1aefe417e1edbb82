"""Interpolation-free transfer between the two curve families (Sec. 8, the
second improvement the conclusions propose: hand values from one family to
the other at the intersection points of their segments, without the
bilinear interpolation through the grid).

Test infrastructure: plain FP64 NumPy/SciPy.  The paper gives the idea
only (no algorithm, no numbers); the pins are mathematical: exactness on
affine data, brute-force searches and the dense fixed point.

Reading of the idea (the paper only sketches it):
  1. every segment of a target curve is intersected with every segment of
     the other (source) family that it meets, closed segments, parallel pairs
     excluded; the value at an intersection is the P1 value on the source
     segment, (1 - t) v_k + t v_{k+1};
  2. along the target curve an intersection sits at the arc-length
     coordinate sigma = (chord sum up to the start of its target segment)
     + s |segment|;
  3. an interior node of the target curve takes the linear interpolant, in
     sigma, between the nearest intersection at or before it and the nearest
     at or after it; where a side has none, the curve's end on that side
     (a point of the boundary, carrying the Dirichlet value) is the bracket.
The paper suggests buckets of segments by azimuthal angle to find the
intersecting pairs; here the candidates are the pairs whose bounding boxes
share a grid cell, an exact test: two segments that meet have overlapping
bounding boxes, and the cell ranges computed from the boxes' ends by floor
then overlap too (floor of a monotone rounding is monotone).

With the transfer X_{G<-B} (beta values to gamma nodes) and X_{B<-G}, one
sweep of eq. (10) on the curve values of the gamma family is
    u_B = X_{B<-G} v_G;   beta substep on the beta-curves  -> v_B
    u_G = X_{G<-B} v_B;   gamma substep on the gamma-curves -> v_G'
(the substeps as in oracle.method).  The stationary iteration starts from
v_G = the bilinear gather of the start field (eq. (22)), measures
rel = |v_G' - v_G|_2 / |Phi(0)|_2 over the interior gamma nodes (Phi(0): the
sweep from zero interior values) and hands back the grid field P_G v_G
(the scatter of Sec. 6), so that it compares with the grid route.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import linefe as lfe


def _segments(fam):
    """First node k of every segment (k, k+1) of the family."""
    start = np.ones(fam.n_nodes - 1, bool)
    start[fam.offsets[1:-1] - 1] = False
    return np.nonzero(start)[0]


def _cell_range(grid, p0, p1, org, h, n_cells):
    lo = np.floor((np.minimum(p0, p1) - org) / h).astype(np.int64)
    hi = np.floor((np.maximum(p0, p1) - org) / h).astype(np.int64)
    return np.clip(lo, 0, n_cells - 1), np.clip(hi, 0, n_cells - 1)


def _cell_members(grid, fam, k):
    """(cell id, segment position) for every grid cell a segment's box overlaps."""
    x0, y0, x1, y1 = fam.x[k], fam.y[k], fam.x[k + 1], fam.y[k + 1]
    ncx, ncy = grid.nx - 1, grid.ny - 1
    i0, i1 = _cell_range(grid, x0, x1, grid.a, grid.hx, ncx)
    j0, j1 = _cell_range(grid, y0, y1, grid.c, grid.hy, ncy)
    wi, wj = i1 - i0 + 1, j1 - j0 + 1
    cnt = wi * wj
    seg = np.repeat(np.arange(len(k)), cnt)
    r = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    ci = i0[seg] + r % wi[seg]
    cj = j0[seg] + r // wi[seg]
    return cj * ncx + ci, seg


def segment_intersection(px0, py0, px1, py1, qx0, qy0, qx1, qy1):
    """Parameters (s, t) of P0 + s (P1 - P0) = Q0 + t (Q1 - Q0) and whether
    both lie in [0, 1]; parallel segments (zero cross product) never meet."""
    rx, ry = px1 - px0, py1 - py0
    qx, qy = qx1 - qx0, qy1 - qy0
    wx, wy = qx0 - px0, qy0 - py0
    den = rx * qy - ry * qx
    ok = den != 0.0
    d = np.where(ok, den, 1.0)
    s = (wx * qy - wy * qx) / d
    t = (wx * ry - wy * rx) / d
    ok &= (s >= 0.0) & (s <= 1.0) & (t >= 0.0) & (t <= 1.0)
    return s, t, ok


def intersections(grid, tgt, src, lines=None):
    """Every meeting of a target segment with a source segment (only the
    target curves in `lines`, if given).

    Returns (kt, s, ks, t): first node of the target segment, position on it,
    first node of the source segment, position on it; sorted by (kt, s, ks)."""
    kt_all, ks_all = _segments(tgt), _segments(src)
    if lines is not None:
        line_of = np.repeat(np.arange(tgt.n_lines), np.diff(tgt.offsets))
        kt_all = kt_all[np.isin(line_of[kt_all], np.asarray(lines))]
    ct, st_ = _cell_members(grid, tgt, kt_all)
    cs, ss_ = _cell_members(grid, src, ks_all)
    # pairs of (target, source) segments sharing a cell
    order = np.argsort(cs, kind="stable")
    cs, ss_ = cs[order], ss_[order]
    lo = np.searchsorted(cs, ct, "left")
    hi = np.searchsorted(cs, ct, "right")
    cnt = hi - lo
    ti = np.repeat(st_, cnt)
    r = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    si = ss_[np.repeat(lo, cnt) + r]
    pair = np.unique(ti.astype(np.int64) * len(ks_all) + si)
    ti, si = pair // len(ks_all), pair % len(ks_all)
    kt, ks = kt_all[ti], ks_all[si]
    s, t, ok = segment_intersection(tgt.x[kt], tgt.y[kt], tgt.x[kt + 1], tgt.y[kt + 1],
                                    src.x[ks], src.y[ks], src.x[ks + 1], src.y[ks + 1])
    kt, s, ks, t = kt[ok], s[ok], ks[ok], t[ok]
    o = np.lexsort((ks, s, kt))
    return kt[o], s[o], ks[o], t[o]


def arc_coordinates(fam):
    """sigma of every node: the chord sum from its line's first node (in order)."""
    h = lfe.chords(fam)
    sig = np.zeros(fam.n_nodes)
    for l in range(fam.n_lines):
        a, b = fam.offsets[l], fam.offsets[l + 1]
        acc = 0.0
        for k in range(a + 1, b):
            acc = acc + h[k]
            sig[k] = acc
    return sig, h


def transfer(grid, tgt, src, lines=None):
    """The direct transfer onto the target family's interior nodes (of the
    target curves in `lines` only, if given: for sampled checks on large
    grids; the other rows stay zero).

    Returns (X, e0, e1): X sparse (tgt nodes x src nodes) and, per target
    node, the weights of its own line's first and last node values (the
    Dirichlet ends, brackets where a side has no intersection).  A target
    node's value is X v_src + e0 * (first end value) + e1 * (last end value);
    rows of end nodes are zero."""
    kt, s, ks, t = intersections(grid, tgt, src, lines)
    sig, h = arc_coordinates(tgt)
    sx = sig[kt] + s * h[kt + 1]            # arc coordinate of each intersection
    line_of = np.repeat(np.arange(tgt.n_lines), np.diff(tgt.offsets))
    lx = line_of[kt]
    rows, cols, vals = [], [], []
    e0 = np.zeros(tgt.n_nodes)
    e1 = np.zeros(tgt.n_nodes)
    inner = tgt.interior()
    for l in (range(tgt.n_lines) if lines is None else lines):
        a, b = tgt.offsets[l], tgt.offsets[l + 1]
        sel = np.nonzero(lx == l)[0]     # sorted by (kt, s): sigma non-decreasing
        xs = sx[sel]
        send = sig[b - 1]
        for q in range(a + 1, b - 1):
            sq = sig[q]
            iL = np.searchsorted(xs, sq, "right") - 1   # last sigma <= sq
            iR = np.searchsorted(xs, sq, "left")        # first sigma >= sq
            if iL >= 0:
                sL, left = xs[iL], sel[iL]
            else:
                sL, left = 0.0, -1
            if iR < len(xs):
                sR, right = xs[iR], sel[iR]
            else:
                sR, right = send, -1
            if sR > sL:
                wL, wR = (sR - sq) / (sR - sL), (sq - sL) / (sR - sL)
            else:
                wL, wR = 1.0, 0.0
            for w, j, end in ((wL, left, 0), (wR, right, 1)):
                if j < 0:
                    (e0 if end == 0 else e1)[q] += w
                else:
                    rows += [q, q]
                    cols += [ks[j], ks[j] + 1]
                    vals += [w * (1.0 - t[j]), w * t[j]]
    X = sp.csr_matrix((vals, (rows, cols)), shape=(tgt.n_nodes, src.n_nodes))
    e0[~inner] = 0.0
    e1[~inner] = 0.0
    return X, e0, e1


class DirectSweeps:
    """The stationary iteration of eq. (10) with the direct transfer, on the
    operators of an oracle.method.Oracle."""

    def __init__(self, o):
        self.o = o
        fB, fG = o.fams
        self.XBG, self.e0B, self.e1B = transfer(o.grid, fB, fG)
        self.XGB, self.e0G, self.e1G = transfer(o.grid, fG, fB)
        self.ends = []
        for fam, ge in zip(o.fams, o.gend):
            first = np.repeat(ge[fam.offsets[:-1]], np.diff(fam.offsets))
            last = np.repeat(ge[fam.offsets[1:] - 1], np.diff(fam.offsets))
            self.ends.append((first, last))

    def to_beta(self, vG, bc=True):
        o = self.o
        u = self.XBG @ vG
        if bc:
            first, last = self.ends[0]
            u = u + self.e0B * first + self.e1B * last
        ends = ~o.inner[0]
        u[ends] = o.gend[0][ends] if bc else 0.0
        return u

    def to_gamma(self, vB, bc=True):
        o = self.o
        u = self.XGB @ vB
        if bc:
            first, last = self.ends[1]
            u = u + self.e0G * first + self.e1G * last
        ends = ~o.inner[1]
        u[ends] = o.gend[1][ends] if bc else 0.0
        return u

    def sweep(self, vG, theta, dt):
        """v_G -> v_G' (one step of eq. (10) on the curve values)."""
        o = self.o
        u = self.to_beta(vG)
        A = o.MB + o.SB.scale(theta * dt)
        rhs = o.MB.apply(u) - (1.0 - theta) * dt * o.SB.apply(u) + dt * o.L
        vB = lfe.solve_lines(A, rhs, o.inner[0], o.gend[0])
        u = self.to_gamma(vB)
        A = o.MG + o.KG.scale(theta * dt * o.mu)
        rhs = o.MG.apply(u) - (1.0 - theta) * dt * o.mu * o.KG.apply(u)
        return lfe.solve_lines(A, rhs, o.inner[1], o.gend[1])

    def linear_sweep(self, vG, theta, dt):
        """The linear part of sweep: zero load and zero Dirichlet values at every
        curve end (the map that carries an update of v_G to the next one)."""
        o = self.o
        u = self.to_beta(vG, bc=False)
        A = o.MB + o.SB.scale(theta * dt)
        rhs = o.MB.apply(u) - (1.0 - theta) * dt * o.SB.apply(u)
        vB = lfe.solve_lines(A, rhs, o.inner[0], np.zeros(o.fams[0].n_nodes))
        u = self.to_gamma(vB, bc=False)
        A = o.MG + o.KG.scale(theta * dt * o.mu)
        rhs = o.MG.apply(u) - (1.0 - theta) * dt * o.mu * o.KG.apply(u)
        return lfe.solve_lines(A, rhs, o.inner[1], np.zeros(o.fams[1].n_nodes))

    def zero_state(self):
        o = self.o
        v = np.zeros(o.fams[1].n_nodes)
        ends = ~o.inner[1]
        v[ends] = o.gend[1][ends]
        return v

    def start(self, U0):
        """v_G from a grid field: the bilinear gather (eq. (22)), g at the ends."""
        return self.o.gather(1, self.o.with_boundary(U0))

    def norm(self, v):
        return float(np.linalg.norm(v[self.o.inner[1]]))

    def iterate(self, U0, theta, dt, max_iters, tol, history=False):
        """Returns (grid field P_G v_G, iterations, rel, history, v_G)."""
        cn = self.norm(self.sweep(self.zero_state(), theta, dt))
        v = self.start(U0)
        rel, it, hist = np.inf, 0, []
        while it < max_iters:
            vn = self.sweep(v, theta, dt)
            rel = self.norm(vn - v) / cn
            v = vn
            it += 1
            hist.append(rel)
            if rel <= tol or not np.isfinite(rel):
                break
        return self.o.scatter(1, v), it, rel, (hist if history else None), v


def hybrid_iterate(o, ds, U0, theta, dt, m, max_iters, tol):
    """The stationary iteration of eq. (10) on the grid (o.step, the grid
    transfer) whose extra sweeps between two full sweeps are taken with the
    direct transfer: after a full sweep U -> U' with update d = U' - U, the
    next m updates are approximated on the gamma-curves, v_1 = T_d G_G d,
    v_{k+1} = T_d v_k (T_d = ds.linear_sweep, G_G the bilinear gather with
    zero ends), and U' + P_G (v_1 + ... + v_m) starts the next full sweep
    (P_G the gamma scatter's linear part).  Only the full sweeps measure
    rel = |U' - U| / |Phi(0)| and stop the iteration, so its limit is the
    grid route's fixed point; the direct sweeps count as sweeps.  Blocks of m
    fixed; m = 0 is o.iterate.  Returns (U, sweeps, rel)."""
    cn = o.c_norm(theta, dt)
    U = o.with_boundary(U0)
    k, rel = 0, np.inf
    inner = o.inner[1]
    while k < max_iters:
        Un = o.step(U, theta, dt)
        d = Un - U
        rel = o.norm(d) / cn
        U = Un
        k += 1
        if rel <= tol or not np.isfinite(rel) or k + m + 1 > max_iters:
            break
        if m:
            v = o.G[1] @ d
            v[~inner] = 0.0
            S = np.zeros_like(v)
            for _ in range(m):
                v = ds.linear_sweep(v, theta, dt)
                S += v
            U = U + o.P[1] @ S
            k += m
    return U, k, rel
