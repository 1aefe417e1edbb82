"""Geometry of the method: the grid over the bounding box, the domain, the unit
fields b and p, the inflow sets and the two curve families.

Test infrastructure (see the package docstring): plain FP64 NumPy.

Paper passages followed:
  Sec. 3: b = beta/|beta|, gamma = (beta2, -beta1), p = gamma/|gamma|.
  eq. (12): inflow sets Gamma_beta = {n.beta < 0}, Gamma_gamma = {n.gamma < 0}.
  eq. (13)-(14): curves are integral curves of beta (resp. gamma) started on
  the inflow sets; finite subsets of each family are taken (end of Sec. 6 intro).
  eq. (20): bounding box P covered by a rectangular mesh.
  eq. (21)-(23): cell index and bilinear interpolation.

Readings where the paper is silent (each stated once here):
  * A point value of the nodal field beta is its bilinear interpolant, eq. (22),
    with the cell index of eq. (21) taken as a 0-based floor clamped to the last
    cell and the y index computed from y (the printed formula uses x: a typo).
    Outside the box the clamped cell extrapolates linearly.
  * Curves are integrated in arc length, dz/dl = b(z) (same curves as
    x_t = beta(x)), by classical RK4 with step h_l = h (the finer grid spacing).
    When a step leaves the closed domain, the exit point is found by 44
    bisections of the step length and projected onto Gamma.  A last element
    shorter than 0.1 h_l is merged into the previous one.
  * Seeds: each connected inflow arc is split into equal increments h_perp = h of
    the measure int |n.b| ds (the transverse spacing of the curves) and one seed is
    placed in the middle of each increment.  The measure is integrated with the
    midpoint rule on sub-segments of length <= h/4.
  * Curves with no interior node are dropped; a curve longer than four
    perimeters means a closed streamline, which eq. (1)'s assumptions exclude.
"""
from __future__ import annotations

import math

import numpy as np

CEIL_TOL = 1e-9      # guard for integer decisions taken from real quotients
N_BISECT = 44        # 2**-44 < 1e-13: exit located to 1e-13 h_l
MERGE_FRAC = 0.1     # last element shorter than this * h_l is merged
NODE_MARGIN = 1e-9   # interior grid node: inside Omega by more than this * h


class BetaError(ValueError):
    """Flow field not admissible: closed/too long streamline or |beta| ~ 0."""


class Grid:
    """Rectangular mesh over the bounding box P = [a,b] x [c,d], eq. (20)."""

    def __init__(self, box, nx, ny):
        self.a, self.b, self.c, self.d = (float(v) for v in box)
        self.nx, self.ny = int(nx), int(ny)
        self.hx = (self.b - self.a) / (self.nx - 1)
        self.hy = (self.d - self.c) / (self.ny - 1)
        self.h = min(self.hx, self.hy)
        self.x = self.a + self.hx * np.arange(self.nx)
        self.y = self.c + self.hy * np.arange(self.ny)

    def cell(self, x, y):
        """eq. (21) and (23): cell (i, j) and fractional offsets (lx, ly)."""
        X = (np.asarray(x, float) - self.a) / self.hx
        Y = (np.asarray(y, float) - self.c) / self.hy
        i = np.clip(np.floor(X), 0, self.nx - 2).astype(np.int64)
        j = np.clip(np.floor(Y), 0, self.ny - 2).astype(np.int64)
        return i, j, X - i, Y - j

    def interp(self, F, x, y):
        """eq. (22): bilinear value of nodal field F (shape (ny, nx)) at (x, y).

        Corners p11, p12, p21, p22 are bottom-left, bottom-right, top-left, top-right.
        """
        i, j, lx, ly = self.cell(x, y)
        p11 = F[j, i]
        p12 = F[j, i + 1]
        p21 = F[j + 1, i]
        p22 = F[j + 1, i + 1]
        return ((1 - ly) * (1 - lx) * p11 + (1 - ly) * lx * p12
                + ly * (1 - lx) * p21 + ly * lx * p22)


# ---------------------------------------------------------------------------
# Domains
# ---------------------------------------------------------------------------

class Polygon:
    """Simple polygon with counter-clockwise vertices (the box is one)."""

    def __init__(self, verts, is_box=False):
        self.V = np.asarray(verts, float)
        self.m = len(self.V)
        self.is_box = is_box
        e = np.roll(self.V, -1, axis=0) - self.V
        cross = e[:, 0] * np.roll(e, -1, axis=0)[:, 1] - e[:, 1] * np.roll(e, -1, axis=0)[:, 0]
        self.convex = bool(np.all(cross >= 0))
        self.perimeter = float(np.sum(np.hypot(e[:, 0], e[:, 1])))

    def inside(self, x, y):
        x = np.asarray(x, float)
        y = np.asarray(y, float)
        if self.is_box:
            a, c = self.V[0]
            b, d = self.V[2]
            return (x > a) & (x < b) & (y > c) & (y < d)
        res = np.zeros(np.broadcast(x, y).shape, bool)
        for q in range(self.m):
            x0, y0 = self.V[q]
            x1, y1 = self.V[(q + 1) % self.m]
            cond = (y0 > y) != (y1 > y)
            with np.errstate(divide="ignore", invalid="ignore"):
                xint = x0 + (y - y0) * (x1 - x0) / (y1 - y0)
            res ^= cond & (x < xint)
        return res

    def dist(self, x, y):
        x = np.asarray(x, float)
        y = np.asarray(y, float)
        best = np.full(np.broadcast(x, y).shape, np.inf)
        for q in range(self.m):
            x0, y0 = self.V[q]
            x1, y1 = self.V[(q + 1) % self.m]
            ex, ey = x1 - x0, y1 - y0
            t = np.clip(((x - x0) * ex + (y - y0) * ey) / (ex * ex + ey * ey), 0.0, 1.0)
            best = np.minimum(best, np.hypot(x - (x0 + t * ex), y - (y0 + t * ey)))
        return best

    def project(self, x, y):
        x = np.asarray(x, float)
        y = np.asarray(y, float)
        best = np.full(x.shape, np.inf)
        px = np.array(x, copy=True)
        py = np.array(y, copy=True)
        for q in range(self.m):
            x0, y0 = self.V[q]
            x1, y1 = self.V[(q + 1) % self.m]
            ex, ey = x1 - x0, y1 - y0
            t = np.clip(((x - x0) * ex + (y - y0) * ey) / (ex * ex + ey * ey), 0.0, 1.0)
            cx, cy = x0 + t * ex, y0 + t * ey
            dd = np.hypot(x - cx, y - cy)
            better = dd < best
            best = np.where(better, dd, best)
            px = np.where(better, cx, px)
            py = np.where(better, cy, py)
        return px, py

    def chord_crosses(self, x0, y0, x1, y1):
        """True where the chord (x0,y0)->(x1,y1) meets Gamma after its start."""
        hit = np.zeros(np.shape(x0), bool)
        dx, dy = x1 - x0, y1 - y0
        for q in range(self.m):
            vx, vy = self.V[q]
            wx, wy = self.V[(q + 1) % self.m]
            ex, ey = wx - vx, wy - vy
            den = dx * ey - dy * ex
            with np.errstate(divide="ignore", invalid="ignore"):
                t = ((vx - x0) * ey - (vy - y0) * ex) / den
                u = ((vx - x0) * dy - (vy - y0) * dx) / den
            hit |= (den != 0) & (t > 1e-9) & (t <= 1.0) & (u >= 0.0) & (u <= 1.0)
        return hit

    def exits(self, x0, y0, x1, y1):
        out = ~self.inside(x1, y1)
        if not self.convex:
            out |= self.chord_crosses(x0, y0, x1, y1)
        return out

    def first_hit(self, x0, y0, x1, y1):
        """Smallest t in (0,1] with (x0,y0)+t((x1,y1)-(x0,y0)) on Gamma; 1 if none."""
        x0, y0, x1, y1 = (np.asarray(v, float) for v in (x0, y0, x1, y1))
        best = np.ones(x0.shape)
        dx, dy = x1 - x0, y1 - y0
        for q in range(self.m):
            vx, vy = self.V[q]
            wx, wy = self.V[(q + 1) % self.m]
            ex, ey = wx - vx, wy - vy
            den = dx * ey - dy * ex
            with np.errstate(divide="ignore", invalid="ignore"):
                t = ((vx - x0) * ey - (vy - y0) * ex) / den
                u = ((vx - x0) * dy - (vy - y0) * dx) / den
            ok = (den != 0) & (t > 0.0) & (t <= 1.0) & (u >= 0.0) & (u <= 1.0)
            best = np.where(ok & (t < best), t, best)
        return best

    def subsegments(self, h):
        """Sub-segments of Gamma (CCW, starting at vertex 0), length <= h/4.

        Returns dict of arrays: start/end points, midpoint, outward normal, length.
        """
        xs0, ys0, xs1, ys1, nxs, nys, lens = [], [], [], [], [], [], []
        for q in range(self.m):
            x0, y0 = self.V[q]
            x1, y1 = self.V[(q + 1) % self.m]
            ell = math.hypot(x1 - x0, y1 - y0)
            K = max(1, math.ceil(ell / (0.25 * h) - CEIL_TOL))
            s = np.arange(K + 1) / K
            px = x0 + s * (x1 - x0)
            py = y0 + s * (y1 - y0)
            xs0.append(px[:-1]); ys0.append(py[:-1])
            xs1.append(px[1:]); ys1.append(py[1:])
            nxs.append(np.full(K, (y1 - y0) / ell))
            nys.append(np.full(K, -(x1 - x0) / ell))
            lens.append(np.full(K, ell / K))
        d = dict(x0=np.concatenate(xs0), y0=np.concatenate(ys0),
                 x1=np.concatenate(xs1), y1=np.concatenate(ys1),
                 nx=np.concatenate(nxs), ny=np.concatenate(nys), len=np.concatenate(lens))
        d["xm"] = 0.5 * (d["x0"] + d["x1"])
        d["ym"] = 0.5 * (d["y0"] + d["y1"])
        return d

    def subsegment_point(self, sub, s, frac):
        return (sub["x0"][s] + frac * (sub["x1"][s] - sub["x0"][s]),
                sub["y0"][s] + frac * (sub["y1"][s] - sub["y0"][s]))


class Disc:
    def __init__(self, cx, cy, r):
        self.cx, self.cy, self.r = float(cx), float(cy), float(r)
        self.convex = True
        self.perimeter = 2.0 * math.pi * self.r

    def inside(self, x, y):
        return (np.asarray(x) - self.cx) ** 2 + (np.asarray(y) - self.cy) ** 2 < self.r * self.r

    def dist(self, x, y):
        return np.abs(self.r - np.hypot(np.asarray(x) - self.cx, np.asarray(y) - self.cy))

    def project(self, x, y):
        dx = np.asarray(x, float) - self.cx
        dy = np.asarray(y, float) - self.cy
        rho = np.hypot(dx, dy)
        return self.cx + self.r * dx / rho, self.cy + self.r * dy / rho

    def exits(self, x0, y0, x1, y1):
        return ~self.inside(x1, y1)

    def first_hit(self, x0, y0, x1, y1):
        x0, y0, x1, y1 = (np.asarray(v, float) for v in (x0, y0, x1, y1))
        dx, dy = x1 - x0, y1 - y0
        px, py = x0 - self.cx, y0 - self.cy
        A = dx * dx + dy * dy
        B = px * dx + py * dy
        C = px * px + py * py - self.r * self.r
        disc = np.maximum(B * B - A * C, 0.0)
        t = (-B + np.sqrt(disc)) / A
        return np.clip(t, 0.0, 1.0)

    def subsegments(self, h):
        K = max(1, math.ceil(self.perimeter / (0.25 * h) - CEIL_TOL))
        th = 2.0 * math.pi * np.arange(K + 1) / K
        t0, t1 = th[:-1], th[1:]
        tm = 0.5 * (t0 + t1)
        d = dict(t0=t0, t1=t1,
                 x0=self.cx + self.r * np.cos(t0), y0=self.cy + self.r * np.sin(t0),
                 x1=self.cx + self.r * np.cos(t1), y1=self.cy + self.r * np.sin(t1),
                 xm=self.cx + self.r * np.cos(tm), ym=self.cy + self.r * np.sin(tm),
                 nx=np.cos(tm), ny=np.sin(tm), len=np.full(K, self.r * 2.0 * math.pi / K))
        return d

    def subsegment_point(self, sub, s, frac):
        t = sub["t0"][s] + frac * (sub["t1"][s] - sub["t0"][s])
        return self.cx + self.r * math.cos(t), self.cy + self.r * math.sin(t)


def make_domain(kind, params, box):
    """kind 0: the box itself; 1: disc (cx, cy, r); 2: polygon (CCW vertex list)."""
    a, b, c, d = box
    if kind == 0:
        return Polygon([(a, c), (b, c), (b, d), (a, d)], is_box=True)
    if kind == 1:
        return Disc(*params)
    if kind == 2:
        return Polygon(params)
    raise ValueError(f"unknown domain kind {kind}")


def interior_mask(grid, dom):
    """Grid nodes strictly inside Omega (by more than NODE_MARGIN*h): the unknowns."""
    X, Y = np.meshgrid(grid.x, grid.y, indexing="xy")
    return dom.inside(X, Y) & (dom.dist(X, Y) > NODE_MARGIN * grid.h)


# ---------------------------------------------------------------------------
# Unit fields (Sec. 3)
# ---------------------------------------------------------------------------

def beta_from_psi(grid, psi):
    """beta = (psi_y, -psi_x) at the nodes from a nodal stream function (Sec. 2:
    beta divergence free): second-order differences, central inside and
    one-sided, (-3 f0 + 4 f1 - f2) / (2 h), on the grid's edges."""
    P = np.asarray(psi, float)

    def d(axis, h):
        out = np.empty_like(P)
        A = np.moveaxis(P, axis, 0)
        O = np.moveaxis(out, axis, 0)
        O[1:-1] = (A[2:] - A[:-2]) / (2.0 * h)
        O[0] = (-3.0 * A[0] + 4.0 * A[1] - A[2]) / (2.0 * h)
        O[-1] = (3.0 * A[-1] - 4.0 * A[-2] + A[-3]) / (2.0 * h)
        return out

    return d(0, grid.hy), -d(1, grid.hx)


class Flow:
    """beta from nodal values; b = beta/|beta|; p = gamma/|gamma| = (b2, -b1)."""

    def __init__(self, grid, beta1, beta2):
        self.grid = grid
        self.B1 = np.asarray(beta1, float)
        self.B2 = np.asarray(beta2, float)

    def beta(self, x, y):
        return self.grid.interp(self.B1, x, y), self.grid.interp(self.B2, x, y)

    def unit(self, x, y, family):
        b1, b2 = self.beta(x, y)
        nrm = np.hypot(b1, b2)
        if np.any(nrm <= 0):
            raise BetaError("|beta| vanishes: the direction b is undefined")
        b1 = b1 / nrm
        b2 = b2 / nrm
        if family == 0:
            return b1, b2
        return b2, -b1

    def rk4(self, x, y, s, family):
        """One classical RK4 step of length s for dz/dl = b(z) (family 0) or p(z) (family 1)."""
        k1x, k1y = self.unit(x, y, family)
        k2x, k2y = self.unit(x + 0.5 * s * k1x, y + 0.5 * s * k1y, family)
        k3x, k3y = self.unit(x + 0.5 * s * k2x, y + 0.5 * s * k2y, family)
        k4x, k4y = self.unit(x + s * k3x, y + s * k3y, family)
        return (x + s / 6.0 * (k1x + 2.0 * k2x + 2.0 * k3x + k4x),
                y + s / 6.0 * (k1y + 2.0 * k2y + 2.0 * k3y + k4y))


# ---------------------------------------------------------------------------
# Seeding on the inflow sets (eq. (12)) and tracing (eq. (13)-(14))
# ---------------------------------------------------------------------------

def seeds(flow, dom, family, h_perp):
    """Seed points on Gamma_beta (family 0) or Gamma_gamma (family 1)."""
    sub = dom.subsegments(flow.grid.h)
    ux, uy = flow.unit(sub["xm"], sub["ym"], family)
    q = np.maximum(0.0, -(sub["nx"] * ux + sub["ny"] * uy))
    w = q * sub["len"]
    pos = w > 0
    K = len(w)
    if not pos.any():
        return np.zeros(0), np.zeros(0)
    if pos.all():
        raise BetaError("the whole boundary is inflow")
    start = int(np.argmin(pos))  # a sub-segment with zero inflow
    order = (start + np.arange(K)) % K
    runs, cur = [], []
    for s in order:
        if pos[s]:
            cur.append(s)
        elif cur:
            runs.append(cur)
            cur = []
    if cur:
        runs.append(cur)
    sx, sy = [], []
    for run in runs:
        wr = w[run]
        cum = np.cumsum(wr)  # sequential partial sums
        lam = cum[-1]
        n = int(math.floor(lam / h_perp + 0.5))
        for k in range(n):
            m = (k + 0.5) * lam / n
            r = int(np.searchsorted(cum, m, side="left"))
            r = min(r, len(run) - 1)
            before = cum[r - 1] if r > 0 else 0.0
            frac = (m - before) / wr[r]
            px, py = dom.subsegment_point(sub, run[r], frac)
            sx.append(px)
            sy.append(py)
    return np.array(sx, float), np.array(sy, float)


class Family:
    """One curve family as polylines: nodes of line l are offsets[l]:offsets[l+1]."""

    def __init__(self, offsets, x, y, family):
        self.offsets = np.asarray(offsets, np.int64)
        self.x = np.asarray(x, float)
        self.y = np.asarray(y, float)
        self.family = family

    @property
    def n_lines(self):
        return len(self.offsets) - 1

    @property
    def n_nodes(self):
        return len(self.x)

    def lengths(self):
        return np.diff(self.offsets)

    def interior(self):
        """Boolean mask of interior line nodes (all but the two Dirichlet ends)."""
        m = np.ones(self.n_nodes, bool)
        m[self.offsets[:-1]] = False
        m[self.offsets[1:] - 1] = False
        return m


def trace(flow, dom, sx, sy, family, hl):
    """Integrate the curves from the seeds; returns a Family (empty lines dropped)."""
    n = len(sx)
    max_steps = int(math.ceil(4.0 * dom.perimeter / hl)) + 2
    X = np.full((max_steps + 2, n), np.nan)
    Y = np.full((max_steps + 2, n), np.nan)
    X[0], Y[0] = sx, sy
    cnt = np.ones(n, np.int64)
    active = np.arange(n)
    cx = np.array(sx, float)
    cy = np.array(sy, float)
    for step in range(1, max_steps + 1):
        if len(active) == 0:
            break
        nx_, ny_ = flow.rk4(cx, cy, hl, family)
        ex = dom.exits(cx, cy, nx_, ny_)
        stay = ~ex
        if stay.any():
            ids = active[stay]
            X[step, ids] = nx_[stay]
            Y[step, ids] = ny_[stay]
            cnt[ids] += 1
        if ex.any():
            ids = active[ex]
            bx, by = cx[ex], cy[ex]
            lo = np.zeros(len(ids))
            hi = np.full(len(ids), hl)
            for _ in range(N_BISECT):
                mid = 0.5 * (lo + hi)
                mx, my = flow.rk4(bx, by, mid, family)
                out = dom.exits(bx, by, mx, my)
                hi = np.where(out, mid, hi)
                lo = np.where(out, lo, mid)
            ex_x, ex_y = flow.rk4(bx, by, hi, family)
            ex_x, ex_y = dom.project(ex_x, ex_y)
            short = np.hypot(ex_x - bx, ex_y - by) < MERGE_FRAC * hl
            for t, l in enumerate(ids):
                if short[t] and cnt[l] >= 2:
                    slot = cnt[l] - 1  # replace the last node by the exit point
                else:
                    slot = cnt[l]
                    cnt[l] += 1
                X[slot, l] = ex_x[t]
                Y[slot, l] = ex_y[t]
        cx = nx_[stay]
        cy = ny_[stay]
        active = active[stay]
    if len(active):
        raise BetaError("a curve did not leave the domain within four perimeters")
    keep = cnt >= 3  # at least one interior node
    xs, ys, offs = [], [], [0]
    for l in np.nonzero(keep)[0]:
        xs.append(X[:cnt[l], l])
        ys.append(Y[:cnt[l], l])
        offs.append(offs[-1] + int(cnt[l]))
    if not xs:
        return Family(np.zeros(1, np.int64), np.zeros(0), np.zeros(0), family)
    return Family(np.array(offs), np.concatenate(xs), np.concatenate(ys), family)


def build_families(grid, dom, flow):
    """Both families with line spacing h_perp = h and node spacing h_l = h."""
    fams = []
    for fam in (0, 1):
        sx, sy = seeds(flow, dom, fam, grid.h)
        fams.append(trace(flow, dom, sx, sy, fam, grid.h))
    return fams
