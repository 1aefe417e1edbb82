"""Transfers between the grid and the curve families (Sec. 6, eq. (20)-(23)).

Test infrastructure: plain FP64 NumPy/SciPy.  Both transfers are linear, so
each is built once as a sparse matrix from its definition and applied by a
sparse product.

Gather G (grid -> line nodes), Sec. 6.1: bilinear interpolation, eq. (22), in
the cell of eq. (21)/(23).  Only interior line nodes are gathered; end nodes
are Dirichlet nodes whose values are set, never interpolated.

Scatter P (line nodes -> grid), Sec. 6 (the scheme recalled from the authors'
advection-reaction paper):
  1. every polyline segment is intersected with every grid line it meets; the
     crossing value is the P1 (linear) value on the segment;
  2. on every grid edge (the piece of a grid line between two adjacent nodes)
     only the crossing with the minimal and the one with the maximal
     coordinate are kept;
  3. at a grid node, the closest crossing on each side along its horizontal
     grid line (the max record of the edge to the left, the min record of the
     edge to the right) gives a linear interpolant; the same along the
     vertical grid line;
  4. the node value is the average of the two estimates.
Readings: an edge with no crossing passes the search on to the next edge
outward; where the grid line leaves Omega first, the boundary point acts as a
crossing carrying the Dirichlet value (zero for increments).  Step 4 is the
plain average wherever both estimates are local: an estimate is local when
each of its two brackets lies on one of the LOCAL_EDGES grid edges nearest
the node on that side (within 4 grid spacings).  Where only one estimate is
local, that estimate alone is the node value; this is the case where the
curves run along (or nearly along) a grid line, so that the line carries no
crossing for many edges and its estimate would interpolate across a large
part of the domain.  Where neither is local the plain average is kept.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

LOCAL_EDGES = 4  # a bracket found further out than this many edges is not local


def gather_matrix(grid, fam):
    """Sparse G: (n_line_nodes, nx*ny); zero rows at line ends."""
    inner = np.nonzero(fam.interior())[0]
    i, j, lx, ly = grid.cell(fam.x[inner], fam.y[inner])
    nx = grid.nx
    cols = np.stack([j * nx + i, j * nx + i + 1, (j + 1) * nx + i, (j + 1) * nx + i + 1], 1)
    vals = np.stack([(1 - ly) * (1 - lx), (1 - ly) * lx, ly * (1 - lx), ly * lx], 1)
    rows = np.repeat(inner, 4)
    return sp.csr_matrix((vals.ravel(), (rows, cols.ravel())),
                         shape=(fam.n_nodes, grid.nx * grid.ny))


def crossings(grid, fam):
    """All crossings of polyline segments with grid lines.

    Returns two record sets (vertical grid lines x = x_i, horizontal y = y_j):
    arrays line (grid-line index), coord (coordinate along that grid line),
    k (first node of the segment), t (position on the segment, value
    (1-t) u_k + t u_{k+1}).
    """
    start = np.ones(fam.n_nodes - 1, bool)
    start[fam.offsets[1:-1] - 1] = False  # no segment from a line's last node
    k = np.nonzero(start)[0]
    x0, y0 = fam.x[k], fam.y[k]
    x1, y1 = fam.x[k + 1], fam.y[k + 1]
    out = []
    for axis in (0, 1):
        if axis == 0:   # vertical grid lines x = x_i
            p0, p1, q0, q1 = x0, x1, y0, y1
            org, hh, nl, gl = grid.a, grid.hx, grid.nx, grid.x
        else:           # horizontal grid lines y = y_j
            p0, p1, q0, q1 = y0, y1, x0, x1
            org, hh, nl, gl = grid.c, grid.hy, grid.ny, grid.y
        lo = np.floor((np.minimum(p0, p1) - org) / hh).astype(np.int64) - 1
        hi = np.ceil((np.maximum(p0, p1) - org) / hh).astype(np.int64) + 1
        lo = np.clip(lo, 0, nl - 1)
        hi = np.clip(hi, 0, nl - 1)
        cnt = hi - lo + 1
        seg = np.repeat(np.arange(len(k)), cnt)
        first = np.repeat(np.cumsum(cnt) - cnt, cnt)
        cand = lo[seg] + (np.arange(len(seg)) - first)
        g = gl[cand]
        a0, a1 = p0[seg], p1[seg]
        ok = ((g - a0) * (g - a1) <= 0.0) & (a0 != a1)
        seg, g, cand = seg[ok], g[ok], cand[ok]
        t = (g - p0[seg]) / (p1[seg] - p0[seg])
        coord = q0[seg] + t * (q1[seg] - q0[seg])
        out.append(dict(line=cand, coord=coord, k=k[seg], t=t))
    return out


def _edge_minmax(rec, n_lines, n_edges, org, hh):
    """Per grid edge: index of the min- and max-coordinate record (-1 if empty)."""
    e = np.clip(np.floor((rec["coord"] - org) / hh).astype(np.int64), 0, n_edges - 1)
    eid = rec["line"] * n_edges + e
    order = np.lexsort((rec["coord"], eid))
    emin = np.full(n_lines * n_edges, -1, np.int64)
    emax = np.full(n_lines * n_edges, -1, np.int64)
    se = eid[order]
    if len(se):
        firsts = np.ones(len(se), bool)
        firsts[1:] = se[1:] != se[:-1]
        lasts = np.ones(len(se), bool)
        lasts[:-1] = se[1:] != se[:-1]
        emin[se[firsts]] = order[firsts]
        emax[se[lasts]] = order[lasts]
    return emin.reshape(n_lines, n_edges), emax.reshape(n_lines, n_edges)


def _bracket(emin, emax, inner_line, rec, gl, pos_of_line, dom, along_x, fixed):
    """For every node position p on every grid line (rows: grid lines), find the
    closest record at-or-before and at-or-after along the line.

    inner_line: (n_lines, n_nodes) interior-node mask along each grid line.
    Returns for each side (kind: 0 line record / 1 boundary, idx, coord, depth),
    depth the number of edges from the node to the edge holding the bracket.
    """
    nL, nE = emin.shape
    nN = nE + 1
    edges = np.arange(nE)[None, :]
    # left side: edge e is a stopper if it has records or node e is not interior
    stopL = (emax >= 0) | ~inner_line[:, :-1]
    markL = np.where(stopL, edges, -1)
    nearL = np.maximum.accumulate(markL, axis=1)            # at or left of edge e
    # right side: edge e stops if it has records or node e+1 is not interior
    stopR = (emin >= 0) | ~inner_line[:, 1:]
    markR = np.where(stopR, edges, nE)
    nearR = np.minimum.accumulate(markR[:, ::-1], axis=1)[:, ::-1]
    res = {}
    for side in ("L", "R"):
        kind = np.full((nL, nN), -1, np.int64)
        idx = np.full((nL, nN), -1, np.int64)
        coord = np.full((nL, nN), np.nan)
        depth = np.zeros((nL, nN), np.int64)  # 1 = the node's own edge on that side
        for p in range(nN):
            if side == "L":
                if p == 0:
                    continue
                e = nearL[:, p - 1]
                valid = e >= 0
                rid = np.where(valid, emax[np.arange(nL), np.maximum(e, 0)], -1)
                far = np.maximum(e, 0)           # node on the far side of the edge
                near = far + 1
                depth[:, p] = p - e
            else:
                if p == nN - 1:
                    continue
                e = nearR[:, p]
                valid = e < nE
                rid = np.where(valid, emin[np.arange(nL), np.minimum(e, nE - 1)], -1)
                far = np.minimum(e, nE - 1) + 1
                near = far - 1
                depth[:, p] = e - p + 1
            has = valid & (rid >= 0)
            kind[has, p] = 0
            idx[has, p] = rid[has]
            coord[has, p] = rec["coord"][rid[has]]
            bnd = valid & (rid < 0)
            if bnd.any():
                L = np.nonzero(bnd)[0]
                if along_x:
                    xs0, ys0 = gl[near[L]], fixed[L]
                    xs1, ys1 = gl[far[L]], fixed[L]
                    t = dom.first_hit(xs0, ys0, xs1, ys1)
                    coord[L, p] = xs0 + t * (xs1 - xs0)
                else:
                    xs0, ys0 = fixed[L], gl[near[L]]
                    xs1, ys1 = fixed[L], gl[far[L]]
                    t = dom.first_hit(xs0, ys0, xs1, ys1)
                    coord[L, p] = ys0 + t * (ys1 - ys0)
                kind[L, p] = 1
        res[side] = (kind, idx, coord, depth)
    return res


def scatter_matrix(grid, dom, fam, node_mask, literal=False):
    """Sparse P: (nx*ny, n_line_nodes) and the boundary-record list.

    node_mask: (ny, nx) interior grid nodes (rows of P exist only for these).
    literal: average the two estimates at every node, local or not (the rule
    of Sec. 6 with no fallback; used only to compare the readings).
    Returns P and (rows, coefs, xb, yb): the weight each boundary crossing point
    (xb, yb) carries in row `rows` (used when the scattered field has non-zero
    values on Gamma).
    """
    recs = crossings(grid, fam)
    nx, ny = grid.nx, grid.ny
    # vertical grid lines x = x_i: lines indexed by i, edges along y
    vmin, vmax = _edge_minmax(recs[0], nx, ny - 1, grid.c, grid.hy)
    hmin, hmax = _edge_minmax(recs[1], ny, nx - 1, grid.a, grid.hx)
    # horizontal estimate: along rows j (grid line y = y_j), positions i
    H = _bracket(hmin, hmax, node_mask, recs[1], grid.x, None, dom, True, grid.y)
    V = _bracket(vmin, vmax, node_mask.T, recs[0], grid.y, None, dom, False, grid.x)
    J, I = np.nonzero(node_mask)
    rows_all, cols_all, vals_all = [], [], []
    b_rows, b_coef, b_x, b_y = [], [], [], []

    def side_info(D, a_, b_, rec):
        kind, idx, coord, depth = D
        return kind[a_, b_], idx[a_, b_], coord[a_, b_], depth[a_, b_]

    # horizontal: grid line j, position i ; vertical: grid line i, position j
    kLh, iLh, cLh, eLh = side_info(H["L"], J, I, recs[1])
    kRh, iRh, cRh, eRh = side_info(H["R"], J, I, recs[1])
    kLv, iLv, cLv, eLv = side_info(V["L"], I, J, recs[0])
    kRv, iRv, cRv, eRv = side_info(V["R"], I, J, recs[0])
    xi, yj = grid.x[I], grid.y[J]
    dL_h, dR_h = xi - cLh, cRh - xi
    dL_v, dR_v = yj - cLv, cRv - yj
    # share of the horizontal estimate: 1/2 (the average), or 1 / 0 where only
    # the horizontal / only the vertical estimate is local
    loc_h = (eLh <= LOCAL_EDGES) & (eRh <= LOCAL_EDGES)
    loc_v = (eLv <= LOCAL_EDGES) & (eRv <= LOCAL_EDGES)
    if literal:
        loc_h = loc_v = np.ones(len(J), bool)
    W_h = np.where(loc_h == loc_v, 0.5, np.where(loc_h, 1.0, 0.0))
    W_v = 1.0 - W_h

    def lerp_coefs(dL, dR):
        span = dL + dR
        safe = span > 0
        cl = np.where(safe, dR / np.where(safe, span, 1.0), 0.5)
        cr = np.where(safe, dL / np.where(safe, span, 1.0), 0.5)
        return cl, cr

    clh, crh = lerp_coefs(dL_h, dR_h)
    clv, crv = lerp_coefs(dL_v, dR_v)
    gidx = J * nx + I
    for kind, ridx, coef, rec, along_x, crd in (
            (kLh, iLh, W_h * clh, recs[1], True, cLh),
            (kRh, iRh, W_h * crh, recs[1], True, cRh),
            (kLv, iLv, W_v * clv, recs[0], False, cLv),
            (kRv, iRv, W_v * crv, recs[0], False, cRv)):
        ln = kind == 0
        kk = rec["k"][ridx[ln]]
        tt = rec["t"][ridx[ln]]
        rows_all += [gidx[ln], gidx[ln]]
        cols_all += [kk, kk + 1]
        vals_all += [coef[ln] * (1.0 - tt), coef[ln] * tt]
        bd = kind == 1
        b_rows.append(gidx[bd])
        b_coef.append(coef[bd])
        if along_x:
            b_x.append(crd[bd]); b_y.append(yj[bd])
        else:
            b_x.append(xi[bd]); b_y.append(crd[bd])
        if np.any(kind < 0):
            raise RuntimeError("interior grid node without a bracketing record")
    P = sp.csr_matrix((np.concatenate(vals_all),
                       (np.concatenate(rows_all), np.concatenate(cols_all))),
                      shape=(nx * ny, fam.n_nodes))
    bnd = (np.concatenate(b_rows), np.concatenate(b_coef),
           np.concatenate(b_x), np.concatenate(b_y))
    return P, bnd
