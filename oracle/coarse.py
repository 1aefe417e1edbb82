"""FP64 reference of the coarse-grid transfers of the warm-start network
(test infrastructure: only the tests, the smoke check and the bench's CPU
baseline use this package).

Not in the paper: the network may see the problem on a grid coarsened by an
integer factor r, with the two standard transfers of the multigrid
literature.  A coarse grid of H x W nodes sits inside a fine grid of
Hf = r (H - 1) + 1 by Wf = r (W - 1) + 1 nodes, coarse node (i, j) on fine
node (r i, r j).

* restrict (full weighting): an interior coarse node takes the mean of the
  (2r - 1)^2 fine nodes around its fine node with the tent weights
  (r - |dy|)(r - |dx|) / r^4; a boundary coarse node takes its fine node's
  value (injection).
* prolong (bilinear interpolation): fine node (r i + a, r j + c),
  0 <= a, c < r, takes [(r-a)(r-c) o(i,j) + (r-a) c o(i,j+1)
  + a (r-c) o(i+1,j) + a c o(i+1,j+1)] / r^2.

On interior-supported coarse grids, restrict is the transpose of prolong
divided by r^2; both reproduce bilinear functions.
"""
from __future__ import annotations

import numpy as np


def coarse_shape(Hf, Wf, r):
    H, W = (Hf - 1) // r + 1, (Wf - 1) // r + 1
    if r < 1 or r * (H - 1) + 1 != Hf or r * (W - 1) + 1 != Wf:
        raise ValueError(f"{Hf} x {Wf} is not a grid refined {r} times")
    return H, W


def restrict(fine, r):
    """fine: (B, Hf, Wf) -> coarse (B, H, W)."""
    fine = np.asarray(fine, np.float64)
    B, Hf, Wf = fine.shape
    H, W = coarse_shape(Hf, Wf, r)
    out = fine[:, ::r, ::r].copy()  # injection; interior nodes are overwritten below
    d = np.arange(-(r - 1), r)
    w1 = (r - np.abs(d)) / float(r * r)  # one direction's tent weights, summing to 1
    K = np.outer(w1, w1)
    for i in range(1, H - 1):
        for j in range(1, W - 1):
            patch = fine[:, r * i - (r - 1):r * i + r, r * j - (r - 1):r * j + r]
            out[:, i, j] = (patch * K).sum(axis=(1, 2))
    return out


def prolong(coarse, r):
    """coarse: (B, H, W) -> fine (B, r (H-1) + 1, r (W-1) + 1), bilinear."""
    coarse = np.asarray(coarse, np.float64)
    B, H, W = coarse.shape
    Hf, Wf = r * (H - 1) + 1, r * (W - 1) + 1
    out = np.zeros((B, Hf, Wf))
    x = np.arange(Wf)
    j, c = x // r, x % r
    j1 = np.minimum(j + 1, W - 1)  # c = 0 there, the weight of column j1 is 0
    for y in range(Hf):
        i, a = divmod(y, r)
        i1 = min(i + 1, H - 1)
        out[:, y, :] = ((r - a) * (r - c) * coarse[:, i, j] + (r - a) * c * coarse[:, i, j1]
                        + a * (r - c) * coarse[:, i1, j] + a * c * coarse[:, i1, j1]) / float(r * r)
    return out


def warm_start_prolong(s, sn, out, mask, r):
    """u = s + |s|_inf * prolong(out) where mask is set, 0 elsewhere.

    s: (B, Hf, Wf) fine; sn: (B,); out: (B, H, W) coarse; mask: (Hf, Wf)."""
    p = prolong(out, r)
    u = np.asarray(s, np.float64) + np.asarray(sn, np.float64)[:, None, None] * p
    return np.where(np.asarray(mask, bool)[None], u, 0.0)
