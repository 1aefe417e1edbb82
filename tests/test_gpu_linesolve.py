"""adr_line_solve: the batched tridiagonal solver on given rows (the line
systems of eq. (16)-(19)), against the oracle's Thomas solve per system."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _systems(lens, seed=0, first=7, dominant=True):
    rng = np.random.default_rng(seed)
    off = np.concatenate([[first], first + np.cumsum(lens)]).astype(np.int64)
    n = int(off[-1]) + 3
    lo, up = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    di = (2.5 if dominant else 0.0) + rng.uniform(0, 1, n)
    rhs = rng.standard_normal(n)
    return off, lo, di, up, rhs


def _reference(off, lo, di, up, rhs):
    from oracle import linefe
    x = np.full(len(rhs), np.nan)
    for l in range(len(off) - 1):
        a, b = int(off[l]), int(off[l + 1])
        if b > a:
            x[a:b] = linefe.thomas(lo[a:b].copy(), di[a:b].copy(), up[a:b].copy(), rhs[a:b].copy())
    return x


def _gpu(off, lo, di, up, rhs, **kw):
    import torch
    from paper_2411_11041_amd.adr import line_solve
    t = [torch.from_numpy(np.ascontiguousarray(v)).cuda() for v in (off, lo, di, up, rhs)]
    x = torch.full_like(t[4], float("nan"))
    sing = torch.full((len(off) - 1,), 7, dtype=torch.int32, device="cuda")
    line_solve(*t, x=x, singular=sing, **kw)
    torch.cuda.synchronize()
    return x.cpu().numpy(), sing.cpu().numpy()


def test_ragged_lengths_match_thomas():
    lens = [1, 2, 3, 31, 32, 33, 63, 64, 65, 96, 97, 1000, 0, 5, 2048, 3, 4097]
    print(f"[case] adr_line_solve ragged lengths {lens}", flush=True)
    off, lo, di, up, rhs = _systems(lens)
    x, sing = _gpu(off, lo, di, up, rhs)
    ref = _reference(off, lo, di, up, rhs)
    m = ~np.isnan(ref)
    assert np.max(np.abs(x[m] - ref[m])) < 1e-13
    assert np.isnan(x[~m]).all()  # rows outside the systems untouched
    assert (sing == 0).all()


def test_one_long_system():
    n = 1_000_003
    print(f"[case] adr_line_solve one system of {n} rows", flush=True)
    off, lo, di, up, rhs = _systems([n], seed=1, first=0)
    x, sing = _gpu(off, lo, di, up, rhs)
    ref = _reference(off, lo, di, up, rhs)
    assert np.max(np.abs(x[:n] - ref[:n])) < 1e-12 * np.max(np.abs(ref[:n]))
    assert sing[0] == 0


def test_galerkin_line_systems():
    """The beta-line systems M + dt S of an advection-dominated instance
    (not diagonally dominant: dt |beta| / 2 > h / 6), assembled by the oracle."""
    from oracle.method import Oracle
    print("[case] adr_line_solve on the oracle's beta-line systems (c4 instance 0, n <= 80)", flush=True)
    o = Oracle(W.c4_instance(0, n_max=80))
    A = o.MB + o.SB.scale(0.05)
    F = o.fams[0]
    inner = F.interior()
    rng = np.random.default_rng(2)
    rhs_full = rng.standard_normal(F.n_nodes)
    # interior rows of each curve form one system (ends eliminated, zero end values)
    rows = np.nonzero(inner)[0]
    lens = [int(inner[F.offsets[l]:F.offsets[l + 1]].sum()) for l in range(F.n_lines)]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    lo, di, up, rhs = A.lo[rows], A.di[rows], A.up[rows], rhs_full[rows]
    x, sing = _gpu(off, lo, di, up, rhs)
    ref = _reference(off, lo, di, up, rhs)
    assert np.max(np.abs(x - ref)) < 1e-11 * np.max(np.abs(ref))
    assert (sing == 0).all()


def test_singular_flags():
    """A zero pivot flags its system (its neighbours stay clear); a pivot
    tolerance above every pivot's scale flags every system."""
    print("[case] adr_line_solve singular flags", flush=True)
    off, lo, di, up, rhs = _systems([40, 70, 5], seed=3)
    di[int(off[1]) + 45] = 0.0
    lo[int(off[1]) + 45] = 0.0  # row 45 of system 1: a zero pivot wherever it is eliminated
    _, sing = _gpu(off, lo, di, up, rhs)
    assert list(sing) == [0, 1, 0]
    off, lo, di, up, rhs = _systems([40, 70, 5], seed=3)
    _, sing = _gpu(off, lo, di, up, rhs, pivot_tol=10.0)
    assert list(sing) == [1, 1, 1]
