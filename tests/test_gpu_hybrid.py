"""Direct-transfer increment sweeps on the grid route (options.increments = 1)
against the FP64 oracle, through the C ABI.

The FP64 grid sweeps fix the iterate's limit and its residual, so a converged
solve is held to the FP32-lines bar of the other parity tests (1e-5 relative
L2 to the oracle's grid fixed point); a fixed number of sweeps is held to the
oracle's hybrid iteration (oracle.direct.hybrid_iterate) within the error of
the FP32 increments, derived in the test.
"""
import numpy as np
import pytest

import workloads as W
from oracle import direct as D
from oracle.method import Oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_11041_amd import adr
    adr.load()


def solver(p, **kw):
    from paper_2411_11041_amd.adr import Solver
    return Solver(p, **kw)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("name,maker", [("c2_129", lambda: W.c2(129)), ("c4_0", lambda: W.c4_instance(0, n_max=120))])
@pytest.mark.parametrize("m", [1, 4])
def test_hybrid_blocks_match_the_oracle(name, maker, m):
    """Two blocks (a grid sweep, m direct FP32 sweeps, a grid sweep, m more,
    a grid sweep) against the oracle's hybrid iteration in FP64.  The FP32
    sweeps rebuild the transfer weights from 10- and 11-bit fractions (each
    row off by at most 3 * 2^-11 in sum and summing exactly to 1, so a
    transferred value is off by at most 3 * 2^-11 of the spread of its four
    bracket values, which lie within 2h: under a third of the value here,
    h <= 1/100), and the scatter's factored weights (<= 3e-5): each direct
    sweep adds <= 2 * 2^-11 of its increment, summed over m sweeps of
    increments no larger than the first, <= 2 m 2^-11 |S| per block, and
    |S| <= |U| on these starts from zero (the increments shrink).  Two
    blocks: bar 4 m 2^-11 relative L2."""
    print(f"[case] hybrid blocks {name} m={m}", flush=True)
    p = maker()
    o = Oracle(p)
    s = solver(p, precision="fp32", fp32_sweeps=m, increments="direct")
    u = torch.from_numpy(o.zero_field()).cuda()
    n_sweeps = 1 + 2 * (m + 1)
    it, rel, st = s.split_iterate(u, n_sweeps, 0.0)
    torch.cuda.synchronize()
    assert int(it[0]) == n_sweeps
    Uo, k, relo = D.hybrid_iterate(o, D.DirectSweeps(o), o.zero_field(), 1.0, 0.05, m, n_sweeps, 0.0)
    assert k == n_sweeps
    err = rel_l2(u.cpu().numpy(), Uo)
    # the grid-increment path differs from both by the transfers' difference
    g = solver(p, precision="fp32", fp32_sweeps=m)
    ug = torch.from_numpy(o.zero_field()).cuda()
    g.split_iterate(ug, n_sweeps, 0.0)
    torch.cuda.synchronize()
    far = rel_l2(ug.cpu().numpy(), Uo)
    print(f"[case] rel L2 to the oracle's hybrid {err:.2e} (grid increments {far:.2e}); "
          f"rel {rel[0]:.3e} oracle {relo:.3e}", flush=True)
    assert err < 4 * m * 2.0 ** -11
    # and it is the direct increments that ran: the grid increments' distance
    # from the oracle's hybrid (the two transfers' difference) is far larger
    assert err < 0.1 * far
    assert abs(rel[0] - relo) <= 4 * m * 2.0 ** -11 * relo + 1e-12
    s.close()
    g.close()


@pytest.mark.parametrize("name,maker", [("c1_65", lambda: W.c1(65)), ("c2_257", lambda: W.c2(257)),
                                        ("c4_1", lambda: W.c4_instance(1, n_max=160))])
@pytest.mark.parametrize("adaptive", [False, True])
def test_hybrid_reaches_the_grid_fixed_point(name, maker, adaptive):
    print(f"[case] hybrid converged {name} adaptive={adaptive}", flush=True)
    p = maker()
    o = Oracle(p)
    kw = dict(fp32_sweeps=12, adaptive=True) if adaptive else dict(fp32_sweeps=3)
    s = solver(p, precision="fp32", increments="direct", **kw)
    u = torch.from_numpy(o.zero_field()).cuda()
    it, rel, st = s.split_iterate(u, 3000, 1e-10)
    assert st == 0 and rel[0] <= 1e-10
    Uo, ito, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 3000, 1e-12)
    err = rel_l2(u.cpu().numpy(), Uo)
    print(f"[case] {int(it[0])} sweeps (oracle grid iteration {ito} to 1e-12), rel L2 {err:.2e}", flush=True)
    assert err < 1e-5
    # the residual the library measures on the result is its own FP64 grid sweep's
    r = s.residual(u)
    assert r[0] <= 1.5e-10
    s.close()


@pytest.mark.parametrize("schedule", ["fixed", "adaptive"])
def test_hybrid_batch_equals_single_solves_and_graph_replay(schedule):
    """Every instance's arithmetic is its own: the batch (launch lists
    compacted to the unfinished instances) replayed from captured graphs
    (full lists) equals the eager batch bitwise and in sweep counts, on every
    replay with eager work in between; under the fixed schedule each instance
    solved alone equals it too (the adaptive schedule's block lengths follow
    the whole batch)."""
    print(f"[case] hybrid batch {schedule}", flush=True)
    probs = [W.c1(33), W.c2(65), W.c4_instance(2, n_max=100), W.c4_instance(5, n_max=140)]
    kw = dict(precision="fp32", increments="direct", theta=1.0, dt=0.05)
    kw.update(dict(fp32_sweeps=3) if schedule == "fixed" else dict(fp32_sweeps=8, adaptive=True, split_lines=1))
    tol = 1e-9
    batch = solver(probs, **kw)
    off = batch.layout()
    ub = torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda")
    it_b, rel_b, st = batch.split_iterate(ub, 3000, tol)
    torch.cuda.synchronize()
    assert st == 0 and np.all(rel_b <= tol)
    assert len(set(int(v) for v in it_b)) > 1
    graph = solver(probs, graph=True, **kw)
    ug = torch.zeros_like(ub)
    for rep in range(3):
        ug.zero_()
        it_g, _, _ = graph.split_iterate(ug, 3000, tol)
        torch.cuda.synchronize()
        assert np.array_equal(it_g, it_b), rep
        assert torch.equal(ug, ub), rep
        graph.residual(ug)
    for i, p in enumerate(probs if schedule == "fixed" else []):
        one = solver(p, **kw)
        u1 = torch.zeros(p.nx * p.ny, dtype=torch.float64, device="cuda")
        it1, _, _ = one.split_iterate(u1, 3000, tol)
        torch.cuda.synchronize()
        assert int(it1[0]) == int(it_b[i]), i
        assert torch.equal(u1, ub[int(off[i]):int(off[i + 1])]), i
        one.close()
    U = ub.cpu().numpy()
    for i in (1, 3):
        o = Oracle(probs[i])
        Ui, _, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 3000, 1e-12)
        assert rel_l2(U[off[i]:off[i + 1]], Ui) < 1e-5, i
    batch.close()
    graph.close()


def test_hybrid_autotune_keeps_a_candidate_and_the_fixed_point():
    """A context set up with increments = 1 lets the autotuner time both kinds
    of increment sweeps; whatever it keeps, the solve reaches the oracle's
    fixed point."""
    print("[case] autotune with both increment kinds (c2 129)", flush=True)
    p = W.c2(129)
    s = solver(p, precision="fp32", increments="direct")
    o = Oracle(p)
    work = torch.from_numpy(o.zero_field()).cuda()
    best, adaptive, ms, split, shapes, kr, inc = s.autotune(work, 2000, 1e-10)
    print(f"[case] autotuned: sweeps {best} adaptive {adaptive} split {split} krylov {kr} increments {inc} "
          f"{ms:.2f} ms", flush=True)
    assert inc in (0, 1) and ms > 0
    u = torch.from_numpy(o.zero_field()).cuda()
    it, rel, st = s.split_iterate(u, 2000, 1e-10)
    assert st == 0 and rel[0] <= 1e-10
    Uo, _, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 2000, 1e-12)
    assert rel_l2(u.cpu().numpy(), Uo) < 1e-5
    s.close()


def _with_g(p):
    X, Y = p.coords()
    p.g = np.sin(3 * X) + Y ** 2 - 0.5
    return p


@pytest.mark.parametrize("case", ["dirichlet", "fitted", "concurrent", "judged", "update"])
def test_hybrid_with_the_other_options(case):
    """Direct increments combined with the context's other options, each to
    the oracle's grid fixed point (FP32-lines bar): Dirichlet data on the
    boundary (the increments carry none), exponentially fitted beta-lines
    (the direct line kernels take the same fitting factors), bucketed line
    launches on concurrent streams, the judged start, and adr_update (new
    coefficients and source on the same curves, the direct records kept)."""
    print(f"[case] hybrid with {case}", flush=True)
    tol = 1e-10
    kw = dict(precision="fp32", fp32_sweeps=8, adaptive=True, increments="direct")
    if case == "fitted":
        p = W.c4_instance(0, n_max=90)
        o = Oracle(p, stabilize=True)
        kw["stabilize"] = True
    elif case == "update":
        a = W.c5_sample(1, n=97)
        p = W.c5_sample(2, n=97)
        p.beta1, p.beta2 = a.beta1, a.beta2
        o = Oracle(p)
    else:
        p = _with_g(W.c2(129)) if case != "concurrent" else W.c4_instance(3, n_max=160)
        o = Oracle(p)
    if case == "concurrent":
        kw["split_lines"] = 2
    s = solver(a if case == "update" else p, **kw)
    if case == "update":
        s.update([p])
    u = torch.from_numpy(o.zero_field()).cuda()
    if case == "judged":
        fb = torch.from_numpy(o.zero_field()).cuda()
        u = torch.from_numpy(o.with_boundary(0.5 * o.step(o.zero_field(), 1.0, 0.05))).cuda()
        it, rel, st, used = s.split_iterate_judged(u, fb, 3000, tol)
    else:
        it, rel, st = s.split_iterate(u, 3000, tol)
    torch.cuda.synchronize()
    assert st == 0 and rel[0] <= tol
    Uo, _, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 4000, 1e-12)
    err = rel_l2(u.cpu().numpy(), Uo)
    print(f"[case] {int(it[0])} sweeps, rel L2 to the oracle's fixed point {err:.2e}", flush=True)
    assert err < 1e-5
    s.close()
