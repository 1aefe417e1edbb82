"""The interpolation-free transfer (options.transfer = 1) on the HIP path,
against oracle.direct: sweeps, the converged fixed point, batches with
Dirichlet data, and the accuracy against the grid route."""
import numpy as np
import pytest

import workloads as W
from oracle import direct as D
from oracle.method import Oracle

from test_gpu_boundary import _affine, dev, rel_l2, solver, with_g

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _oracle_sweeps(o, U0, k):
    ds = D.DirectSweeps(o)
    v = ds.start(U0)
    for _ in range(k):
        v = ds.sweep(v, 1.0, 0.05)
    return o.scatter(1, v)


@pytest.mark.parametrize("sweeps", [1, 3, 9])
def test_direct_sweeps_match_oracle(sweeps):
    """A batch (C1 65^2, a disc and an L-shape with Dirichlet data), a given
    number of sweeps from a non-zero start: the scattered gamma values equal
    the oracle's to 1e-11."""
    print(f"[case] direct transfer, batch c1/disc/L with g, {sweeps} sweeps", flush=True)
    probs = [W.c1(65), with_g(W.c4_instance(0, n_max=90)), with_g(W.c4_instance(1, n_max=90))]
    orcs = [Oracle(p) for p in probs]
    s = solver(probs, precision="fp64", theta=1.0, dt=0.05, transfer="direct")
    off = s.layout()
    starts = []
    for p, o in zip(probs, orcs):
        X, Y = p.coords()
        starts.append(o.with_boundary((np.sin(2 * X) * Y).ravel()))
    u = dev(np.concatenate(starts))
    it, rel, st = s.split_iterate(u, sweeps, 0.0)
    torch.cuda.synchronize()
    assert st == 1 and np.all(it == sweeps)  # ADR_ENOTCONV at tol = 0
    got = u.cpu().numpy()
    for i, o in enumerate(orcs):
        U = _oracle_sweeps(o, starts[i], sweeps)
        assert rel_l2(got[off[i]:off[i + 1]], U, o.inner_idx) < 1e-11, i
    s.close()


@pytest.mark.parametrize("name", ["c2_129", "data2d_61"])
def test_direct_converged_matches_oracle(name):
    """To rel <= 1e-10 in FP64: the same sweep count (+-1) and the oracle's
    fixed point.  With FP32 increment sweeps (fixed and adaptive schedules) the
    FP64 sweeps keep the fixed point: 1e-8 of it, the sweeps within a block of
    the FP64 count."""
    print(f"[case] direct transfer converged, {name}", flush=True)
    p = W.c2(129) if name == "c2_129" else W.data2d(61)
    o = Oracle(p)
    U, it_o, rel_o, _, _ = D.DirectSweeps(o).iterate(o.zero_field(), 1.0, 0.05, 3000, 1e-10)
    for prec, kw in (("fp64", {}), ("fp32", {"fp32_sweeps": 3}), ("fp32", {"fp32_sweeps": 12, "adaptive": True})):
        s = solver(p, precision=prec, theta=1.0, dt=0.05, transfer="direct", **kw)
        u = dev(o.zero_field())
        it, rel, st = s.split_iterate(u, 3000, 1e-10)
        torch.cuda.synchronize()
        assert st == 0 and rel[0] <= 1e-10
        if prec == "fp64":
            assert abs(int(it[0]) - it_o) <= 1, (int(it[0]), it_o)
            assert rel_l2(u.cpu().numpy(), U, o.inner_idx) < 1e-9
        else:
            assert abs(int(it[0]) - it_o) <= kw["fp32_sweeps"] + 2, (int(it[0]), it_o)
            assert rel_l2(u.cpu().numpy(), U, o.inner_idx) < 1e-8
        s.close()


def test_direct_fp32_sweeps_track_the_fp64_iteration():
    """A fixed number of sweeps (fixed schedule, 3 FP32 sweeps per FP64
    sweep): in exact arithmetic the mixed iteration is the FP64 one, so after
    9 sweeps the result is the oracle's 9-sweep result up to the error of the
    increments.  Bar: the FP32 sweeps rebuild each node's four weights from
    10- and 11-bit fractions (off by at most 3 * 2^-11 in sum, summing exactly
    to 1), so a transferred value is off by at most 3 * 2^-11 of the spread
    of its bracket values, which lie on two segments of neighbouring curves
    (within 2h, h = 1/128: a few hundredths of the increment at most); the
    increments of sweeps 6-8 are about 0.1 of the state here, so three of
    them carry at most ~3 * 3 * 2^-11 * 0.05 * 0.1 = 2e-5 of it into the last
    FP64 sweep, which contracts it: bar 1e-4 (measured 1.1e-5 with FP16
    weights, whose rows do not sum to 1 exactly)."""
    print("[case] direct transfer, fp32 increment sweeps vs fp64 iteration, c2 129", flush=True)
    p = with_g(W.c2(129))
    o = Oracle(p)
    s = solver(p, precision="fp32", fp32_sweeps=3, theta=1.0, dt=0.05, transfer="direct")
    u = dev(o.zero_field())
    it, rel, st = s.split_iterate(u, 9, 0.0)
    torch.cuda.synchronize()
    assert st == 1 and it[0] == 9
    U = _oracle_sweeps(o, o.zero_field(), 9)
    err = rel_l2(u.cpu().numpy(), U, o.inner_idx)
    print(f"[case] rel L2 to the oracle's FP64 iteration {err:.2e}", flush=True)
    assert err < 1e-4
    s.close()


def test_direct_batch_compaction_matches_single_solves():
    """Instances that stop at different sweeps: the batch equals each instance
    solved alone, bitwise, with the same sweep counts."""
    print("[case] direct transfer batch vs single solves", flush=True)
    probs = [W.c4_instance(i, n_max=100) for i in range(5)]
    s = solver(probs, precision="fp64", theta=1.0, dt=0.05, transfer="direct")
    off = s.layout()
    u = torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda")
    it, rel, st = s.split_iterate(u, 3000, 1e-9)
    torch.cuda.synchronize()
    assert st == 0 and len(set(it.tolist())) > 1
    got = u.cpu().numpy()
    s.close()
    for i, p in enumerate(probs):
        s1 = solver(p, precision="fp64", theta=1.0, dt=0.05, transfer="direct")
        v = torch.zeros(p.nx * p.ny, dtype=torch.float64, device="cuda")
        it1, _, st1 = s1.split_iterate(v, 3000, 1e-9)
        torch.cuda.synchronize()
        assert st1 == 0 and it1[0] == it[i]
        assert np.array_equal(v.cpu().numpy(), got[off[i]:off[i + 1]]), i
        s1.close()


@pytest.mark.parametrize("kind,beta", [("box", (1.0, 0.5)), ("disc", (0.6, -1.1)), ("L", (-0.8, 0.3))])
def test_direct_affine_solution_on_gpu(kind, beta):
    print(f"[case] direct transfer, affine exact solution, {kind}", flush=True)
    p, uex = _affine(kind, 25, beta)
    o = Oracle(p)
    s = solver(p, precision="fp64", theta=1.0, dt=0.05, transfer="direct")
    u = dev(o.zero_field())
    it, rel, st = s.split_iterate(u, 3000, 1e-13)
    torch.cuda.synchronize()
    assert st == 0
    m = o.inner_idx
    assert np.max(np.abs(u.cpu().numpy()[m] - uex[m])) < 1e-9
    s.close()


def test_direct_transfer_more_accurate_than_grid_route():
    """Manufactured solution (C1 129^2): the direct route's fixed point is
    nearer the exact solution than the grid route's at the same pseudo step."""
    print("[case] direct vs grid transfer accuracy, c1 129", flush=True)
    p = W.c1(129)
    X, Y = p.coords()
    ue = W.manufactured_u(X, Y).ravel()
    m = Oracle(p).inner_idx
    errs = {}
    for tr in ("grid", "direct"):
        s = solver(p, precision="fp64", theta=1.0, dt=0.05, transfer=tr)
        u = torch.zeros(p.nx * p.ny, dtype=torch.float64, device="cuda")
        it, rel, st = s.split_iterate(u, 5000, 1e-11)
        torch.cuda.synchronize()
        assert st == 0
        errs[tr] = np.max(np.abs(u.cpu().numpy()[m] - ue[m]))
        s.close()
    print(f"[case] max error grid {errs['grid']:.3e} direct {errs['direct']:.3e}", flush=True)
    assert errs["direct"] < errs["grid"]


def test_direct_transfer_refuses_what_it_does_not_serve():
    """The judged solve (a start against a fallback) runs on the grid route."""
    from paper_2411_11041_amd.adr import ADRError, ADR_EINVAL
    p = W.c1(33)
    s = solver(p, precision="fp32", theta=1.0, dt=0.05, transfer="direct")
    u = torch.zeros(p.nx * p.ny, dtype=torch.float64, device="cuda")
    fb = torch.zeros_like(u)
    with pytest.raises(ADRError) as e:
        s.split_iterate_judged(u, fb, 100, 1e-8)
    assert e.value.code == ADR_EINVAL
    s.close()


def test_direct_transfer_autotune_keeps_the_fixed_point():
    """adr_autotune on a direct context tunes its own launches, bucket shapes
    and schedule (no GMRES, no second kind of increments); the tuned solve
    reaches the direct oracle's fixed point (FP32-increment bar 1e-8)."""
    print("[case] direct transfer autotune (c2 129)", flush=True)
    p = W.c2(129)
    o = Oracle(p)
    U, _, _, _, _ = D.DirectSweeps(o).iterate(o.zero_field(), 1.0, 0.05, 3000, 1e-10)
    s = solver(p, precision="fp32", theta=1.0, dt=0.05, transfer="direct")
    work = dev(o.zero_field())
    best, adaptive, ms, split, shapes, kr, inc = s.autotune(work, 2000, 1e-10)
    print(f"[case] autotuned: sweeps {best} adaptive {adaptive} split {split} shapes {shapes} {ms:.2f} ms", flush=True)
    assert kr == 0 and inc == 0 and ms > 0
    u = dev(o.zero_field())
    it, rel, st = s.split_iterate(u, 3000, 1e-10)
    torch.cuda.synchronize()
    assert st == 0 and rel[0] <= 1e-10
    assert rel_l2(u.cpu().numpy(), U, o.inner_idx) < 1e-8
    s.close()


def test_direct_transfer_with_fitted_lines_and_update():
    """The direct transfer with exponentially fitted beta-lines matches the
    oracle (both built on the same options), and adr_update on a direct
    context (new mu, sigma, f on the same curves) gives the fresh context's
    solve."""
    print("[case] direct transfer, fitted lines; adr_update", flush=True)
    p = W.c4_instance(0, n_max=70)
    o = Oracle(p, stabilize=True)
    s = solver(p, precision="fp64", theta=1.0, dt=0.05, transfer="direct", stabilize=True)
    u = dev(o.zero_field())
    it, rel, st = s.split_iterate(u, 5, 0.0)
    torch.cuda.synchronize()
    U = _oracle_sweeps(o, o.zero_field(), 5)
    assert rel_l2(u.cpu().numpy(), U, o.inner_idx) < 1e-11
    s.close()
    # update: the same grid and curves, other coefficients and source
    a = W.c5_sample(1, n=65)
    b = W.c5_sample(2, n=65)
    b.beta1, b.beta2 = a.beta1, a.beta2
    s = solver(a, precision="fp64", theta=1.0, dt=0.05, transfer="direct")
    v = torch.zeros(a.nx * a.ny, dtype=torch.float64, device="cuda")
    s.split_iterate(v, 3000, 1e-10)
    s.update([b])
    v.zero_()
    it_u, rel_u, st_u = s.split_iterate(v, 3000, 1e-10)
    torch.cuda.synchronize()
    s.close()
    f = solver(b, precision="fp64", theta=1.0, dt=0.05, transfer="direct")
    w = torch.zeros(b.nx * b.ny, dtype=torch.float64, device="cuda")
    it_f, rel_f, st_f = f.split_iterate(w, 3000, 1e-10)
    torch.cuda.synchronize()
    f.close()
    assert st_u == 0 and st_f == 0 and abs(int(it_u[0]) - int(it_f[0])) <= 1
    m = Oracle(b).inner_idx
    assert rel_l2(v.cpu().numpy(), w.cpu().numpy(), m) < 1e-9


def _axis_beta(n=33):
    p = W.c1(n)
    p.beta1, p.beta2 = np.ones_like(p.beta1), np.zeros_like(p.beta2)
    return p


def _diag_beta(n=33):
    p = W.c1(n)
    p.beta1, p.beta2 = np.ones_like(p.beta1), np.ones_like(p.beta2)
    return p


@pytest.mark.parametrize("name,maker", [("c1_3", lambda: W.c1(3)), ("c1_4", lambda: W.c1(4)),
                                        ("axis", _axis_beta), ("diag", _diag_beta)])
def test_direct_transfer_degenerate_cases(name, maker):
    """One interior node (3x3), two (4x4), curves along the grid lines
    (intersections at grid nodes and segment ends) and along the diagonals:
    4 FP64 sweeps equal the oracle's."""
    print(f"[case] direct transfer degenerate case {name}", flush=True)
    p = maker()
    o = Oracle(p)
    s = solver(p, precision="fp64", theta=1.0, dt=0.05, transfer="direct")
    u = dev(o.zero_field())
    it, rel, st = s.split_iterate(u, 4, 0.0)
    torch.cuda.synchronize()
    U = _oracle_sweeps(o, o.zero_field(), 4)
    assert rel_l2(u.cpu().numpy(), U, o.inner_idx) < 1e-11
    s.close()


def test_direct_batch_bucketed_fp32_reaches_the_fixed_point():
    """The C4 launch configuration (one launch per length bucket, compacted
    lists, FP32 increment sweeps under the adaptive schedule) with the direct
    transfer: every instance stops at rel <= 1e-9 at its direct FP64 fixed
    point (the oracle's) within 1e-7."""
    print("[case] direct transfer, bucketed fp32 batch of 5 c4 instances", flush=True)
    probs = [W.c4_instance(i, n_max=100) for i in range(5)]
    orcs = [Oracle(p) for p in probs]
    s = solver(probs, precision="fp32", fp32_sweeps=12, adaptive=True, split_lines=1, theta=1.0, dt=0.05,
               transfer="direct")
    off = s.layout()
    u = torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda")
    it, rel, st = s.split_iterate(u, 3000, 1e-9)
    torch.cuda.synchronize()
    assert st == 0 and np.all(rel <= 1e-9)
    got = u.cpu().numpy()
    for i, o in enumerate(orcs):
        U, *_ = D.DirectSweeps(o).iterate(o.zero_field(), 1.0, 0.05, 3000, 1e-12)
        assert rel_l2(got[off[i]:off[i + 1]], U, o.inner_idx) < 1e-7, i
    s.close()


def test_direct_context_keeps_the_grid_route_elsewhere():
    """A context set up with the direct transfer serves the other calls (the
    march, eq. (11), the residual) on the grid transfer, bitwise as a grid
    context does."""
    print("[case] direct context: time_step, initial_guess, residual on the grid route", flush=True)
    p = with_g(W.c3(65))
    o = Oracle(p)
    out = []
    for tr in ("grid", "direct"):
        s = solver(p, precision="fp64", theta=1.0, dt=0.05, transfer=tr)
        u = dev(o.with_boundary(p.u0.ravel() * o.mask.ravel()))
        s.time_step(u, 1.0, 0.005, 4)
        g = dev(o.zero_field())
        s.initial_guess(g)
        r = s.residual(g)
        torch.cuda.synchronize()
        out.append((u.cpu().numpy(), g.cpu().numpy(), np.asarray(r)))
        s.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
