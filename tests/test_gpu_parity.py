"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Tolerances: FP64 mode 1e-11 relative (iterate by iterate: same geometry, same
sweep sequence); FP32 line solves with the FP64 state and residual: 1e-5
relative L2 on the converged solution.
"""
import numpy as np
import pytest

import workloads as W
from oracle.method import Oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


def rel_l2(a, b, mask=None):
    if mask is not None:
        a, b = a[mask], b[mask]
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_11041_amd import adr
    adr.load()


def solver(p, **kw):
    from paper_2411_11041_amd.adr import Solver
    return Solver(p, **kw)


@pytest.mark.parametrize("sweeps", [1, 3, 12])
def test_fp64_sweeps_match_oracle_c1(sweeps):
    print(f"[case] c1 65 fp64 sweeps={sweeps}", flush=True)
    p = W.c1(65)
    o = Oracle(p)
    s = solver(p, precision="fp64", theta=1.0, dt=0.05)
    u = dev(o.zero_field())
    iters, rel, st = s.split_iterate(u, sweeps, 0.0)
    torch.cuda.synchronize()
    U = o.zero_field()
    for _ in range(sweeps):
        U = o.step(U, 1.0, 0.05)
    assert iters[0] == sweeps
    assert rel_l2(u.cpu().numpy(), U) < 1e-11
    s.close()


def test_fp64_converged_and_residual_c1():
    print("[case] c1 65 fp64 converged", flush=True)
    p = W.c1(65)
    o = Oracle(p)
    s = solver(p, precision="fp64", theta=1.0, dt=0.05)
    u = dev(o.zero_field())
    iters, rel, st = s.split_iterate(u, 400, 1e-10)
    Uo, ito, relo, _ = o.iterate(o.zero_field(), 1.0, 0.05, 400, 1e-10)
    assert st == 0 and rel[0] <= 1e-10
    assert abs(int(iters[0]) - ito) <= 1
    assert rel_l2(u.cpu().numpy(), Uo) < 1e-9
    # adr_residual equals the oracle's measure.  Near convergence the update is a
    # difference of nearly equal FP64 numbers, so compare in absolute terms there
    # (units of |Phi(0)|) and relatively on an unconverged iterate.
    r = s.residual(dev(Uo))
    assert abs(r[0] - o.rel_residual(Uo, 1.0, 0.05)) <= 1e-13
    U5 = o.zero_field()
    for _ in range(5):
        U5 = o.step(U5, 1.0, 0.05)
    r5 = s.residual(dev(U5))
    assert abs(r5[0] - o.rel_residual(U5, 1.0, 0.05)) <= 1e-11 * r5[0]
    s.close()


@pytest.mark.parametrize("name,maker", [("c1_65", lambda: W.c1(65)), ("c2_257", lambda: W.c2(257))])
def test_fp32_lines_converged(name, maker):
    print(f"[case] {name} fp32 lines converged", flush=True)
    p = maker()
    o = Oracle(p)
    s = solver(p, precision="fp32", fp32_sweeps=3, theta=1.0, dt=0.05)
    u = dev(o.zero_field())
    iters, rel, st = s.split_iterate(u, 2000, 1e-10)
    assert st == 0 and rel[0] <= 1e-10
    Uo, ito, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 2000, 1e-12)
    assert rel_l2(u.cpu().numpy(), Uo) < 1e-5
    s.close()


def test_time_march_c3_small():
    print("[case] c3 129 time march 10 steps fp64", flush=True)
    p = W.c3(129)
    o = Oracle(p)
    s = solver(p, precision="fp64")
    u0 = p.u0.ravel() * o.mask.ravel()
    u = dev(u0)
    s.time_step(u, 1.0, 0.005, 10)
    torch.cuda.synchronize()
    U = o.march(u0, 1.0, 0.005, 10)
    assert rel_l2(u.cpu().numpy(), U) < 1e-11
    s.close()


def test_data2d_paper_experiment():
    """Sec. 7 set-up: eq. (11) start, theta = 1/2, 50 steps of dt = 0.001."""
    print("[case] data2d 61 theta=0.5 50 steps", flush=True)
    p = W.data2d(61)
    o = Oracle(p)
    s = solver(p, precision="fp64")
    u = dev(o.zero_field())
    s.initial_guess(u)
    torch.cuda.synchronize()
    U0 = o.s_guess()
    assert rel_l2(u.cpu().numpy(), U0) < 1e-12
    s.time_step(u, 0.5, 0.001, 50)
    torch.cuda.synchronize()
    U = o.march(U0, 0.5, 0.001, 50)
    assert rel_l2(u.cpu().numpy(), U) < 1e-11
    s.close()


@pytest.mark.parametrize("split,shapes", [(0, None), (1, None), (2, None), (1, (0, 0, 1, 1, 1)),
                                          (1, (0, 0, 0, 2, 2)), (1, (1, 1, 2, 1, 1))])
def test_batched_instances_match_oracle(split, shapes):
    """Disc and L-shape instances of uneven sizes in one context (one launch per
    kernel for all of them, or one per length bucket: curves of up to 256
    nodes on 64-thread workgroups, up to 512 on 128, up to 1024 on 512):
    every instance matches its own oracle."""
    print(f"[case] batched c4 x4 fp64 8 sweeps, line launches {split}, shapes {shapes}", flush=True)
    probs = [W.c4_instance(i, n_max=140) for i in range(3)] + [W.c4_instance(7, n_max=600)]
    s = solver(probs, precision="fp64", theta=1.0, dt=0.05, split_lines=split)
    if shapes is not None:
        s.set_line_shapes(shapes)
    off = s.layout()
    u = torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda")
    iters, rel, st = s.split_iterate(u, 8, 0.0)
    torch.cuda.synchronize()
    U = u.cpu().numpy()
    for i, p in enumerate(probs):
        o = Oracle(p)
        Ui = o.zero_field()
        for _ in range(8):
            Ui = o.step(Ui, 1.0, 0.05)
        assert rel_l2(U[off[i]:off[i + 1]], Ui) < 1e-11, i
    s.close()


def test_batched_early_exit_per_instance():
    """Instances converge at different sweeps; a converged one stops changing."""
    print("[case] batched convergence per instance", flush=True)
    probs = [W.c1(33), W.c2(65)]
    s = solver(probs, precision="fp64", theta=1.0, dt=0.05)
    off = s.layout()
    u = torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda")
    iters, rel, st = s.split_iterate(u, 500, 1e-9)
    assert st == 0 and np.all(rel <= 1e-9)
    for i, p in enumerate(probs):
        o = Oracle(p)
        Ui, it, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 500, 1e-9)
        assert abs(int(iters[i]) - it) <= 1
        assert rel_l2(u.cpu().numpy()[off[i]:off[i + 1]], Ui) < 1e-8
    s.close()


def test_deterministic_fp64():
    print("[case] determinism", flush=True)
    p = W.c2(129)
    s = solver(p, precision="fp64")
    a = torch.zeros(p.nx * p.ny, dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)
    s.split_iterate(a, 7, 0.0)
    s.split_iterate(b, 7, 0.0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    s.close()


def test_graph_replay_matches_eager():
    """The captured-graph path replays the same kernels: every replay, with eager
    work and synchronisations in between, equals the eager result bitwise."""
    print("[case] hipGraph replay vs eager (fp32 lines, c2 129)", flush=True)
    p = W.c2(129)
    eager = solver(p, precision="fp32", fp32_sweeps=3)
    graph = solver(p, precision="fp32", fp32_sweeps=3, graph=True)
    ref = torch.zeros(p.nx * p.ny, dtype=torch.float64, device="cuda")
    it_e, rel_e, _ = eager.split_iterate(ref, 41, 0.0)
    torch.cuda.synchronize()
    u = torch.zeros_like(ref)
    for rep in range(3):
        u.zero_()
        it_g, rel_g, _ = graph.split_iterate(u, 41, 0.0)
        torch.cuda.synchronize()
        assert int(it_g[0]) == int(it_e[0]) == 41
        assert torch.equal(u, ref), rep
        # eager work on the same context between replays
        r = graph.residual(u)
        assert abs(r[0] - rel_e[0]) <= 1e-12 + 1e-9 * rel_e[0] or r[0] < rel_e[0]
    # convergence stop inside the graph
    u.zero_()
    it, rel, st = graph.split_iterate(u, 400, 1e-9)
    assert st == 0 and rel[0] <= 1e-9
    eager.close()
    graph.close()


def test_update_swaps_coefficients_on_same_curves():
    """adr_update replaces mu, sigma and f on the traced curves: the next sweeps
    equal the oracle of the new problems, and the set-up's sizes are kept."""
    print("[case] adr_update c5 65 x2 fp64 6 sweeps", flush=True)
    a = [W.c5_sample(s, n=65) for s in (0, 1)]
    b = [W.c5_sample(s, n=65) for s in (7, 8)]
    for p in b:
        p.beta1, p.beta2 = a[0].beta1, a[0].beta2
    for p in a[1:]:
        p.beta1, p.beta2 = a[0].beta1, a[0].beta2
    s = solver(a, precision="fp64", theta=1.0, dt=0.05)
    off = s.layout()
    u = torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda")
    s.split_iterate(u, 3, 0.0)
    s.update(b)
    u.zero_()
    iters, rel, st = s.split_iterate(u, 6, 0.0)
    torch.cuda.synchronize()
    U = u.cpu().numpy()
    for i, p in enumerate(b):
        o = Oracle(p)
        Ui = o.zero_field()
        for _ in range(6):
            Ui = o.step(Ui, 1.0, 0.05)
        assert rel_l2(U[off[i]:off[i + 1]], Ui) < 1e-11, i
    with pytest.raises(Exception):
        s.update(b[:1])
    s.close()


def test_autotune_keeps_a_candidate_and_the_fixed_point():
    """The autotuner picks one of its candidate FP32-sweep counts; the solve
    with the chosen count reaches the oracle's fixed point (FP32-lines bar)."""
    print("[case] autotune c2 129 fp32 lines", flush=True)
    p = W.c2(129)
    s = solver(p, precision="fp32", fp32_sweeps=3)
    work = torch.zeros(p.nx * p.ny, dtype=torch.float64, device="cuda")
    best, adaptive, ms, split, shapes, kr, inc = s.autotune(work, 2000, 1e-10)
    assert ((best in (2, 3, 4, 6) and not adaptive) or (best in (6, 8, 12, 16, 24) and adaptive)) and ms > 0
    assert split in (0, 1, 2)
    assert all(0 <= v < n for v, n in zip(shapes, (2, 2, 3, 3, 3)))
    u = torch.zeros_like(work)
    iters, rel, st = s.split_iterate(u, 2000, 1e-10)
    assert st == 0 and rel[0] <= 1e-10
    o = Oracle(p)
    Uo, _, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 3000, 1e-12)
    assert rel_l2(u.cpu().numpy(), Uo) < 1e-5
    s.close()


def _const_beta(n, b1, b2):
    p = W.c1(n)
    p.beta1, p.beta2 = np.full_like(p.beta1, b1), np.full_like(p.beta2, b2)
    return p


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("name,maker", [("c1_3", lambda: W.c1(3)), ("c1_4", lambda: W.c1(4)),
                                        ("c1_5", lambda: W.c1(5)),
                                        ("axis_33", lambda: _const_beta(33, 1.0, 0.0)),
                                        ("diag_33", lambda: _const_beta(33, 1.0, 1.0))])
def test_degenerate_cases_match_oracle(name, maker, split):
    """One interior node; curves on grid lines; curves through grid nodes."""
    print(f"[case] degenerate {name} fp64 6 sweeps, line launches {split}", flush=True)
    p = maker()
    o = Oracle(p)
    s = solver(p, precision="fp64", theta=1.0, dt=0.05, split_lines=split)
    u = dev(o.zero_field())
    s.split_iterate(u, 6, 0.0)
    torch.cuda.synchronize()
    U = o.zero_field()
    for _ in range(6):
        U = o.step(U, 1.0, 0.05)
    assert rel_l2(u.cpu().numpy(), U) < 1e-11
    s.close()


def test_curve_beyond_the_line_solver_is_rejected():
    """The longest curve the LDS line solver holds is 3072 nodes: C2's flow on
    2700^2 has gamma-curves of up to 3216 nodes, which set-up rejects (2049^2,
    the benchmark size, has at most 2440)."""
    print("[case] c2 2700 set-up (a curve over 3072 nodes)", flush=True)
    from paper_2411_11041_amd.adr import ADRError, ADR_EINVAL
    with pytest.raises(ADRError) as e:
        solver(W.c2(2700), precision="fp32")
    assert e.value.code == ADR_EINVAL and "3072" in str(e.value)


def test_batched_fp32_lines_match_oracle_fixed_points():
    """FP32 line solves on a batch of disc and L-shape instances of uneven sizes
    (grids that are no multiple of the 8 x 4 blocks of the FP32 increment
    fields): every instance reaches its oracle fixed point (FP32-lines bar)."""
    print("[case] batched c4 x4 fp32 lines to 1e-10", flush=True)
    probs = [W.c4_instance(i, n_max=140) for i in range(4)]
    s = solver(probs, precision="fp32", fp32_sweeps=3, theta=1.0, dt=0.05)
    off = s.layout()
    u = torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda")
    iters, rel, st = s.split_iterate(u, 3000, 1e-10)
    assert st == 0 and np.all(rel <= 1e-10)
    U = u.cpu().numpy()
    for i, p in enumerate(probs):
        assert p.nx % 8 or p.ny % 4 or i == 0  # at least the later sizes are ragged
        o = Oracle(p)
        Ui, _, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 3000, 1e-12)
        assert rel_l2(U[off[i]:off[i + 1]], Ui) < 1e-5, i
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_compaction_matches_single_solves(precision):
    """Instances of a batch converge at different sweeps, so the eager solve
    shrinks its launches to the unfinished instances after each check.  Every
    instance's arithmetic is its own, so each must equal, bitwise and in sweep
    count, the same instance solved alone (no compaction) and the batch replayed
    from a captured graph (full launches)."""
    print(f"[case] batch compaction vs single solves ({precision})", flush=True)
    probs = [W.c1(33), W.c2(65), W.c4_instance(2, n_max=100), W.c4_instance(5, n_max=140)]
    kw = dict(precision=precision, theta=1.0, dt=0.05)
    if precision == "fp32":
        kw["fp32_sweeps"] = 3
    tol = 1e-9
    batch = solver(probs, **kw)
    off = batch.layout()
    ub = torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda")
    it_b, rel_b, st = batch.split_iterate(ub, 2000, tol)
    torch.cuda.synchronize()
    assert st == 0 and np.all(rel_b <= tol)
    assert len(set(int(v) for v in it_b)) > 1  # the instances stop at different sweeps
    graph = solver(probs, graph=True, **kw)
    ug = torch.zeros_like(ub)
    it_g, _, _ = graph.split_iterate(ug, 2000, tol)
    torch.cuda.synchronize()
    assert np.array_equal(it_g, it_b)
    assert torch.equal(ug, ub)
    for i, p in enumerate(probs):
        one = solver(p, **kw)
        u1 = torch.zeros(p.nx * p.ny, dtype=torch.float64, device="cuda")
        it1, _, _ = one.split_iterate(u1, 2000, tol)
        torch.cuda.synchronize()
        assert int(it1[0]) == int(it_b[i]), i
        assert torch.equal(u1, ub[int(off[i]):int(off[i + 1])]), i
        one.close()
    batch.close()
    graph.close()


@pytest.mark.parametrize("name,maker,tol", [("c2_257", lambda: [W.c2(257)], 1e-10),
                                            ("batch", lambda: [W.c1(33), W.c2(65), W.c4_instance(2, n_max=100)], 1e-9)])
def test_adaptive_schedule_reaches_the_fixed_point(name, maker, tol):
    """The adaptive schedule (FP64 sweeps placed where rel is predicted to reach
    tol) stops every instance at rel <= tol on an FP64 sweep and reaches the
    oracle's fixed point (FP32-lines bar); a single instance needs at most one
    sweep more than the fixed schedule (4 FP32 sweeps per FP64 sweep)."""
    print(f"[case] adaptive schedule {name}", flush=True)
    probs = maker()
    fixed = solver(probs, precision="fp32", fp32_sweeps=4)
    ada = solver(probs, precision="fp32", fp32_sweeps=8, adaptive=True)
    off = fixed.layout()
    uf = torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda")
    ua = torch.zeros_like(uf)
    it_f, rel_f, st_f = fixed.split_iterate(uf, 3000, tol)
    it_a, rel_a, st_a = ada.split_iterate(ua, 3000, tol)
    assert st_f == 0 and st_a == 0 and np.all(rel_a <= tol)
    if len(probs) == 1:
        assert int(it_a[0]) <= int(it_f[0]) + 1
    U = ua.cpu().numpy()
    for i, p in enumerate(probs):
        o = Oracle(p)
        Ui, _, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 3000, 1e-12)
        assert rel_l2(U[off[i]:off[i + 1]], Ui) < 1e-5, i
    fixed.close()
    ada.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_judged_iterate_keeps_a_better_start_bitwise(precision):
    """A start whose residual is below the fallback's is kept: the judged solve
    then equals the plain solve from that start, bitwise and in sweep count
    (the fallback's residual sweep leaves the state alone)."""
    print(f"[case] judged iterate, better start kept ({precision})", flush=True)
    probs = [W.c1(33), W.c2(65), W.c4_instance(2, n_max=100)]
    kw = dict(precision=precision, theta=1.0, dt=0.05)
    if precision == "fp32":
        kw["fp32_sweeps"] = 3
    tol = 1e-9
    s = solver(probs, **kw)
    off = s.layout()
    start = torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda")
    s.split_iterate(start, 6, 0.0)  # six sweeps from zero: residual below zero's (1)
    zero = torch.zeros_like(start)
    u_p = start.clone()
    it_p, rel_p, st_p = s.split_iterate(u_p, 2000, tol)
    u_j = start.clone()
    it_j, rel_j, st_j, used = s.split_iterate_judged(u_j, zero, 2000, tol)
    torch.cuda.synchronize()
    assert st_p == 0 and st_j == 0
    assert not used.any()
    assert np.array_equal(it_j, it_p)
    assert torch.equal(u_j, u_p)
    s.close()


def test_judged_iterate_restarts_worse_starts():
    """Instances whose start is worse than the fallback (a NaN start, a start
    far from the solution) restart from the fallback (the eq. (11) iterate);
    the others keep theirs.  Every instance converges to the plain solve's
    fixed point."""
    print("[case] judged iterate, worse starts restart", flush=True)
    probs = [W.c1(33), W.c2(65), W.c4_instance(2, n_max=100), W.c4_instance(5, n_max=140)]
    s = solver(probs, precision="fp64", theta=1.0, dt=0.05)
    off = [int(v) for v in s.layout()]
    g = torch.zeros(off[-1], dtype=torch.float64, device="cuda")
    s.initial_guess(g)
    ref = g.clone()
    s.split_iterate(ref, 3000, 1e-13)
    u = g + 0.9 * (ref - g)  # closer than the eq. (11) iterate on every instance
    u[off[0]:off[1]] = float("nan")
    rng = np.random.default_rng(0)
    u[off[2]:off[3]] += torch.from_numpy(10.0 * rng.standard_normal(off[3] - off[2])).cuda()
    tol = 1e-10
    it, rel, st, used = s.split_iterate_judged(u, g, 3000, tol)
    torch.cuda.synchronize()
    assert list(used) == [1, 0, 1, 0]
    assert st == 0 and np.all(rel <= tol)
    assert torch.isfinite(u).all()
    a, b = u.cpu().numpy(), ref.cpu().numpy()
    for i in range(len(probs)):
        e = np.linalg.norm(a[off[i]:off[i + 1]] - b[off[i]:off[i + 1]]) / np.linalg.norm(b[off[i]:off[i + 1]])
        assert e < 100 * tol, (i, e)
    s.close()


def _bucket(nodes):
    per = (nodes + 255) // 256
    return 4 if per <= 1 else 3 if per <= 2 else 2 if per <= 4 else 1 if per <= 8 else 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_split_line_launches_equal_the_single_launch(precision):
    """One launch per length bucket (the short curves on 64- and 128-thread
    workgroups, so partitioned differently) against the single launch: a
    batch whose curves fill all five buckets reaches, with launch lists
    compacted as instances finish, the same fixed point (to rounding in FP64,
    to the FP32-lines bar with FP32 lines) in the same sweeps (+-1).  The
    graph replay (full lists) and the concurrent launches give the eager
    bucketed result bitwise."""
    print(f"[case] split line launches vs one launch ({precision})", flush=True)
    probs = [W.c2(2049), W.c4_instance(2, n_max=100), W.c1(33), W.c4_instance(7, n_max=600)]
    kw = dict(precision=precision, theta=1.0, dt=0.05)
    if precision == "fp32":
        kw["fp32_sweeps"] = 3
    one = solver(probs, **kw)
    buckets = set()
    for i in range(len(probs)):
        for fam in (0, 1):
            off, _, _ = one.export_lines(i, fam)
            buckets |= {_bucket(int(c)) for c in np.diff(off)}
    assert buckets == {0, 1, 2, 3, 4}, buckets
    spl = solver(probs, split_lines=True, **kw)
    off = spl.layout()
    tol = 1e-9
    u1 = torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda")
    u2 = torch.zeros_like(u1)
    it1, rel1, st1 = one.split_iterate(u1, 3000, tol)
    it2, rel2, st2 = spl.split_iterate(u2, 3000, tol)
    torch.cuda.synchronize()
    assert st1 == 0 and st2 == 0
    assert len(set(int(v) for v in it2)) > 1  # compaction took place
    assert np.all(np.abs(it1.astype(int) - it2.astype(int)) <= 1)
    d = float(torch.max(torch.abs(u1 - u2)) / torch.max(torch.abs(u1)))
    print(f"[case] max relative difference {d:.2e} (bitwise: {bool(torch.equal(u1, u2))})", flush=True)
    assert d <= (1e-11 if precision == "fp64" else 1e-6)
    spl_g = solver(probs, split_lines=True, graph=True, **kw)
    u3 = torch.zeros_like(u1)
    it3, _, st3 = spl_g.split_iterate(u3, 3000, tol)
    torch.cuda.synchronize()
    assert st3 == 0 and np.array_equal(it3, it2)
    assert torch.equal(u3, u2)
    # the same launches on three streams at once (forked and joined by events)
    conc = solver(probs, split_lines=2, **kw)
    for rep in range(2):
        u4 = torch.zeros_like(u1)
        it4, _, st4 = conc.split_iterate(u4, 3000, tol)
        torch.cuda.synchronize()
        assert st4 == 0 and np.array_equal(it4, it2)
        assert torch.equal(u4, u2), rep
    # the 512-thread shapes of the buckets of long curves (6, 4 and 2 rows per thread)
    wide = solver(probs, split_lines=True, **kw)
    wide.set_line_shapes((1, 1, 2, 0, 0))
    u5 = torch.zeros_like(u1)
    it5, _, st5 = wide.split_iterate(u5, 3000, tol)
    torch.cuda.synchronize()
    d5 = float(torch.max(torch.abs(u5 - u2)) / torch.max(torch.abs(u2)))
    print(f"[case] 512-thread shapes: max relative difference {d5:.2e}", flush=True)
    assert st5 == 0 and np.all(np.abs(it5.astype(int) - it2.astype(int)) <= 1)
    assert d5 <= (1e-11 if precision == "fp64" else 1e-6)
    for s in (one, spl, spl_g, conc, wide):
        s.close()


def test_copy_probe_copies():
    """The measurement copy (the bench's measured HBM bandwidth) copies exactly,
    including a size that is not a multiple of the workgroup; bad sizes are
    rejected."""
    print("[case] copy probe", flush=True)
    from paper_2411_11041_amd.adr import copy_probe, ADRError
    a = torch.randn(1000003 * 4, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    copy_probe(a, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    with pytest.raises(ADRError):
        copy_probe(a[:5], torch.zeros(5, dtype=torch.float32, device="cuda"))  # 20 bytes: not a multiple of 16


def test_adaptive_schedule_graph_replay_equals_eager():
    """The adaptive schedule replayed from per-block-length graphs (full launch
    lists, finished instances exiting at once) gives the eager solve's result
    (compacted lists) bitwise, with the same sweep counts, on every replay with
    eager work in between."""
    print("[case] adaptive schedule: graph replay vs eager, batch of 6", flush=True)
    probs = [W.c4_instance(i, n_max=70) for i in range(6)]
    kw = dict(precision="fp32", fp32_sweeps=8, adaptive=True, split_lines=1, theta=1.0, dt=0.05)
    eager = solver(probs, **kw)
    graph = solver(probs, graph=True, **kw)
    n = int(eager.layout()[-1])
    ref = torch.zeros(n, dtype=torch.float64, device="cuda")
    it_e, rel_e, _ = eager.split_iterate(ref, 2000, 1e-9)
    torch.cuda.synchronize()
    assert len(set(int(v) for v in it_e)) > 1  # instances stop at different sweeps
    u = torch.zeros_like(ref)
    for rep in range(3):
        u.zero_()
        it_g, rel_g, _ = graph.split_iterate(u, 2000, 1e-9)
        torch.cuda.synchronize()
        assert np.array_equal(it_g, it_e), rep
        assert torch.equal(u, ref), rep
        graph.residual(u)  # eager work on the same context between replays
    # switching the mode on a context keeps the result
    eager.set_graph(True)
    v = torch.zeros_like(ref)
    eager.split_iterate(v, 2000, 1e-9)
    torch.cuda.synchronize()
    assert torch.equal(v, ref)
    eager.close()
    graph.close()
