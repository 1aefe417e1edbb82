"""Learned warm start on the GPU: dataset generation with the splitting solver,
training with the matrix-core kernels, and the warm-started solve.

What is asserted is what holds for any trained network: training lowers the
loss; the solve started from the network's prediction converges to the same
fixed point as the solve from zero (within the bound that the stopping test
implies); a corrupted network falls back to the eq. (11) iterate.  The sweep
counts of the three starts are printed (the gain is measured, not assumed).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N_GRID = 129
TRAIN = list(range(0, 256))
TEST = list(range(20000, 20016))


@pytest.fixture(scope="module", params=[1, 4], ids=["fine", "coarse4"])
def trained(request):
    """The network on the 129^2 grid itself, and on every 4th node (33^2)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_11041_amd import warmstart as WS
    from paper_2411_11041_amd.adr import Net
    r = request.param
    print(f"[case] warm start: generate 256 samples 129^2, network grid every {r} nodes, train 12 epochs",
          flush=True)
    wl = WS.Workload(n=N_GRID, batch=64, coarsen=r)
    net = Net(*wl.coarse_shape(), 64)
    net.set_params(WS.he_init(0))
    x, t = wl.generate(net, TRAIN, tol=1e-10)
    losses = WS.train(net, x, t, wl.mask_c, len(TRAIN), wl.HWc, 12, batch=32, lr=2e-3, lr_end=1e-4)
    yield wl, net, losses
    net.close()
    wl.solver.close()


def test_training_lowers_loss(trained):
    _, _, losses = trained
    print("[case] losses", [f"{v:.2e}" for v in losses], flush=True)
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0]


def test_warm_started_solve_reaches_the_same_fixed_point(trained):
    wl, net, _ = trained
    tol = 1e-10
    u0, it0, rel0, t0 = wl.solve_batch(TEST, tol)
    us, its, rels, ts, _ = wl.warm_started(net, TEST, tol, use_net=False)
    un, itn, reln, tn, fb = wl.warm_started(net, TEST, tol, use_net=True)
    print(f"[case] sweeps to {tol:g}: zero {it0.mean():.1f}, eq. (11) {its.mean():.1f}, "
          f"network {itn.mean():.1f} (fallbacks {fb})", flush=True)
    assert np.all(rel0 <= tol) and np.all(rels <= tol) and np.all(reln <= tol)
    HW = wl.HW
    a = u0.view(len(TEST), HW).cpu().numpy()
    for u in (us, un):
        b = u.view(len(TEST), HW).cpu().numpy()
        # contraction ~0.75 per sweep: the stopped iterate is within a few
        # tol * |Phi(0)| of the fixed point; 100 tol relative is a safe bound
        err = np.linalg.norm(a - b, axis=1) / np.linalg.norm(a, axis=1)
        assert np.all(err < 100 * tol), err.max()


def test_network_start_is_closer_than_zero(trained):
    """The prediction itself (before any sweep) is closer to the converged
    solution than the zero start."""
    wl, net, _ = trained
    u_ref, _, _, _ = wl.solve_batch(TEST, 1e-12)
    probs = wl.problems(TEST)
    s = wl._bind(probs)
    B = len(TEST)
    g = torch.zeros(B * wl.HW, dtype=torch.float64, device="cuda")
    s.initial_guess(g)
    x0, _, sn = wl._net_inputs(net, B, wl.f_tensor(probs), g, [p.mu for p in probs])
    out = net.forward(B, x0)
    u = torch.empty_like(g)
    if wl.r > 1:
        net.warm_start_prolong(B, wl.r, g, sn, out, wl.mask, u)
    else:
        net.warm_start(B, g, sn, out, wl.mask, u)
    e_net = float(torch.linalg.norm(u - u_ref) / torch.linalg.norm(u_ref))
    e_s = float(torch.linalg.norm(g - u_ref) / torch.linalg.norm(u_ref))
    print(f"[case] relative L2 error of the start: eq. (11) {e_s:.3e}, network {e_net:.3e}", flush=True)
    assert e_net < 1.0


def test_corrupted_network_falls_back(trained):
    wl, net, _ = trained
    good = net.get_params()
    try:
        bad = good.copy()
        bad[:] = np.nan
        net.set_params(bad)
        u, it, rel, _, fb = wl.warm_started(net, TEST[:4], 1e-8)
        print(f"[case] NaN network: fallbacks {fb}", flush=True)
        assert fb == 4
        assert np.all(rel <= 1e-8) and torch.isfinite(u).all()
    finally:
        net.set_params(good)


def test_trained_network_gains_over_the_method_without_it():
    """What the learned warm start gains, on held-out seeds at the warm-start
    configuration's shape (257^2, the network on every 8th node): after
    training on 8 192 method-generated solutions, the network's start is closer
    to the fixed point than the eq. (11) iterate, and the judged solve from it
    needs fewer sweeps on average than the solve from zero and the solve from
    the eq. (11) iterate, all to the same fixed point."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_11041_amd import warmstart as WS
    from paper_2411_11041_amd.adr import Net
    print("[case] warm-start gain: 257^2, network on 33^2, train 8192 x 400, 64 held-out seeds", flush=True)
    wl = WS.Workload(n=257, batch=128, coarsen=8)
    net = Net(*wl.coarse_shape(), 128)
    net.set_params(WS.he_init(0))
    x, t = wl.generate(net, list(range(8192)), tol=1e-10)
    WS.train(net, x, t, wl.mask_c, 8192, wl.HWc, 400, batch=32, lr=2e-3, lr_end=2e-5)
    del x, t
    test = list(range(20000, 20064))
    tol = 1e-8
    u0, it0, rel0, _ = wl.solve_batch(test, tol)
    us, its, rels, _, _ = wl.warm_started(net, test, tol, use_net=False)
    un, itn, reln, _, fb = wl.warm_started(net, test, tol, use_net=True)
    # distance of the starts from the fixed point (network start vs eq. (11))
    u_ref, _, _, _ = wl.solve_batch(test, 1e-12)
    probs = wl.problems(test)
    s = wl._bind(probs)
    g = torch.zeros(len(test) * wl.HW, dtype=torch.float64, device="cuda")
    s.initial_guess(g)
    x0, _, sn = wl._net_inputs(net, len(test), wl.f_tensor(probs), g, [p.mu for p in probs])
    out = net.forward(len(test), x0)
    ustart = torch.empty_like(g)
    net.warm_start_prolong(len(test), wl.r, g, sn, out, wl.mask, ustart)
    e_net = float(torch.linalg.norm(ustart - u_ref) / torch.linalg.norm(u_ref))
    e_s = float(torch.linalg.norm(g - u_ref) / torch.linalg.norm(u_ref))
    print(f"[case] start error: eq. (11) {e_s:.3e}, network {e_net:.3e}; mean sweeps to {tol:g}: "
          f"zero {it0.mean():.2f}, eq. (11) {its.mean():.2f}, network {itn.mean():.2f} (fallbacks {fb})",
          flush=True)
    assert np.all(rel0 <= tol) and np.all(rels <= tol) and np.all(reln <= tol)
    assert e_net < e_s
    assert itn.mean() < its.mean() < it0.mean()
    net.close()
    wl.solver.close()
