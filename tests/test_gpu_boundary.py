"""The boundary of the problem statement on the HIP path, against the oracle:
Dirichlet data g on Gamma, beta from a stream function, the singular-pivot
flag, and implicit Euler steps iterated to convergence."""
import numpy as np
import pytest

import workloads as W
from oracle.method import Oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


def rel_l2(a, b, idx):
    return float(np.linalg.norm(a[idx] - b[idx]) / max(np.linalg.norm(b[idx]), 1e-300))


def solver(p, **kw):
    from paper_2411_11041_amd.adr import Solver
    return Solver(p, **kw)


def with_g(p, kind="smooth"):
    X, Y = p.coords()
    p.g = np.sin(3 * X) + Y ** 2 - 0.5 if kind == "smooth" else 0.2 + X - 0.5 * Y
    return p


def _affine(kind, n, beta):
    a, b, c, mu, sigma = 0.7, -1.3, 0.4, 0.05, 2.0
    p = W.constant_beta(n, mu, sigma, beta, f=0.0)
    X, Y = p.coords()
    u = a + b * X + c * Y
    p.f = beta[0] * b + beta[1] * c + sigma * u
    p.g = u.copy()
    if kind == "disc":
        p.domain, p.dom_params = W.DOM_DISC, (0.5, 0.5, 0.45)
    elif kind == "L":
        p.domain, p.dom_params = W.DOM_POLYGON, W.L_SHAPE
    return p, u.ravel()


@pytest.mark.parametrize("sweeps", [1, 4, 12])
def test_dirichlet_fp64_sweeps_match_oracle(sweeps):
    """A box, a disc and an L-shape with non-zero g in one batch, FP64 sweep by sweep."""
    print(f"[case] dirichlet g, batch box/disc/L, fp64 sweeps={sweeps}", flush=True)
    probs = [with_g(W.c1(65)), with_g(W.c4_instance(0, n_max=90)), with_g(W.c4_instance(1, n_max=90))]
    s = solver(probs, precision="fp64", theta=1.0, dt=0.05)
    off = s.layout()
    orcs = [Oracle(p) for p in probs]
    u0 = np.concatenate([o.zero_field() for o in orcs])
    u = dev(u0)
    iters, rel, st = s.split_iterate(u, sweeps, 0.0)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    for i, o in enumerate(orcs):
        U = o.zero_field()
        for _ in range(sweeps):
            U = o.step(U, 1.0, 0.05)
        assert iters[i] == sweeps
        assert rel_l2(got[off[i]:off[i + 1]], U, o.inner_idx) < 1e-11, i
    s.close()


def test_dirichlet_fp32_lines_converged():
    print("[case] dirichlet g, c2 129 fp32 lines converged", flush=True)
    p = with_g(W.c2(129))
    o = Oracle(p)
    s = solver(p, precision="fp32", fp32_sweeps=3, theta=1.0, dt=0.05)
    u = dev(o.zero_field())
    iters, rel, st = s.split_iterate(u, 3000, 1e-10)
    assert st == 0 and rel[0] <= 1e-10
    Uo, _, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 3000, 1e-12)
    assert rel_l2(u.cpu().numpy(), Uo, o.inner_idx) < 1e-5
    s.close()


@pytest.mark.parametrize("kind,beta", [("box", (1.0, 0.5)), ("disc", (0.6, -1.1)), ("L", (-0.8, 0.3))])
def test_dirichlet_affine_solution_on_gpu(kind, beta):
    """The affine solution with g = u on Gamma is the method's exact fixed point
    (a closed form, independent of the oracle); eq. (11) returns it too."""
    print(f"[case] affine exact solution, {kind}", flush=True)
    p, uex = _affine(kind, 49, beta)
    o = Oracle(p)
    s = solver(p, precision="fp64", theta=1.0, dt=0.05)
    u = dev(o.zero_field())
    iters, rel, st = s.split_iterate(u, 4000, 1e-13)
    assert st == 0
    m = o.inner_idx
    assert np.max(np.abs(u.cpu().numpy()[m] - uex[m])) < 1e-9
    g0 = dev(o.zero_field())
    s.initial_guess(g0)
    torch.cuda.synchronize()
    assert np.max(np.abs(g0.cpu().numpy()[m] - uex[m])) < 1e-11
    s.close()


def test_dirichlet_initial_guess_and_march():
    print("[case] dirichlet g, eq. (11) and theta = 1/2 march", flush=True)
    p = with_g(W.data2d(41))
    o = Oracle(p)
    s = solver(p, precision="fp64")
    u = dev(o.zero_field())
    s.initial_guess(u)
    torch.cuda.synchronize()
    U0 = o.s_guess()
    assert rel_l2(u.cpu().numpy(), U0, o.inner_idx) < 1e-12
    s.time_step(u, 0.5, 0.001, 20)
    torch.cuda.synchronize()
    U = o.march(U0, 0.5, 0.001, 20)
    assert rel_l2(u.cpu().numpy(), U, o.inner_idx) < 1e-11
    s.close()


def test_beta_from_stream_function():
    """beta1 = beta2 = NULL: the library differentiates psi (second order)."""
    print("[case] c2 129 from psi, fp64 3 sweeps", flush=True)
    p = W.c2(129)
    p.beta1 = p.beta2 = None
    o = Oracle(p)
    s = solver(p, precision="fp64", theta=1.0, dt=0.05)
    u = dev(o.zero_field())
    s.split_iterate(u, 3, 0.0)
    torch.cuda.synchronize()
    U = o.zero_field()
    for _ in range(3):
        U = o.step(U, 1.0, 0.05)
    assert rel_l2(u.cpu().numpy(), U, o.inner_idx) < 1e-11
    s.close()


def test_singular_pivot_flag_forced_from_the_host():
    """A pivot threshold above every pivot's scale (set by the host) makes every
    line solve flag its instance: the solve and the residual return
    ADR_ESINGULAR; the default threshold flags nothing on the same problem."""
    from paper_2411_11041_amd.adr import ADRError, ADR_ESINGULAR
    print("[case] singular flag forced by pivot_tol", flush=True)
    probs = [W.c4_instance(0, n_max=60), W.c4_instance(1, n_max=60)]
    for prec in ("fp64", "fp32"):
        s = solver(probs, precision=prec, fp32_sweeps=3, pivot_tol=10.0)
        u = torch.zeros(int(s.layout()[-1]), dtype=torch.float64, device="cuda")
        with pytest.raises(ADRError) as e:
            s.split_iterate(u, 5, 0.0)
        assert e.value.code == ADR_ESINGULAR and "2 instance" in str(e.value)
        with pytest.raises(ADRError) as e:
            s.residual(u)
        assert e.value.code == ADR_ESINGULAR
        s.close()
        s = solver(probs, precision=prec, fp32_sweeps=3)
        it, rel, st = s.split_iterate(u, 5, 0.0)  # no flag: tol 0 ends at max_iters (ADR_ENOTCONV)
        assert st == 1 and np.all(np.isfinite(rel))
        s.close()


def test_converged_time_steps_match_oracle():
    """Implicit Euler steps iterated to convergence (the stationary iteration on
    each step's problem): FP64 with a fixed sweep count per step (tol 0) is
    compared sweep for sweep; to a tolerance, the counts agree within one and
    the march within the tolerance.  The stationary solve is unchanged after."""
    print("[case] c3 65 converged implicit Euler, 4 steps", flush=True)
    p = with_g(W.c3(65))
    o = Oracle(p)
    s = solver(p, precision="fp64", theta=1.0, dt=0.05)
    u0 = o.with_boundary(p.u0.ravel() * o.mask.ravel())
    m = o.inner_idx
    u = dev(u0)
    it, st = s.time_step(u, 1.0, 0.005, 4, inner_max=6, inner_tol=0.0)
    torch.cuda.synchronize()
    assert (it == 6).all() and st == 1  # ADR_ENOTCONV: every step stopped at inner_max
    U = o.with_boundary(u0)
    for _ in range(4):
        S, L = o.step_operators(U, 0.005)
        for _ in range(6):
            U = o.step(U, 1.0, 0.05, S=S, L=L)
    assert rel_l2(u.cpu().numpy(), U, m) < 1e-11
    u = dev(u0)
    it, st = s.time_step(u, 1.0, 0.005, 4, inner_max=500, inner_tol=1e-11)
    Uo, cnt = o.march_converged(u0, 0.005, 4, 0.05, 1e-11, 500)
    assert st == 0 and np.all(np.abs(it[:, 0] - np.array(cnt)) <= 1)
    assert rel_l2(u.cpu().numpy(), Uo, m) < 1e-9
    # the stationary coefficients, loads and |Phi(0)| are restored
    a = dev(o.zero_field())
    s.split_iterate(a, 3, 0.0)
    Us = o.zero_field()
    for _ in range(3):
        Us = o.step(Us, 1.0, 0.05)
    assert rel_l2(a.cpu().numpy(), Us, m) < 1e-11
    s.close()


def test_converged_time_steps_fp32_lines():
    print("[case] c3 129 converged implicit Euler, fp32 lines, 3 steps", flush=True)
    p = W.c3(129)
    o = Oracle(p)
    s = solver(p, precision="fp32", fp32_sweeps=3, theta=1.0, dt=0.05)
    u0 = p.u0.ravel() * o.mask.ravel()
    u = dev(u0)
    it, st = s.time_step(u, 1.0, 0.005, 3, inner_max=500, inner_tol=1e-10)
    assert st == 0
    Uo, cnt = o.march_converged(u0, 0.005, 3, 0.05, 1e-12, 500)
    assert rel_l2(u.cpu().numpy(), Uo, o.inner_idx) < 1e-5
    s.close()


@pytest.mark.parametrize("name,theta,dt,steps", [("data2d_61", 0.5, 0.001, 30), ("c3_129", 1.0, 0.005, 10)])
def test_strang_march_matches_oracle(name, theta, dt, steps):
    """The symmetric splitting (beta dt/2, gamma dt, beta dt/2), FP64, step by step."""
    print(f"[case] strang march {name} theta={theta} {steps} steps", flush=True)
    p = W.data2d(61) if name.startswith("data2d") else with_g(W.c3(129))
    o = Oracle(p)
    s = solver(p, precision="fp64", splitting="strang")
    U0 = o.s_guess() if name.startswith("data2d") else o.with_boundary(p.u0.ravel() * o.mask.ravel())
    u = dev(U0)
    s.time_step(u, theta, dt, steps)
    torch.cuda.synchronize()
    U = o.march(U0, theta, dt, steps, strang=True)
    assert rel_l2(u.cpu().numpy(), U, o.inner_idx) < 1e-11
    # the order-of-eq.-(10) march of the same context differs (a different scheme)
    v = dev(U0)
    lie = solver(p, precision="fp64")
    lie.time_step(v, theta, dt, steps)
    torch.cuda.synchronize()
    assert rel_l2(v.cpu().numpy(), U, o.inner_idx) > 1e-6
    s.close()
    lie.close()


def test_fitted_lines_match_oracle():
    """Exponentially fitted beta-lines (options.stabilize): FP64 sweeps and the
    eq. (11) s-solve of an advection-dominated batch (a coarse high-Peclet box
    and a disc with mu ~ 1e-4), and the FP32-lines fixed point."""
    print("[case] fitted beta-lines vs oracle", flush=True)
    box = W.constant_beta(33, 2e-4, 1.0, (1.0, 0.4), f=1.0)
    disc = W.c4_instance(0, n_max=70)
    probs = [box, disc]
    orcs = [Oracle(p, stabilize=True) for p in probs]
    s = solver(probs, precision="fp64", theta=1.0, dt=0.05, stabilize=True)
    off = s.layout()
    u = dev(np.concatenate([o.zero_field() for o in orcs]))
    s.split_iterate(u, 5, 0.0)
    g = dev(np.concatenate([o.zero_field() for o in orcs]))
    s.initial_guess(g)
    torch.cuda.synchronize()
    got, gg = u.cpu().numpy(), g.cpu().numpy()
    for i, o in enumerate(orcs):
        U = o.zero_field()
        for _ in range(5):
            U = o.step(U, 1.0, 0.05)
        assert rel_l2(got[off[i]:off[i + 1]], U, o.inner_idx) < 1e-11, i
        assert rel_l2(gg[off[i]:off[i + 1]], o.s_guess(), o.inner_idx) < 1e-12, i
    assert gg[off[0]:off[1]][orcs[0].inner_idx].min() >= 0.0  # no undershoot (Galerkin: < -0.1)
    s.close()
    s = solver(probs, precision="fp32", fp32_sweeps=3, theta=1.0, dt=0.05, stabilize=True)
    u = dev(np.concatenate([o.zero_field() for o in orcs]))
    it, rel, st = s.split_iterate(u, 3000, 1e-10)
    assert st == 0
    got = u.cpu().numpy()
    for i, o in enumerate(orcs):
        Uo, _, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 3000, 1e-12)
        assert rel_l2(got[off[i]:off[i + 1]], Uo, o.inner_idx) < 1e-5, i
    s.close()
