"""GMRES(m) acceleration of the stationary solve (options.krylov) on the HIP
path: the same fixed point as the plain iteration (the oracle's dense LU and
its converged iteration), in about the sweep count of the oracle's GMRES."""
import numpy as np
import pytest

import workloads as W
from oracle import dense, krylov
from oracle.method import Oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


def rel_l2(a, b, idx):
    return float(np.linalg.norm(a[idx] - b[idx]) / np.linalg.norm(b[idx]))


def solver(p, **kw):
    from paper_2411_11041_amd.adr import Solver
    return Solver(p, **kw)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gmres_reaches_the_dense_fixed_point(prec):
    print(f"[case] gmres(10) c1 33 ({prec} context) vs dense fixed point", flush=True)
    p = W.c1(33)
    o = Oracle(p)
    Ud = dense.fixed_point(o, 1.0, 0.05)
    s = solver(p, precision=prec, theta=1.0, dt=0.05, krylov=10)
    u = dev(o.zero_field())
    it, rel, st = s.split_iterate(u, 500, 1e-12)
    assert st == 0 and rel[0] <= 1e-12
    assert rel_l2(u.cpu().numpy(), Ud, o.inner_idx) < 1e-10
    _, n_or, _ = krylov.solve_fixed_point(o, 1.0, 0.05, 1e-12, restart=10)
    _, it_plain, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 5000, 1e-12)
    print(f"[case] sweeps: gpu gmres {int(it[0])}, oracle gmres {n_or}, plain {it_plain}", flush=True)
    assert abs(int(it[0]) - n_or) <= 3
    assert int(it[0]) < it_plain
    s.close()


def test_gmres_batch_with_dirichlet_data():
    """Instances converge on their own Krylov spaces in one batch (box, disc,
    L-shape, non-zero g)."""
    print("[case] gmres(15) batch box/disc/L with g vs oracle fixed points", flush=True)
    probs = [W.c2(65), W.c4_instance(0, n_max=90), W.c4_instance(1, n_max=90)]
    for p in probs:
        X, Y = p.coords()
        p.g = 0.3 * np.sin(2 * X) - 0.2 * Y
    orcs = [Oracle(p) for p in probs]
    s = solver(probs, precision="fp64", theta=1.0, dt=0.05, krylov=15)
    off = s.layout()
    u = dev(np.concatenate([o.zero_field() for o in orcs]))
    it, rel, st = s.split_iterate(u, 800, 1e-11)
    assert st == 0 and np.all(rel <= 1e-11)
    got = u.cpu().numpy()
    plain = solver(probs, precision="fp64", theta=1.0, dt=0.05)
    v = dev(np.concatenate([o.zero_field() for o in orcs]))
    it_p, _, _ = plain.split_iterate(v, 3000, 1e-11)
    for i, o in enumerate(orcs):
        Uo, _, _, _ = o.iterate(o.zero_field(), 1.0, 0.05, 5000, 1e-13)
        assert rel_l2(got[off[i]:off[i + 1]], Uo, o.inner_idx) < 1e-9, i
    print(f"[case] sweeps gmres {list(it)}, plain {list(it_p)}", flush=True)
    assert np.all(it < it_p)
    s.close()
    plain.close()
