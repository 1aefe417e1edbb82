"""Full-size (2049 x 2049) parity in the benchmark's launch configuration,
against oracle values stored by tests/golden/make_c2_full.py at 2000 seeded
interior nodes (the oracle needs minutes at this size)."""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_2049_samples.json")


@pytest.fixture(scope="module")
def golden():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with open(GOLDEN) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def problem():
    return W.c2(2049)


def test_c2_full_fp64_three_sweeps(golden, problem):
    print("[case] c2 2049 fp64 3 sweeps vs stored oracle samples", flush=True)
    from paper_2411_11041_amd.adr import Solver
    s = Solver(problem, precision="fp64", theta=1.0, dt=0.05)
    u = torch.zeros(problem.nx * problem.ny, dtype=torch.float64, device="cuda")
    s.split_iterate(u, 3, 0.0)
    torch.cuda.synchronize()
    idx = np.array(golden["nodes"])
    got = u.cpu().numpy()[idx]
    ref = np.array(golden["after3"])
    assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))
    # the FP64 residual measure agrees with the oracle's
    r = s.residual(u)
    assert abs(r[0] - golden["rel_after3"]) <= 1e-10 * golden["rel_after3"]
    assert abs(float(torch.linalg.norm(u)) - golden["after3_norm"]) <= 1e-11 * golden["after3_norm"]
    s.close()


def test_c2_full_fp32_lines_bench_configuration(golden, problem):
    """FP32 line solves, 3 FP32 sweeps per FP64 sweep, tol 1e-8: the converged
    iterate matches the oracle's fixed point within 1e-5 relative L2."""
    print("[case] c2 2049 fp32 lines to 1e-8 vs stored oracle fixed point", flush=True)
    from paper_2411_11041_amd.adr import Solver
    s = Solver(problem, precision="fp32", fp32_sweeps=3, theta=1.0, dt=0.05)
    u = torch.zeros(problem.nx * problem.ny, dtype=torch.float64, device="cuda")
    iters, rel, st = s.split_iterate(u, 5000, 1e-8)
    assert st == 0 and rel[0] <= 1e-8
    idx = np.array(golden["nodes"])
    got = u.cpu().numpy()[idx]
    ref = np.array(golden["fixed_point"])
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
    full = float(torch.linalg.norm(u))
    assert abs(full - golden["fixed_point_norm"]) <= 1e-5 * golden["fixed_point_norm"]
    s.close()
