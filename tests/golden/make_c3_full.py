"""Writes c3_2049_samples.json: oracle values of the full 2049 x 2049
parabolic problem (implicit Euler, theta = 1, dt = 0.005, one eq. (10) step per
time step from the Gaussian bump) at 2000 seeded interior nodes after 10 and
after 200 steps.  Calls only the oracle and the input generators.  ~2 min on
one core.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle.method import Oracle  # noqa: E402


def main():
    t0 = time.time()
    p = W.c3(2049)
    th, dt, steps = p.extra["theta"], p.extra["dt"], p.extra["steps"]
    o = Oracle(p)
    rng = np.random.default_rng(20241203)
    idx = np.sort(rng.choice(o.inner_idx, size=2000, replace=False))
    U = np.asarray(p.u0, float).ravel().copy()
    U10 = o.march(U, th, dt, 10)
    U200 = o.march(U10, th, dt, steps - 10)
    out = dict(problem=f"c3 2049x2049, theta={th}, dt={dt}", nodes=idx.tolist(),
               after10=U10[idx].tolist(), after200=U200[idx].tolist(),
               max10=float(np.abs(U10).max()), max200=float(np.abs(U200).max()),
               seconds=time.time() - t0)
    with open(os.path.join(HERE, "c3_2049_samples.json"), "w") as fh:
        json.dump(out, fh)
    print("wrote", len(idx), "samples in", round(time.time() - t0), "s; max after 200 steps", out["max200"])


if __name__ == "__main__":
    main()
