"""Writes c2_2049_samples.json: oracle values of the full 2049 x 2049
advection-dominated problem at 2000 seeded interior nodes, (a) after 3 FP64
sweeps from zero and (b) at the stationary fixed point (relative update
<= 1e-11).  Calls only the oracle and the input generators.  ~3 min on one core.
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
    p = W.c2(2049)
    o = Oracle(p)
    rng = np.random.default_rng(20241117)
    idx = np.sort(rng.choice(o.inner_idx, size=2000, replace=False))
    U = o.zero_field()
    for _ in range(3):
        U = o.step(U, 1.0, 0.05)
    s3 = U[idx].tolist()
    r3 = o.rel_residual(U, 1.0, 0.05)
    Uc, it, rel, _ = o.iterate(U, 1.0, 0.05, 400, 1e-11)
    out = dict(problem="c2 2049x2049, theta=1, dt=0.05", nodes=idx.tolist(),
               after3=s3, rel_after3=r3, fixed_point=Uc[idx].tolist(),
               fixed_point_sweeps=3 + it, fixed_point_rel=rel,
               fixed_point_norm=float(np.linalg.norm(Uc[o.inner_idx])),
               after3_norm=float(np.linalg.norm(U[o.inner_idx])),
               seconds=time.time() - t0)
    with open(os.path.join(HERE, "c2_2049_samples.json"), "w") as fh:
        json.dump(out, fh)
    print("wrote", len(idx), "samples in", round(time.time() - t0), "s; sweeps", 3 + it, "rel", rel)


if __name__ == "__main__":
    main()
