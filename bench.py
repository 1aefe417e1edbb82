"""Benchmark of the directional diffusion splitting hot path on one MI355X.

Step = one stationary solve (eq. (10) sweeps to the fixed point, Sec. 2 limit)
of the advection-dominated 2049 x 2049 problem from zero to a relative
fixed-point residual of 1e-8, FP32 line solves with FP64 state, residual and
convergence test.  value = line unknowns solved per second (every sweep solves
one tridiagonal system per curve of both families); ms_per_step is the
time to the 1e-8 residual.  Inputs are resident in device memory before the
timed region; set-up (curve tracing, tables, upload) is outside it.

Extra fields: the dominant kernel's roofline (HIP-event durations measured in
the timed region, algorithmic bytes from the line/grid counts) and the FP64
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "line-unknowns/s + time-to-1e-8 residual: plain vs batched/warm-start, 1 GPU"
HBM_PEAK_GBS = 8000.0

# Algorithmic (compulsory) bytes per line unknown of one line-solve pass: node
# geometry read once (cell index 4 B, two cell offsets, chord; beta family also
# |beta| and the load), the gathered field value (each grid value is read by
# about one line node) and the written line value.
LINE_BYTES = {("fp32", 0): 4 + 4 * 2 + 4 + 4 + 4 + 4 + 4, ("fp32", 1): 4 + 4 * 2 + 4 + 4 + 4,
              ("fp64", 0): 4 + 8 * 2 + 8 + 8 + 8 + 8 + 8, ("fp64", 1): 4 + 8 * 2 + 8 + 8 + 8}
# Scatter: per interior grid node its grid index (4 B), its 4 records (the
# first record's line node 4 B and three 16-bit offsets 6 B; two weights per
# record: FP16 pair in the FP32 sweeps, 2 x FP64 in the FP64 sweeps), the 8
# line values they reference (each line value is referenced by ~2 nodes: 4 per
# node) and the written grid value (FP64 update: read+write state, write the
# FP32 increment).  Keys: (precision, 2) beta half sweep, (precision, 3) gamma
# half sweep.
SCATTER_BYTES = {("fp32", 2): 4 + 10 + 4 * 4 + 4 * 4 + 4, ("fp32", 3): 4 + 10 + 4 * 4 + 4 * 4 + 8 + 8 + 4,
                 ("fp64", 2): 4 + 10 + 4 * 16 + 4 * 8 + 8, ("fp64", 3): 4 + 10 + 4 * 16 + 4 * 8 + 8 + 8 + 4}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2049, help="grid nodes per side")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--fp32-sweeps", type=int, default=3)
    ap.add_argument("--adaptive", action="store_true",
                    help="c2/c4 with --no-autotune: adaptive schedule with at most --fp32-sweeps FP32 sweeps per FP64 sweep")
    ap.add_argument("--split-lines", type=int, choices=[0, 1, 2], default=0,
                    help="c2/c4 with --no-autotune (and c3): line-solve launches, 0 one per family, 1 one per "
                         "length bucket, 2 one per length bucket on concurrent streams")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sweeps", type=int, default=12)
    ap.add_argument("--workload", choices=["c2", "c3", "c4", "c5"], default="c2",
                    help="c2: one 2049^2 problem (default); c3: the 2049^2 parabolic march (200 steps); "
                         "c4: the 512-instance batch; "
                         "c5: learned warm start (train, then zero / eq. (11) / network starts)")
    ap.add_argument("--train", type=int, default=8192, help="c5: training samples")
    ap.add_argument("--epochs", type=int, default=400, help="c5: training epochs")
    ap.add_argument("--coarsen", type=int, default=8,
                    help="c5: the network runs on every coarsen-th node (1: on the 257x257 grid itself)")
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--graph", action="store_true", help="replay sweep blocks from a HIP graph")
    ap.add_argument("--no-autotune", action="store_true",
                    help="c2/c4: keep --fp32-sweeps instead of choosing it with adr_autotune (before the timed region)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="before the timed region, run one plain elementwise copy of 256 MiB in / 256 MiB out, "
                         "the reference dispatch for scaling hardware byte counters")
    return ap.parse_args()


def gen_c4(n_inst):
    from concurrent.futures import ThreadPoolExecutor
    import workloads as W
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(W.c4_instance, range(n_inst)))


def bench_c4(args):
    """Batched workload: every instance of the batch in one launch per kernel."""
    import numpy as np
    import torch
    from paper_2411_11041_amd.adr import Solver
    t0 = time.time()
    probs = gen_c4(args.instances)
    gen_s = time.time() - t0
    t0 = time.time()
    s = Solver(probs, precision="fp32", fp32_sweeps=args.fp32_sweeps, theta=1.0, dt=0.05, graph=args.graph,
               adaptive=args.adaptive, split_lines=args.split_lines)
    setup_s = time.time() - t0
    counts = s.counts()
    per_inst = []
    for i in range(len(probs)):
        lu = 0
        for f in (0, 1):
            off, x, _ = s.export_lines(i, f)
            lu += len(x) - 2 * (len(off) - 1)
        per_inst.append(lu)
    per_inst = np.array(per_inst, np.int64)
    off = s.layout()
    u = torch.zeros(int(off[-1]), dtype=torch.float64, device="cuda")
    tuned = None
    if not args.no_autotune:
        tuned = s.autotune(u, 3000, args.tol)

    def solve():
        u.zero_()
        return s.split_iterate(u, 3000, args.tol)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = None
    for _ in range(args.steps):
        its, rel, st = solve()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    el_ev, times = events_pass(s, solve, args.steps)  # eager launches with events
    solved = int((its.astype(np.int64) * per_inst).sum()) * args.steps
    out = {"metric": METRIC, "value": solved / el, "unit": "line-unknowns/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 line solves, f64 state/residual", "data": "synthetic",
           "config": {"workload": f"c4: {len(probs)} stationary instances (disc/L-shape, 33..1025 per side, "
                                  "mu logU[1e-4,1e-1], sigma U[0.1,10], random divergence-free beta), "
                                  "one launch per kernel for the batch, to 1e-8 per instance",
                      "time_to_1e-8_ms": 1e3 * el / args.steps, "grid_unknowns": counts["grid_unknowns"],
                      "line_unknowns_per_sweep": int(per_inst.sum()), "lines": [counts["lines_b"], counts["lines_g"]],
                      "sweeps_min_median_max": [int(its.min()), int(np.median(its)), int(its.max())],
                      "converged": int((rel <= args.tol).sum()), "gen_s": round(gen_s, 1), "setup_s": round(setup_s, 1),
                      "graph": bool(args.graph),
                      "fp32_sweeps_per_fp64": tuned[0] if tuned else args.fp32_sweeps,
                      "adaptive_schedule": tuned[1] if tuned else bool(args.adaptive),
                      "line_launches": LINE_LAUNCHES[tuned[3] if tuned else args.split_lines],
                      "line_shapes": tuned[4] if tuned else [0] * 5,
                      "autotune_ms": round(tuned[2], 2) if tuned else None}}
    if True:
        out["config"]["kernels"] = {pr: {k: {"ms": round(v[0], 3), "launches": v[1]} for k, v in times[pr].items()}
                                    for pr in times}
        rf = kernel_roofline(times, counts, tuned[3] if tuned else args.split_lines)
        per_sweep_units = rf["units"]
        # every instance converges at its own sweep: the measured launches cover
        # sum_i iters_i sweeps of instance i; use the mean per launch
        frac_active = float((its.astype(np.int64) * per_inst).sum()) / max(1, int(its.max()) * int(per_inst.sum()))
        bytes_per_launch = rf["bytes_per_unit"] * per_sweep_units * frac_active
        avg_launch_s = rf["total_ms"] / rf["launches"] / 1e3
        achieved = bytes_per_launch / avg_launch_s / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": rf["kernel"],
                           "avg_launch_us": round(avg_launch_s * 1e6, 2), "bytes_per_launch": int(bytes_per_launch),
                           "note": "bytes scaled by the fraction of instance-sweeps still active",
                           "events_pass_ms_per_step": round(1e3 * el_ev / args.steps, 2)}
    print(json.dumps(out), flush=True)
    s.close()


CNN_FLOP_PER_PIXEL = 2 * 9 * (4 * 32 + 32 * 32 + 32 * 32 + 32)  # forward, 4 conv layers
MFMA_BF16_PEAK_TFS = 2500.0


def bench_c5(args):
    """Learned warm start: dataset from the solver, training, then the 64 test
    seeds solved to the tolerance from zero, from the eq. (11) iterate and from
    the network's prediction (inference and the residual-judged fallback
    inside the timed region)."""
    import numpy as np
    import torch
    from paper_2411_11041_amd import warmstart as WS
    from paper_2411_11041_amd.adr import Net
    n, B = 257, 64
    wl = WS.Workload(n=n, batch=128, coarsen=args.coarsen)
    Hc, Wc = wl.coarse_shape()
    net = Net(Hc, Wc, 128)
    net.set_params(WS.he_init(0))
    t0 = time.time()
    x, t = wl.generate(net, list(range(args.train)), tol=1e-10)
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    t0 = time.time()
    losses = WS.train(net, x, t, wl.mask_c, args.train, wl.HWc, args.epochs, batch=32, lr=2e-3, lr_end=2e-5)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    del x, t
    test = list(range(20000, 20000 + B))
    res = {}
    for name in ("zero", "eq11", "network"):
        for rep in range(args.warmup + 1):
            if name == "zero":
                u, it, rel, sec = wl.solve_batch(test, args.tol)
                fb = 0
            else:
                u, it, rel, sec, fb = wl.warm_started(net, test, args.tol, use_net=name == "network")
        res[name] = {"ms": round(sec * 1e3, 2), "sweeps_mean": round(float(it.mean()), 2), "sweeps_max": int(it.max()),
                     "converged": int((rel <= args.tol).sum()), "fallbacks": int(fb)}
    # forward pass: HIP events on the network's stream (torch's current stream)
    probs = wl.problems(test)
    s = wl._bind(probs)
    g = torch.zeros(B * wl.HW, dtype=torch.float64, device="cuda")
    s.initial_guess(g)
    x0, _, _ = wl._net_inputs(net, B, wl.f_tensor(probs), g, [p.mu for p in probs])
    out = net.forward(B, x0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        net.forward(B, x0, out)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / reps
    tflops = CNN_FLOP_PER_PIXEL * B * wl.HWc / (fwd_ms * 1e-3) / 1e12
    c = s.counts()
    per_sweep = (c["line_unknowns_b"] + c["line_unknowns_g"])
    value = per_sweep * res["network"]["sweeps_mean"] * 1.0 / (res["network"]["ms"] * 1e-3)
    outj = {"metric": METRIC, "value": value, "unit": "line-unknowns/s", "n_gpus": 1, "steps": 1,
            "warmup": args.warmup, "ms_per_step": res["network"]["ms"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 line solves, f64 state/residual; bf16 MFMA network, f32 accumulation",
            "data": "synthetic",
            "config": {"workload": f"c5: {B} test seeds, unit square {n}x{n}, sigma=1, curved stream, "
                                   "mu logU[1e-3,1e-1], 1..8 Gaussians; solved to the tolerance from three starts",
                       "tol": args.tol, "starts": res, "network_grid": f"{Hc}x{Wc} (every {args.coarsen}th node)",
                       "train_samples": args.train, "epochs": args.epochs,
                       "final_train_loss": losses[-1], "gen_s": round(gen_s, 1), "train_s": round(train_s, 1),
                       "train_samples_per_s": round(args.train * args.epochs / train_s, 1),
                       "forward_ms_batch64": round(fwd_ms, 3)},
            "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": MFMA_BF16_PEAK_TFS,
                         "unit": "TFLOP/s", "frac": round(tflops / MFMA_BF16_PEAK_TFS, 5), "traffic": None,
                         "kernel": "network forward (3 MFMA conv layers + last layer)"}}
    print(json.dumps(outj), flush=True)
    net.close()
    wl.solver.close()


def events_pass(s, solve, steps):
    """A second timed region over the same steps with per-launch HIP events on
    the library's stream (a few us between launches, so it is kept apart from
    the region that gives value); returns its seconds and the kernel times."""
    import torch
    s.kernel_times("fp64", reset=True)
    s.kernel_times("fp32", reset=True)
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        solve()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s.set_timing(False)
    times = {pr: s.kernel_times(pr, reset=True) for pr in ("fp64", "fp32")}
    return el, times


def copy_bandwidth_gbs(nbytes=1 << 30, reps=10):
    """HBM bandwidth of a plain device copy (the library's copy kernel, nbytes
    in and nbytes out, on torch's current stream), timed with events: the
    measured counterpart of the vendor peak."""
    import torch
    from paper_2411_11041_amd.adr import copy_probe
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    copy_probe(a, b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        copy_probe(a, b)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def measured_traffic(kernel, profile="c2_2049_fp32lines.md"):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when the
    summary is missing or was taken on other kernel sources."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in ("adr_kernels.hip", "adr_kernels.h"):
        with open(os.path.join(ROOT, "paper_2411_11041_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    text = open(path).read()
    if f"Kernel source sha256[:16] = {h.hexdigest()[:16]}" not in text:
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 4 and cells[0] == "adr::" + kernel:
            return float(cells[3])
    return None


def bench_c3(args):
    """Parabolic march: 200 implicit-Euler steps of eq. (10) (one splitting
    step per time step, FP64) on 2049^2 from the Gaussian bump."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2411_11041_amd.adr import Solver
    p = W.c3(args.n)
    th, dt, nst = p.extra["theta"], p.extra["dt"], p.extra["steps"]
    t0 = time.time()
    s = Solver(p, precision="fp64", theta=th, dt=dt, split_lines=args.split_lines)
    setup_s = time.time() - t0
    c = s.counts()
    per_step = c["line_unknowns_b"] + c["line_unknowns_g"]
    u0 = torch.from_numpy(np.ascontiguousarray(p.u0, np.float64).ravel()).cuda()
    u = torch.empty_like(u0)
    for _ in range(args.warmup):
        u.copy_(u0)
        s.time_step(u, th, dt, nst)
    def march():
        u.copy_(u0)
        s.time_step(u, th, dt, nst)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        march()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    el_ev, times = events_pass(s, march, args.steps)
    times["fp32"] = {}
    rf = kernel_roofline(times, c, args.split_lines)
    if rf["cls"].startswith("scatter"):  # the march writes both half steps (no update/norm mode)
        rf["bytes_per_unit"], rf["kernel"] = SCATTER_BYTES[("fp64", 2)], "k_scatter<double, double, 0>"
    work_launches = nst * args.steps
    bytes_per_launch = rf["bytes_per_unit"] * rf["units"]
    avg_launch_s = rf["total_ms"] / work_launches / 1e3
    achieved = bytes_per_launch / avg_launch_s / 1e9
    out = {"metric": METRIC, "value": per_step * nst * args.steps / el, "unit": "line-unknowns/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"c3: parabolic ADR, unit square {args.n}x{args.n}, mu=1e-2, sigma=0.5, C2's beta, "
                                  f"f=0, Gaussian bump u0; implicit Euler theta={th}, dt={dt}, {nst} steps "
                                  "(one eq.(10) splitting step per time step); a step of the bench = the whole march",
                      "time_steps_per_s": nst * args.steps / el, "ms_per_time_step": 1e3 * el / (nst * args.steps),
                      "line_unknowns_per_time_step": per_step, "setup_s": round(setup_s, 2),
                      "kernels": {k: {"ms": round(v[0], 3), "launches": v[1]} for k, v in times["fp64"].items()}},
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": rf["kernel"],
                        "avg_launch_us": round(avg_launch_s * 1e6, 2), "bytes_per_launch": int(bytes_per_launch)}}
    print(json.dumps(out), flush=True)
    s.close()


LINE_LAUNCHES = {0: "one per family", 1: "one per length bucket", 2: "one per length bucket, concurrent streams"}


def kernel_roofline(times, counts, split_lines=0):
    """Dominant kernel class over both precisions; achieved = bytes / time."""
    best = None
    for prec in ("fp64", "fp32"):
        for cls, (ms, cnt) in times[prec].items():
            if cnt == 0 or cls == "norm":
                continue
            if best is None or ms > best[2]:
                best = (prec, cls, ms, cnt)
    prec, cls, ms, cnt = best
    fam = 0 if cls.endswith("beta") else 1
    if cls.startswith("line"):
        units = counts["line_unknowns_b" if fam == 0 else "line_unknowns_g"]
        per = LINE_BYTES[(prec, fam)]
        tn = 'float' if prec == 'fp32' else 'double'
        kname = f"k_line_b<{tn}, {fam}, 12|8|4|2|1> ({LINE_LAUNCHES[split_lines]})" if split_lines else \
            f"k_line<{tn}, {fam}>"
    else:
        units = counts["grid_unknowns"]
        per = SCATTER_BYTES[(prec, 2 if fam == 0 else 3)]
        # beta half-sweep writes the grid field; gamma half-sweep updates the state
        kname = {("fp32", 0): "k_scatter<float, float, 0>", ("fp32", 1): "k_scatter<float, double, 2>",
                 ("fp64", 0): "k_scatter<double, double, 0>", ("fp64", 1): "k_scatter<double, double, 1>"}[(prec, fam)]
    # launches of this class per sweep (one per non-empty length bucket)
    return dict(prec=prec, cls=cls, kernel=kname, total_ms=ms, launches=cnt, bytes_per_unit=per, units=units)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design note, not a measured path.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c4":
        bench_c4(args)
        return
    if args.workload == "c5":
        bench_c5(args)
        return
    if args.workload == "c3":
        bench_c3(args)
        return
    import numpy as np
    import torch
    import workloads as W
    from paper_2411_11041_amd.adr import Solver

    if args.calibrate_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
    p = W.c2(args.n)
    t0 = time.time()
    s = Solver(p, precision="fp32", fp32_sweeps=args.fp32_sweeps, theta=1.0, dt=0.05, adaptive=args.adaptive,
               split_lines=args.split_lines)
    setup_s = time.time() - t0
    counts = s.counts()
    per_sweep = counts["line_unknowns_b"] + counts["line_unknowns_g"]
    u = torch.zeros(p.nx * p.ny, dtype=torch.float64, device="cuda")
    tuned = None
    if not args.no_autotune:
        tuned = s.autotune(u, 5000, args.tol)
        args.fp32_sweeps, args.adaptive, args.split_lines = tuned[0], tuned[1], tuned[3]
    shapes = tuned[4] if tuned else [0] * 5

    def solve():
        u.zero_()
        return s.split_iterate(u, 5000, args.tol)

    for _ in range(args.warmup):
        solve()
    # timed region 1 (value, ms_per_step): no per-launch events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sweeps = []
    for _ in range(args.steps):
        iters, rel, st = solve()
        sweeps.append(int(iters[0]))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # timed region 2 (roofline): the same steps with HIP events around every launch
    el_ev, times = events_pass(s, solve, args.steps)
    total_unknowns = per_sweep * sum(sweeps)
    value = total_unknowns / el
    ms_step = 1e3 * el / args.steps

    rf = kernel_roofline(times, counts, args.split_lines)
    # one launch per sweep of its precision processes `units` line unknowns (or
    # grid nodes).  Launches made after the convergence flag was set exit at
    # once and carry no work: the average is taken over the work-carrying
    # launches (their total time includes the empty ones, a conservative bound).
    if args.adaptive:  # the host stops at the converging sweep: every launch carries work
        work_launches = max(1, rf["launches"])
    else:
        n_sw_prec = sum(1 for k in range(sweeps[0]) if (k % (args.fp32_sweeps + 1) == 0) == (rf["prec"] == "fp64"))
        work_launches = max(1, n_sw_prec * args.steps)
    bytes_per_launch = rf["bytes_per_unit"] * rf["units"]
    avg_launch_s = rf["total_ms"] / work_launches / 1e3
    achieved = bytes_per_launch / avg_launch_s / 1e9
    copy_gbs = copy_bandwidth_gbs()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(rf["kernel"]),
                "copy_measured": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                "kernel": rf["kernel"], "avg_launch_us": round(avg_launch_s * 1e6, 2),
                "bytes_per_launch": int(bytes_per_launch), "launches": rf["launches"],
                "work_launches": work_launches, "events_pass_ms_per_step": round(1e3 * el_ev / args.steps, 3)}

    kernels = {pr: {k: {"ms": round(v[0], 3), "launches": v[1]} for k, v in times[pr].items()} for pr in times}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(p, args.cpu_sweeps)

    out = {
        "metric": METRIC, "value": value, "unit": "line-unknowns/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 line solves, f64 state/residual", "data": "synthetic",
        "config": {"workload": f"c2: stationary ADR, unit square {args.n}x{args.n}, mu=1e-3, sigma=1, "
                               "beta=curl psi, psi=x+0.5y+0.1 sin(pi x) sin(pi y), f=8 seeded Gaussians; "
                               "eq.(10) sweeps theta=1 dt=0.05 to 1e-8",
                   "time_to_1e-8_ms": ms_step, "sweeps_per_solve": sweeps[0],
                   "fp32_sweeps_per_fp64": args.fp32_sweeps, "adaptive_schedule": bool(args.adaptive),
                   "line_launches": LINE_LAUNCHES[args.split_lines], "line_shapes": shapes,
                   "autotuned": tuned is not None,
                   "line_unknowns_per_sweep": per_sweep,
                   "grid_unknowns": counts["grid_unknowns"], "lines": [counts["lines_b"], counts["lines_g"]],
                   "setup_s": round(setup_s, 2), "final_rel": float(rel[0]), "kernels": kernels},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    s.close()


def cpu_baseline(p, sweeps):
    """FP64 oracle (as it stands) on the same problem: `sweeps` sweeps, timed."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.method import Oracle
    t0 = time.time()
    o = Oracle(p)
    setup = time.time() - t0
    per = int(sum(int(f.interior().sum()) for f in o.fams))
    U = o.zero_field()
    with threadpool_limits(limits=1):  # one core, as reported
        t0 = time.perf_counter()
        for _ in range(sweeps):
            U = o.step(U, 1.0, 0.05)
        el = time.perf_counter() - t0
    return {"value": per * sweeps / el, "unit": "line-unknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"{sweeps} FP64 sweeps of the same {p.nx}x{p.ny} problem "
                      f"(oracle set-up {setup:.0f} s not timed; numpy/scipy, single thread)",
            "s_per_sweep": el / sweeps}


if __name__ == "__main__":
    main()
