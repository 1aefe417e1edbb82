"""Benchmark of the directional diffusion splitting hot path on one MI355X.

Default run (one JSON line): the stationary advection-dominated 2049 x 2049
problem (the step and `value`), with the batched 512-instance workload and the
learned warm start as two more legs of the same line.

Step = one stationary solve (eq. (10) sweeps to the fixed point, Sec. 2 limit)
of the 2049 x 2049 problem from zero to a relative fixed-point residual of
1e-8: FP64 sweeps (state, residual, convergence test) with FP32 increment
sweeps between them, whose transfer between the families is the grid's or the
direct one at the curves' intersections, as the autotuner picks (quantised
transfer weights either way); the FP64 sweeps fix the limit.  value = line
unknowns solved per second (every sweep solves one tridiagonal system per
curve of both families);
ms_per_step is the time to the 1e-8 residual.  Inputs are resident in device
memory before the timed region; set-up (curve tracing, tables, upload) and the
autotuner are outside it.

Each leg carries the roofline of its dominant kernel class: algorithmic bytes
(the method's own data, byte model below) per launch over the kernel's average
launch duration from HIP events on the library's stream, and separately the
bytes with the precomputed gather and scatter tables.  cpu_baseline is the
FP64 oracle, unchanged, run by one worker process per host core on the same
2049 x 2049 problem.
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
CLASSES = ("line_beta", "line_gamma", "scatter_beta", "scatter_gamma")
DTYPE = ("f32 line solves with quantised transfer weights (increment sweeps), "
         "f64 line solves, state, residual and convergence test (every FP64 sweep)")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# --------------------------------------------------------------------------
# Byte model per unit of work (line unknown for a line solve, interior grid
# node for a scatter).  w = 4 (FP32 sweeps) or 8 (FP64 sweeps).
#
# Line solve, algorithmic: the gathered grid value (one grid value per line
# unknown), the chord, |beta| (beta family), the load L (beta family, only in
# the sweeps that compute the iterate, i.e. the FP64 sweeps; the FP32
# increment sweeps d <- T d have no source) and the written line value.
# Tables: the bilinear stencil of eq. (22): cell index (4 B) and the two
# cell offsets (2w).
#
# Scatter, algorithmic: every line value of the family read once
# ((line unknowns + 2 ends) / grid nodes per node) and the grid traffic of the
# mode: FP32 beta write 4; FP64 beta write 8; the gamma half sweep of the
# stationary solve reads and writes the FP64 state and writes the FP32
# increment (8 + 8 + 4); in the time march the gamma scatter writes the state
# (8).  Tables: the slot's grid index (4), the first record's line node (4),
# three 16-bit offsets (6) and the weights of 4 records as their factors: the
# estimates' weight code and bracket weights and the records' positions (12 in
# the FP32 sweeps, quantised; 4 + 6 x 8 = 52 in FP64).
# --------------------------------------------------------------------------
def line_bytes(prec, fam):
    w = 4 if prec == "fp32" else 8
    state = prec == "fp64"
    alg = w + w + (w if fam == 0 else 0) + (w if (fam == 0 and state) else 0) + w
    meta = 4 + 2 * w
    return alg, meta


def scatter_bytes(prec, fam, counts, march=False):
    w = 4 if prec == "fp32" else 8
    key = "b" if fam == 0 else "g"
    nodes = counts[f"line_unknowns_{key}"] + 2 * counts[f"lines_{key}"]
    vals = w * nodes / counts["grid_unknowns"]
    if fam == 0:
        grid = w
    else:
        grid = 8 if march else 8 + 8 + 4
    meta = 4 + 4 + 6 + (12 if prec == "fp32" else 52)
    return vals + grid, meta


def direct_line_bytes(prec, fam, hybrid=False):
    """Line solve of the direct transfer, per line unknown (w = 4 FP32, 8
    FP64): algorithmic = one source value, the chord, |beta| (beta), the load
    (beta, FP64 sweeps only), the written value, and on the gamma-curves the
    update: FP64 sweeps read the old value and write the FP32 increment, FP32
    sweeps read and write the FP64 state (the FP32 sum of the block's
    increments when they steer the grid route, hybrid); tables = the two
    bracket indices and four weights (FP64: 8 + 32 B; FP32 sweeps: 10 B, a
    source node, a 16-bit offset and three packed fractions)."""
    w = 4 if prec == "fp32" else 8
    if fam == 0:
        alg = w + w + w + (w if prec == "fp64" else 0) + w
    else:
        alg = w + w + w + (8 + 4 if prec == "fp64" else (8 if hybrid else 16))
    return alg, (10 if prec == "fp32" else 40)


def hybrid_gather_bytes():
    """The block's gather of the FP64 sweep's FP32 update onto the gamma-curves
    (direct increments on the grid route), per gamma line unknown:
    algorithmic = one grid value, the written curve value and the cleared sum
    (4 + 4 + 4); tables = the bilinear stencil (cell index and two offsets)."""
    return 12.0, 12.0


def kernel_name(prec, cls, split_lines=0, march=False, direct=False, hybrid=False):
    tn = "float" if prec == "fp32" else "double"
    fam = 0 if cls.endswith("beta") else 1
    if hybrid and prec == "fp32":
        # direct increments on the grid route: the FP32 classes are the direct
        # line solves, the block's gather (class 2) and its closing scatter (3)
        direct = True
        if cls == "scatter_beta":
            return "k_line_values<float>"
    if cls.startswith("line"):
        d = "true" if direct else "false"  # the line kernels' direct-transfer flag
        if split_lines:
            return f"k_line_b<{tn}, {fam}, J, NT, {d}> (one launch per length bucket)"
        return f"k_line<{tn}, {fam}, {d}>"
    if prec == "fp32":
        return "k_scatter<float, float, 0>" if fam == 0 else "k_scatter<float, double, 2>"
    if fam == 0 or march:
        return "k_scatter<double, double, 0>"
    return "k_scatter<double, double, 1>"


def roofline(times, counts, split_lines=0, march=False, profile=None, direct=False, hybrid=False):
    """Per kernel class: algorithmic and with-table bytes of its timed
    launches (work counted by the library per launch) over their summed event
    time.  The dominant class (largest total time) gives the roofline object;
    `classes` lists every class.  hybrid: the FP32 classes are the direct
    increments of the grid route (options.increments = 1)."""
    rows = []
    for prec in ("fp64", "fp32"):
        for cls in CLASSES:
            ms, cnt, work = times[prec][cls]
            if cnt == 0 or ms <= 0:
                continue
            fam = 0 if cls.endswith("beta") else 1
            hyb = hybrid and prec == "fp32"
            if cls.startswith("line"):
                alg, meta = (direct_line_bytes(prec, fam, hyb) if (direct or hyb) else line_bytes(prec, fam))
            elif hyb and cls == "scatter_beta":
                alg, meta = hybrid_gather_bytes()
            else:
                alg, meta = scatter_bytes(prec, fam, counts, march)
            sec = ms / 1e3
            name = kernel_name(prec, cls, split_lines, march, direct, hybrid)
            rows.append(dict(kernel=name, prec=prec, cls=cls, ms=round(ms, 3), launches=cnt,
                             avg_launch_us=round(1e3 * ms / cnt, 2), work_per_launch=round(work / cnt),
                             alg_bytes_per_unit=round(alg, 2), table_bytes_per_unit=round(meta, 2),
                             achieved=round(alg * work / sec / 1e9, 1),
                             frac=round(alg * work / sec / 1e9 / HBM_PEAK_GBS, 4),
                             with_tables=round((alg + meta) * work / sec / 1e9, 1)))
    rows.sort(key=lambda r: -r["ms"])
    top = rows[0]
    out = {"bound": "hbm", "achieved": top["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": top["frac"], "traffic": None, "kernel": top["kernel"],
           "avg_launch_us": top["avg_launch_us"],
           "bytes_per_launch": int(top["alg_bytes_per_unit"] * top["work_per_launch"]),
           "with_tables": {"achieved": top["with_tables"], "frac": round(top["with_tables"] / HBM_PEAK_GBS, 4),
                           "bytes_per_launch": int((top["alg_bytes_per_unit"] + top["table_bytes_per_unit"])
                                                   * top["work_per_launch"])},
           "target_frac": 0.6, "classes": rows}
    if profile:
        out["traffic"] = measured_traffic(top["kernel"], profile)
    return out


def measured_traffic(kernel, profile):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when the
    summary is missing or was taken on other kernel sources.  A bucketed line
    class (one dispatch per length bucket and family per sweep) sums the
    dispatches of its kernels, one per bucket shape."""
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
    bucketed = kernel.startswith("k_line_b<")
    head, tail = (kernel.split(", J, NT, ")[0] + ", ", ", " + kernel.split(", J, NT, ")[1].split(">")[0] + ">") \
        if bucketed else (None, None)
    total, found = 0.0, False
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) != 4:
            continue
        name = cells[0]
        if not bucketed and name == "adr::" + kernel:
            return float(cells[3])
        if bucketed and name.startswith("adr::" + head) and name.endswith(tail):
            total += float(cells[3])
            found = True
    return total if found else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2049, help="grid nodes per side (c2, c3)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--fp32-sweeps", type=int, default=3)
    ap.add_argument("--adaptive", action="store_true",
                    help="with --no-autotune: adaptive schedule with at most --fp32-sweeps FP32 sweeps per FP64 sweep")
    ap.add_argument("--split-lines", type=int, choices=[0, 1, 2], default=0,
                    help="with --no-autotune (and c3): line-solve launches, 0 one per family, 1 one per "
                         "length bucket, 2 one per length bucket on concurrent streams")
    ap.add_argument("--line-shapes", type=str, default=None,
                    help="c4 with --no-autotune: the five bucket shapes, comma-separated (adr_set_line_shapes)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sweeps", type=int, default=3, help="FP64 oracle sweeps per worker process")
    ap.add_argument("--cpu-workers", type=int, default=0, help="oracle worker processes (0: one per host core, <= 16)")
    ap.add_argument("--acc-n", type=int, default=1025, help="direct leg: grid of the accuracy comparison (C1)")
    ap.add_argument("--direct-sweeps", type=int, default=12,
                    help="direct leg with --no-autotune: at most this many FP32 sweeps per FP64 sweep "
                         "(adaptive schedule)")
    ap.add_argument("--workload", choices=["all", "c2", "c3", "c4", "c5", "direct"], default="all",
                    help="all: c2 (the step and value) with the c4 and c5 legs (default); c2: one 2049^2 problem; "
                         "c3: the 2049^2 parabolic march (200 steps); c4: the 512-instance batch; "
                         "c5: learned warm start (train, then zero / eq. (11) / network starts)")
    ap.add_argument("--train", type=int, default=20480, help="c5: training samples")
    ap.add_argument("--epochs", type=int, default=160, help="c5: training epochs")
    ap.add_argument("--coarsen", type=int, default=8,
                    help="c5: the network runs on every coarsen-th node (1: on the 257x257 grid itself)")
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--graph", action="store_true", help="replay sweep blocks from a HIP graph")
    ap.add_argument("--krylov", type=int, default=0,
                    help="with --no-autotune: GMRES(m) on (I - T) U = c instead of the sweep schedule (m > 0)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="c2/c4: keep the given schedule and launches instead of choosing them with adr_autotune")
    ap.add_argument("--increments", choices=["auto", "grid", "direct"], default="auto",
                    help="c2/c4/c5: the FP32 increment sweeps' transfer on the grid route (auto: the "
                         "autotuner's choice of the two; grid with --no-autotune)")
    ap.add_argument("--transfer", choices=["grid", "direct"], default="grid",
                    help="c4: values handed between the families through the grid or at their intersections")
    ap.add_argument("--single-mode", action="store_true",
                    help="c4: time one launch mode only (no graph-replay comparison); for profiles")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="before the timed region, run one plain elementwise copy of 256 MiB in / 256 MiB out, "
                         "the reference dispatch for scaling hardware byte counters")
    return ap.parse_args()


def events_pass(s, solve, steps):
    """A second timed region over the same steps with per-launch HIP events on
    the library's stream (a few us between launches, so it is kept apart from
    the region that gives value); returns its seconds and, per precision and
    kernel class, (ms, launches, work)."""
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
    times = {pr: s.kernel_times(pr, reset=True, work=True) for pr in ("fp64", "fp32")}
    return el, times


def kernels_table(times):
    return {pr: {k: {"ms": round(v[0], 3), "launches": v[1], "work": v[2]} for k, v in times[pr].items() if v[1]}
            for pr in times}


def copy_bandwidth_gbs(nbytes=1 << 30, reps=10):
    """HBM bandwidth of a plain device copy (the library's copy kernel, nbytes
    in and nbytes out, on torch's current stream), timed with events."""
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


# ------------------------------------------------------------------ legs
def leg_c2(args):
    """One stationary 2049^2 solve per step (the bench's step and value)."""
    import torch
    import workloads as W
    from paper_2411_11041_amd.adr import Solver
    p = W.c2(args.n)
    t0 = time.time()
    # increments "auto": the direct-transfer records are built and the
    # autotuner times both kinds of increment sweeps
    inc = args.increments if args.increments != "auto" else ("grid" if args.no_autotune else "direct")
    s = Solver(p, precision="fp32", fp32_sweeps=args.fp32_sweeps, theta=1.0, dt=0.05, adaptive=args.adaptive,
               split_lines=args.split_lines, krylov=args.krylov, increments=inc)
    setup_s = time.time() - t0
    counts = s.counts()
    per_sweep = counts["line_unknowns_b"] + counts["line_unknowns_g"]
    u = torch.zeros(p.nx * p.ny, dtype=torch.float64, device="cuda")
    fp32_sweeps, adaptive, split, shapes, tuned = args.fp32_sweeps, args.adaptive, args.split_lines, [0] * 5, None
    kr = args.krylov
    hybrid = inc == "direct"
    if not args.no_autotune:
        tuned = s.autotune(u, 5000, args.tol)
        fp32_sweeps, adaptive, split, shapes, kr = tuned[0], tuned[1], tuned[3], tuned[4], tuned[5]
        hybrid = tuned[6] == 1
    log(f"c2: set-up {setup_s:.1f} s, schedule {fp32_sweeps} adaptive={adaptive} lines={split} krylov={kr} "
        f"increments={'direct' if hybrid else 'grid'}")

    def solve():
        u.zero_()
        return s.split_iterate(u, 5000, args.tol)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sweeps = []
    for _ in range(args.steps):
        iters, rel, st = solve()
        sweeps.append(int(iters[0]))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    el_ev, times = events_pass(s, solve, args.steps)
    rf = roofline(times, counts, split, profile="c2_2049_fp32lines.md", hybrid=hybrid)
    rf["copy_measured"] = round(copy_bandwidth_gbs(), 1)
    rf["frac_of_copy"] = round(rf["achieved"] / rf["copy_measured"], 4)
    rf["events_pass_ms_per_step"] = round(1e3 * el_ev / args.steps, 3)
    s.close()
    return {"value": per_sweep * sum(sweeps) / el, "ms_per_step": 1e3 * el / args.steps, "roofline": rf,
            "config": {"workload": f"c2: stationary ADR, unit square {args.n}x{args.n}, mu=1e-3, sigma=1, "
                                   "beta=curl psi, psi=x+0.5y+0.1 sin(pi x) sin(pi y), f=8 seeded Gaussians; "
                                   "eq.(10) sweeps theta=1 dt=0.05 from zero to 1e-8",
                       "time_to_1e-8_ms": round(1e3 * el / args.steps, 3), "sweeps_per_solve": sweeps[0],
                       "final_rel": float(rel[0]), "fp32_sweeps_per_fp64": fp32_sweeps,
                       "adaptive_schedule": bool(adaptive), "line_launches": LINE_LAUNCHES[split],
                       "line_shapes": shapes, "autotuned": tuned is not None, "krylov_gmres_m": kr,
                       "increment_sweeps": "direct transfer" if hybrid else "grid transfer",
                       "autotune_best_ms": round(tuned[2], 3) if tuned else None,
                       "line_unknowns_per_sweep": per_sweep, "grid_unknowns": counts["grid_unknowns"],
                       "lines": [counts["lines_b"], counts["lines_g"]], "setup_s": round(setup_s, 2),
                       "kernels": kernels_table(times)}}


def leg_direct(args):
    """The interpolation-free transfer against the grid route: C2 time to 1e-8
    and sweeps with every sweep in FP64 (both routes) and with FP32 increment
    sweeps (direct route, its launches and schedule from adr_autotune, or the
    adaptive schedule of --direct-sweeps with --no-autotune; the grid route's
    is the main leg), and the distance of each route's fixed point from the
    exact solution of the manufactured problem (C1)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2411_11041_amd.adr import Solver
    p = W.c2(args.n)
    res = {}
    variants = (("grid_fp64", "grid", {"precision": "fp64"}),
                ("direct_fp64", "direct", {"precision": "fp64"}),
                ("direct_fp32", "direct", {"precision": "fp32", "fp32_sweeps": args.direct_sweeps, "adaptive": True}))
    for name, tr, kw in variants:
        t0 = time.time()
        s = Solver(p, theta=1.0, dt=0.05, split_lines=0, transfer=tr, **kw)
        setup_s = time.time() - t0
        counts = s.counts()
        per_sweep = counts["line_unknowns_b"] + counts["line_unknowns_g"]
        u = torch.zeros(p.nx * p.ny, dtype=torch.float64, device="cuda")
        tuned = None
        if kw["precision"] == "fp32" and not args.no_autotune:
            # the direct route's own launches and schedule (the grid route's
            # FP32 solve is the main leg)
            tuned = s.autotune(u, 5000, args.tol)
            log(f"direct leg: {name} autotuned schedule {tuned[0]} adaptive={tuned[1]} lines={tuned[3]} "
                f"shapes={tuned[4]}")

        def solve():
            u.zero_()
            return s.split_iterate(u, 5000, args.tol)

        for _ in range(args.warmup):
            solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            iters, rel, st = solve()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        el_ev, times = events_pass(s, solve, args.steps)
        rf = roofline(times, counts, tuned[3] if tuned else 0, direct=(tr == "direct"),
                      profile="c2_2049_direct.md" if name == "direct_fp32" else None)
        res[name] = {"ms_per_step": round(1e3 * el / args.steps, 3), "sweeps": int(iters[0]),
                     "final_rel": float(rel[0]), "value": per_sweep * int(iters[0]) * args.steps / el,
                     "setup_s": round(setup_s, 2), "events_pass_ms_per_step": round(1e3 * el_ev / args.steps, 3),
                     "autotuned": None if tuned is None else {
                         "fp32_sweeps_per_fp64": tuned[0], "adaptive_schedule": bool(tuned[1]),
                         "line_launches": LINE_LAUNCHES[tuned[3]], "line_shapes": list(tuned[4])},
                     "roofline": rf, "kernels": kernels_table(times)}
        log(f"direct leg: {name} {res[name]['ms_per_step']:.2f} ms, {res[name]['sweeps']} sweeps")
        s.close()
    # accuracy on the manufactured problem
    q = W.c1(args.acc_n)
    X, Y = q.coords()
    ue = W.manufactured_u(X, Y).ravel()
    errs = {}
    for tr in ("grid", "direct"):
        s = Solver(q, precision="fp64", theta=1.0, dt=0.05, transfer=tr)
        u = torch.zeros(q.nx * q.ny, dtype=torch.float64, device="cuda")
        s.split_iterate(u, 5000, 1e-11)
        # the solve writes the interior nodes; the others stay zero, as ue is on Gamma
        e = np.abs(u.cpu().numpy() - ue)
        errs[tr] = float(e.max() / np.abs(ue).max())
        s.close()
    best = res["direct_fp32"]
    return {"value": best["value"], "unit": "line-unknowns/s", "ms_per_step": best["ms_per_step"],
            "roofline": best["roofline"],
            "config": {"workload": f"c2 {args.n}x{args.n} stationary to 1e-8: values handed between the families "
                                   "directly at their segment intersections (transfer=direct) against the grid "
                                   "route (scatter + bilinear gather)",
                       "direct_fp32": {k: v for k, v in best.items() if k != "roofline"},
                       "direct_fp64": res["direct_fp64"], "grid_fp64": res["grid_fp64"],
                       f"c1_{args.acc_n}_max_rel_error_vs_exact": errs}}


def gen_c4(n_inst):
    from concurrent.futures import ThreadPoolExecutor
    import workloads as W
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(W.c4_instance, range(n_inst)))


def leg_c4(args):
    """Batched workload: every instance of the batch in each launch."""
    import numpy as np
    import torch
    from paper_2411_11041_amd.adr import Solver
    t0 = time.time()
    probs = gen_c4(args.instances)
    gen_s = time.time() - t0
    t0 = time.time()
    # increments "auto" on the grid transfer: both kinds of increment sweeps
    # for the autotuner (the direct transfer's increments are direct already)
    inc = args.increments if args.increments != "auto" else (
        "direct" if (args.transfer == "grid" and not args.no_autotune) else "grid")
    s = Solver(probs, precision="fp32", fp32_sweeps=args.fp32_sweeps, theta=1.0, dt=0.05, graph=args.graph,
               adaptive=args.adaptive, split_lines=args.split_lines, krylov=args.krylov, transfer=args.transfer,
               increments=inc)
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
    fp32_sweeps, adaptive, split, shapes, tuned = args.fp32_sweeps, args.adaptive, args.split_lines, [0] * 5, None
    kr = args.krylov
    hybrid = inc == "direct" and args.transfer == "grid"
    if args.no_autotune and args.line_shapes:
        shapes = [int(v) for v in args.line_shapes.split(",")]
        s.set_line_shapes(shapes)
    if not args.no_autotune:
        tuned = s.autotune(u, 3000, args.tol)
        fp32_sweeps, adaptive, split, shapes, kr = tuned[0], tuned[1], tuned[3], tuned[4], tuned[5]
        hybrid = tuned[6] == 1 and args.transfer == "grid"
    log(f"c4: gen {gen_s:.1f} s, set-up {setup_s:.1f} s, schedule {fp32_sweeps} adaptive={adaptive} lines={split} "
        f"krylov={kr} increments={'direct' if hybrid else 'grid'}")

    def solve():
        u.zero_()
        return s.split_iterate(u, 3000, args.tol)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = rel = None
    for _ in range(args.steps):
        its, rel, st = solve()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    el_ev, times = events_pass(s, solve, args.steps)
    rf = roofline(times, counts, split, profile="c4_512_fp32lines.md" if args.transfer == "grid" else None,
                  direct=args.transfer == "direct", hybrid=hybrid)
    inc_kind = "direct transfer" if (hybrid or args.transfer == "direct") else "grid transfer"
    rf["events_pass_ms_per_step"] = round(1e3 * el_ev / args.steps, 2)
    solved = int((its.astype(np.int64) * per_inst).sum()) * args.steps
    # the same solves with the blocks replayed from HIP graphs (one per block
    # length, captured in the warm-up) instead of eager launches on the lists
    # compacted to the unfinished instances
    if args.single_mode or args.transfer == "direct":  # graphs serve the grid transfer only
        s.close()
        return c4_result(args, probs, counts, per_inst, its, rel, el, rf, gen_s, setup_s, fp32_sweeps, adaptive,
                         split, shapes, kr, tuned, solved, times, None, inc_kind)
    s.set_graph(not args.graph)
    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        its_g, rel_g, _ = solve()
    torch.cuda.synchronize()
    el_g = time.perf_counter() - t0
    s.set_graph(args.graph)
    other = {"graph_replay": not args.graph, "ms_per_step": round(1e3 * el_g / args.steps, 2),
             "value": int((its_g.astype(np.int64) * per_inst).sum()) * args.steps / el_g,
             "converged": int((rel_g <= args.tol).sum())}
    log(f"c4: {'graph replay' if not args.graph else 'eager'} {other['ms_per_step']} ms")
    s.close()
    return c4_result(args, probs, counts, per_inst, its, rel, el, rf, gen_s, setup_s, fp32_sweeps, adaptive, split,
                     shapes, kr, tuned, solved, times, other, inc_kind)


def c4_result(args, probs, counts, per_inst, its, rel, el, rf, gen_s, setup_s, fp32_sweeps, adaptive, split, shapes,
              kr, tuned, solved, times, other, inc_kind):
    import numpy as np
    return {"value": solved / el, "unit": "line-unknowns/s", "ms_per_step": 1e3 * el / args.steps, "roofline": rf,
            "config": {"workload": f"c4: {len(probs)} stationary instances (disc/L-shape, 33..1025 per side, "
                                   "mu logU[1e-4,1e-1], sigma U[0.1,10], random divergence-free beta), "
                                   "every instance in each launch, to 1e-8 per instance",
                       "time_to_1e-8_ms": round(1e3 * el / args.steps, 2), "grid_unknowns": counts["grid_unknowns"],
                       "line_unknowns_per_sweep": int(per_inst.sum()), "lines": [counts["lines_b"], counts["lines_g"]],
                       "sweeps_min_median_max": [int(its.min()), int(np.median(its)), int(its.max())],
                       "converged": int((rel <= args.tol).sum()), "gen_s": round(gen_s, 1),
                       "setup_s": round(setup_s, 1), "graph": bool(args.graph),
                       "fp32_sweeps_per_fp64": fp32_sweeps, "adaptive_schedule": bool(adaptive),
                       "line_launches": LINE_LAUNCHES[split], "line_shapes": shapes, "krylov_gmres_m": kr,
                       "autotune_ms": round(tuned[2], 2) if tuned else None, "transfer": args.transfer,
                       "increment_sweeps": inc_kind,
                       "other_launch_mode": other, "kernels": kernels_table(times)}}


CNN_FLOP_PER_PIXEL = 2 * 9 * (4 * 32 + 32 * 32 + 32 * 32 + 32)  # forward, 4 conv layers
MFMA_BF16_PEAK_TFS = 2500.0


def leg_c5(args):
    """Learned warm start: dataset from the solver, training, then the 64 test
    seeds solved to the tolerance from zero, from the eq. (11) iterate and from
    the network's prediction (inference and the residual-judged fallback
    inside the timed region)."""
    import torch
    from paper_2411_11041_amd import warmstart as WS
    from paper_2411_11041_amd.adr import Net
    n, B = 257, 64
    # the batch configuration of C4 (short curves: one launch per length bucket,
    # adaptive schedule, eager launches on the compacted lists) for the dataset
    wl = WS.Workload(n=n, batch=128, coarsen=args.coarsen, fp32_sweeps=12, adaptive=True, split_lines=1,
                     graph=False, increments="direct" if args.increments != "grid" else "grid")
    Hc, Wc = wl.coarse_shape()
    net = Net(Hc, Wc, 128)
    net.set_params(WS.he_init(0))
    t0 = time.time()
    x, t = wl.generate(net, list(range(args.train)), tol=1e-10)
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    log(f"c5: {args.train} samples generated in {gen_s:.1f} s")
    t0 = time.time()
    losses = WS.train(net, x, t, wl.mask_c, args.train, wl.HWc, args.epochs, batch=32, lr=2e-3, lr_end=2e-5)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    log(f"c5: trained {args.epochs} epochs in {train_s:.1f} s, loss {losses[-1]:.2e}")
    del x, t
    test = list(range(20000, 20000 + B))
    # the test batch's context, autotuned once (not timed); all three starts use it
    tuned = wl.tune(test, args.tol)
    log(f"c5: autotuned schedule {tuned[0]} adaptive={tuned[1]} lines={tuned[3]} shapes={tuned[4]} "
        f"krylov={tuned[5]} increments={'direct' if tuned[6] == 1 else 'grid'}")
    res = {}
    for name in ("zero", "eq11", "network"):
        for _ in range(args.warmup + 1):
            if name == "zero":
                u, it, rel, sec = wl.solve_batch(test, args.tol)
                fb = 0
            else:
                u, it, rel, sec, fb = wl.warm_started(net, test, args.tol, use_net=name == "network")
        res[name] = {"ms": round(sec * 1e3, 2), "sweeps_mean": round(float(it.mean()), 2), "sweeps_max": int(it.max()),
                     "converged": int((rel <= args.tol).sum()), "fallbacks": int(fb)}
    s = wl.solver
    counts = s.counts()
    per_sweep = counts["line_unknowns_b"] + counts["line_unknowns_g"]
    # solve kernels of the network-started solve, with events
    _, times = events_pass(s, lambda: wl.warm_started(net, test, args.tol, use_net=True), 1)
    rf = roofline(times, counts)
    # the network forward on the matrix cores, with events on torch's stream
    probs = wl.problems(test)
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
    net.close()
    wl.solver.close()
    nw = res["network"]
    return {"value": per_sweep * nw["sweeps_mean"] / (nw["ms"] * 1e-3), "unit": "line-unknowns/s",
            "ms_per_step": nw["ms"], "roofline": rf,
            "config": {"workload": f"c5: {B} test seeds, unit square {n}x{n}, sigma=1, curved stream, "
                                   "mu logU[1e-3,1e-1], 1..8 Gaussians; solved to the tolerance from three starts "
                                   "(the step: the network start, inference included)",
                       "tol": args.tol, "starts": res,
                       "gain_vs_eq11": round(res["eq11"]["ms"] / nw["ms"], 4),
                       "gain_vs_zero": round(res["zero"]["ms"] / nw["ms"], 4),
                       "network_grid": f"{Hc}x{Wc} (every {args.coarsen}th node)",
                       "solver": {"fp32_sweeps_per_fp64": tuned[0], "adaptive_schedule": bool(tuned[1]),
                                  "line_launches": LINE_LAUNCHES[tuned[3]], "line_shapes": list(tuned[4]),
                                  "krylov_gmres_m": tuned[5], "autotune_ms": round(tuned[2], 2),
                                  "increment_sweeps": "direct transfer" if tuned[6] == 1 else "grid transfer"},
                       "train_samples": args.train, "epochs": args.epochs,
                       "final_train_loss": losses[-1], "gen_s": round(gen_s, 1), "train_s": round(train_s, 1),
                       "train_samples_per_s": round(args.train * args.epochs / train_s, 1),
                       "forward": {"ms_batch64": round(fwd_ms, 4), "achieved_tflops": round(tflops, 2),
                                   "peak_tflops": MFMA_BF16_PEAK_TFS, "frac": round(tflops / MFMA_BF16_PEAK_TFS, 5),
                                   "bound": "mfma"}}}


def leg_c3(args):
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

    def march():
        u.copy_(u0)
        s.time_step(u, th, dt, nst)

    for _ in range(args.warmup):
        march()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        march()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    _, times = events_pass(s, march, args.steps)
    rf = roofline(times, c, args.split_lines, march=True, profile="c3_2049_fp64_march.md")
    s.close()
    return {"value": per_step * nst * args.steps / el, "unit": "line-unknowns/s",
            "ms_per_step": 1e3 * el / args.steps, "roofline": rf, "dtype": "f64",
            "config": {"workload": f"c3: parabolic ADR, unit square {args.n}x{args.n}, mu=1e-2, sigma=0.5, "
                                   f"C2's beta, f=0, Gaussian bump u0; implicit Euler theta={th}, dt={dt}, "
                                   f"{nst} steps (one eq.(10) splitting step per time step); a step of the "
                                   "bench = the whole march",
                       "time_steps_per_s": nst * args.steps / el, "ms_per_time_step": 1e3 * el / (nst * args.steps),
                       "line_unknowns_per_time_step": per_step, "setup_s": round(setup_s, 2),
                       "kernels": kernels_table(times)}}


LINE_LAUNCHES = {0: "one per family", 1: "one per length bucket", 2: "one per length bucket, concurrent streams"}


# ------------------------------------------------------------ CPU baseline
_ORC = None


def _oracle_worker(sweeps):
    from threadpoolctl import threadpool_limits
    o = _ORC
    U = o.zero_field()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for _ in range(sweeps):
            U = o.step(U, 1.0, 0.05)
        t1 = time.perf_counter()
    return t0, t1


def cpu_baseline(n, sweeps, workers):
    """The FP64 oracle, unchanged, on the same n^2 problem: built once, then
    `workers` forked processes (one per host core, single-threaded BLAS) each
    run `sweeps` sweeps from zero; value = line unknowns solved per second over
    the span from the first worker's start to the last one's end.  Runs before
    the process touches the GPU."""
    import multiprocessing as mp
    import workloads as W
    from oracle.method import Oracle
    global _ORC
    t0 = time.time()
    _ORC = Oracle(W.c2(n))
    setup = time.time() - t0
    per = int(sum(int(f.interior().sum()) for f in _ORC.fams))
    cores = workers or min(16, len(os.sched_getaffinity(0)))
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        spans = pool.map(_oracle_worker, [sweeps] * cores)
    el = max(b for _, b in spans) - min(a for a, _ in spans)
    per_sweep_s = sum(b - a for a, b in spans) / (sweeps * cores)
    _ORC = None
    return {"value": per * sweeps * cores / el, "unit": "line-unknowns/s", "cores": cores, "kind": "oracle",
            "sample": f"{sweeps} FP64 sweeps from zero of the same {n}x{n} problem in each of {cores} worker "
                      f"processes (one per host core, single-threaded numpy/scipy; oracle set-up {setup:.0f} s "
                      "not timed)",
            "s_per_sweep_per_worker": round(per_sweep_s, 3)}


def calibrate_copy():
    """A plain 256 MiB-in / 256 MiB-out elementwise copy, whose FETCH_SIZE and
    WRITE_SIZE give the counters' scale (read by the profile summaries)."""
    import torch
    a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    del a, b


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design note, not a measured path.", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
    cpu = None
    if args.workload in ("all", "c2") and not args.no_cpu:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(args.n, args.cpu_sweeps, args.cpu_workers)
        log(f"cpu baseline: {cpu['value']:.3e} line-unknowns/s on {cpu['cores']} cores")
    legs = {}
    if args.workload == "c3":
        main_leg = leg_c3(args)
    elif args.workload == "c4":
        main_leg = leg_c4(args)
    elif args.workload == "c5":
        main_leg = leg_c5(args)
    elif args.workload == "direct":
        main_leg = leg_direct(args)
    else:
        main_leg = leg_c2(args)
        log(f"c2: {main_leg['ms_per_step']:.2f} ms to 1e-8")
        if args.workload == "all":
            legs["c4"] = leg_c4(args)
            log(f"c4: {legs['c4']['ms_per_step']:.1f} ms to 1e-8")
            legs["c5"] = leg_c5(args)
            log(f"c5: network start {legs['c5']['ms_per_step']:.2f} ms")
            legs["direct"] = leg_direct(args)
            log(f"direct transfer: {legs['direct']['ms_per_step']:.2f} ms to 1e-8")
    out = {"metric": METRIC, "value": main_leg["value"], "unit": "line-unknowns/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_leg["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": main_leg.get("dtype", DTYPE), "data": "synthetic",
           "config": main_leg["config"], "roofline": main_leg["roofline"], "cpu_baseline": cpu}
    if legs:
        out["legs"] = legs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
