"""Learned warm start driver: dataset generation with the splitting solver,
training of the network (include/adrnn.h kernels) and the warm-started solve.

Every numerical step runs in the HIP library; this module orchestrates the
calls and moves device buffers (torch tensors) between them.

Workload: 257 x 257 unit square, C2's divergence-free beta, sigma = 1,
mu log-uniform in [1e-3, 1e-1], a mixture of 1..8 Gaussians as source
(seeded per sample).  All samples share the grid, the domain and beta, so one
solver context (one set of traced curves) serves every batch: adr_update swaps
in each batch's mu and f.

With coarsen = r > 1 the network sees every sample on the grid of every r-th
node: f, the eq. (11) iterate s and the converged solution are restricted by
full weighting (adrnn_restrict), the network runs on that coarse grid, and
its output is interpolated bilinearly back to the fine nodes inside the warm
start (adrnn_warm_start_prolong).  The network's context is then created for
the coarse grid (coarse_shape()).
"""
from __future__ import annotations

import time

import numpy as np

import workloads as W

from .adr import Net, Solver


class Workload:
    def __init__(self, n=257, batch=128, precision="fp32", fp32_sweeps=3, dt=0.05, graph=True, coarsen=1,
                 adaptive=False, split_lines=0, increments="grid"):
        import torch
        if coarsen < 1 or (n - 1) % coarsen:
            raise ValueError(f"coarsening factor {coarsen} does not divide {n - 1}")
        self.n = n
        self.batch = batch
        grid = W._grid(n)
        _, self.b1, self.b2 = W.curved_stream(*grid)
        self.HW = n * n
        mask = np.zeros((n, n), np.uint8)
        mask[1:-1, 1:-1] = 1
        self.mask_np = mask
        self.mask = torch.from_numpy(mask.ravel()).cuda()
        # the network's grid: every coarsen-th node (the fine grid when 1)
        self.r = coarsen
        self.nc = (n - 1) // coarsen + 1
        self.HWc = self.nc * self.nc
        mc = np.zeros((self.nc, self.nc), np.uint8)
        mc[1:-1, 1:-1] = 1
        self.mask_c = torch.from_numpy(mc.ravel()).cuda()
        # increments="direct": the contexts also hold the direct-transfer records, so
        # that tune() times both kinds of increment sweeps
        self.kw = dict(precision=precision, fp32_sweeps=fp32_sweeps, theta=1.0, dt=dt, graph=graph,
                       adaptive=adaptive, split_lines=split_lines, increments=increments)
        self.solver = None

    def problems(self, seeds):
        out = []
        for s in seeds:
            p = W.c5_sample(int(s), n=self.n)
            p.beta1, p.beta2 = self.b1, self.b2  # shared arrays: one set of curves
            out.append(p)
        return out

    def _bind(self, probs):
        if self.solver is None or self.solver.n != len(probs):
            if self.solver is not None:
                self.solver.close()
            self.solver = Solver(probs, **self.kw)
        else:
            self.solver.update(probs)
        return self.solver

    def tune(self, seeds, tol, max_iters=2000):
        """adr_autotune on the batch of these seeds (from zero): the context
        bound to them keeps the fastest line launches, shapes and schedule.
        Returns the autotuner's choice."""
        import torch
        probs = self.problems(seeds)
        s = self._bind(probs)
        work = torch.zeros(len(probs) * self.HW, dtype=torch.float64, device="cuda")
        return s.autotune(work, max_iters, tol)

    def solve_batch(self, seeds, tol, max_iters=2000, start=None):
        """Returns u (device, B*HW), iters, rel, seconds.  start: None (zero) or a tensor."""
        import torch
        probs = self.problems(seeds)
        s = self._bind(probs)
        u = torch.zeros(len(probs) * self.HW, dtype=torch.float64, device="cuda") if start is None else start
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it, rel, st = s.split_iterate(u, max_iters, tol)
        torch.cuda.synchronize()
        return u, it, rel, time.perf_counter() - t0

    def coarse_shape(self):
        """(H, W) of the network's context."""
        return self.nc, self.nc

    def _net_inputs(self, net, B, f, g, mu, u_star=None):
        """pack() on the network's grid (restricted fields when coarsened)."""
        if self.r > 1:
            f, g = net.restrict(B, self.r, f), net.restrict(B, self.r, g)
            if u_star is not None:
                u_star = net.restrict(B, self.r, u_star)
        return net.pack(B, f, g, self.mask_c, mu, u_star=u_star)

    def f_tensor(self, probs):
        import torch
        return torch.from_numpy(np.concatenate([p.f.ravel() for p in probs])).cuda()

    def generate(self, net, seeds, tol=1e-10, log=None):
        """Network inputs x0 (BF16 bits) and targets for the given seeds, on
        the network's grid."""
        import torch
        N = len(seeds)
        HWc = self.HWc
        x_all = torch.empty(N * HWc * 4, dtype=torch.int16, device="cuda")
        t_all = torch.empty(N * HWc, dtype=torch.float32, device="cuda")
        for c0 in range(0, N, self.batch):
            cs = seeds[c0:c0 + self.batch]
            B = len(cs)
            probs = self.problems(cs)
            s = self._bind(probs)
            u = torch.zeros(B * self.HW, dtype=torch.float64, device="cuda")
            it, rel, _ = s.split_iterate(u, 3000, tol)
            g = torch.zeros_like(u)
            s.initial_guess(g)
            x0, tgt, _ = self._net_inputs(net, B, self.f_tensor(probs), g, [p.mu for p in probs], u_star=u)
            x_all[c0 * HWc * 4:(c0 + B) * HWc * 4] = x0
            t_all[c0 * HWc:(c0 + B) * HWc] = tgt
            if log:
                log(f"generated {c0 + B}/{N} (sweeps max {int(it.max())}, rel max {rel.max():.1e})")
        return x_all, t_all

    def warm_started(self, net, seeds, tol, max_iters=2000, use_net=True):
        """Solve from the eq. (11) iterate, corrected by the network when use_net.

        The splitting residual judges the start (adr_split_iterate_judged):
        an instance whose network start has an FP64 update not below the
        eq. (11) iterate's restarts from the eq. (11) iterate.  Timed from the
        first call (inference included).  Returns u, iters, rel, seconds,
        fallbacks.
        """
        import torch
        probs = self.problems(seeds)
        B = len(probs)
        s = self._bind(probs)
        f = self.f_tensor(probs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = torch.zeros(B * self.HW, dtype=torch.float64, device="cuda")
        s.initial_guess(g)
        fallback = 0
        if use_net:
            x0, _, sn = self._net_inputs(net, B, f, g, [p.mu for p in probs])
            out = net.forward(B, x0)
            u = torch.empty_like(g)
            if self.r > 1:
                net.warm_start_prolong(B, self.r, g, sn, out, self.mask, u)
            else:
                net.warm_start(B, g, sn, out, self.mask, u)
            it, rel, _, used = s.split_iterate_judged(u, g, max_iters, tol)
            fallback = int(used.sum())
        else:
            u = g
            it, rel, _ = s.split_iterate(u, max_iters, tol)
        torch.cuda.synchronize()
        return u, it, rel, time.perf_counter() - t0, fallback


def train(net, x_all, t_all, mask, N, HW, epochs, batch=32, lr=1e-3, lr_end=None, seed=0, log=None,
          on_epoch=None):
    """Adam on shuffled minibatches, the step size decaying from lr to lr_end
    (cosine over all steps; constant when lr_end is None).  on_epoch(ep, loss)
    is called after each epoch.  Returns the per-epoch mean losses."""
    import math

    import torch
    rng = np.random.default_rng(seed)
    xv = x_all.view(N, HW * 4)
    tv = t_all.view(N, HW)
    losses = []
    per_ep = max(N // batch, 1)
    total = epochs * per_ep
    step = 0
    net.loss_sum(reset=True)
    for ep in range(epochs):
        # the epoch's permutation goes to the device once (a copy from pageable
        # host memory waits for the stream); the steps then queue without a
        # host synchronisation, and the loss is summed on the device
        perm = torch.from_numpy(rng.permutation(N)).cuda()
        for b0 in range(0, N - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb = xv.index_select(0, idx).contiguous().view(-1)
            tb = tv.index_select(0, idx).contiguous().view(-1)
            a = lr if lr_end is None else lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * step / total))
            net.train_step(batch, xb, tb, mask, a, want_loss=False)
            step += 1
        tot, nb = net.loss_sum(reset=True)
        losses.append(tot / max(nb, 1))
        if log:
            log(f"epoch {ep + 1}/{epochs} loss {losses[-1]:.3e}")
        if on_epoch:
            on_epoch(ep, losses[-1])
    return losses


def he_init(seed=0, c_in=4):
    """He-normal FP32 weights, zero biases, in the flat layout of include/adrnn.h."""
    rng = np.random.default_rng(seed)
    parts = []
    for c_out, cin in ((32, c_in), (32, 32), (32, 32), (1, 32)):
        w = rng.standard_normal((c_out, 3, 3, cin)) * np.sqrt(2.0 / (9 * cin))
        parts += [w.astype(np.float32).ravel(), np.zeros(c_out, np.float32)]
    return np.concatenate(parts)
