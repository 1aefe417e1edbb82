"""ctypes binding of libadr.so (include/adr.h): argument marshalling only.

Every step of the solver runs in the HIP library; this module converts problem
descriptions into the C structs, passes device pointers of torch tensors and
returns host results.  It fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadr.so")

ADR_OK, ADR_EINVAL, ADR_ENOMEM, ADR_EDEVICE, ADR_EBETA, ADR_ENONFINITE, ADR_ENOTCONV = 0, -1, -2, -3, -4, -5, 1
ADR_ESINGULAR = -6
DOM_BOX, DOM_DISC, DOM_POLYGON = 0, 1, 2
PREC_FP64, PREC_FP32_LINES = 0, 1

EXPORTS = ("adr_setup", "adr_layout", "adr_counts", "adr_update", "adr_split_iterate", "adr_split_iterate_judged",
           "adr_autotune", "adr_set_line_shapes", "adr_set_graph", "adr_time_step",
           "adr_residual", "adr_initial_guess", "adr_export_lines", "adr_export_scatter", "adr_export_scatter_factors",
           "adr_export_direct", "adr_export_direct_packed",
           "adr_set_timing", "adr_kernel_times",
           "adr_destroy", "adr_last_error", "adr_copy_probe", "adr_line_solve", "adr_line_solve_noalloc")

KERNEL_CLASSES = ("line_beta", "line_gamma", "scatter_beta", "scatter_gamma", "norm")


class ADRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"adr status {code}: {msg}")
        self.code = code


class Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("a", C.c_double), ("b", C.c_double), ("c", C.c_double), ("d", C.c_double),
                ("domain", C.c_int32), ("n_dom_params", C.c_int32),
                ("dom_params", C.POINTER(C.c_double)),
                ("mu", C.c_double), ("sigma", C.c_double),
                ("beta1", C.POINTER(C.c_double)), ("beta2", C.POINTER(C.c_double)),
                ("f", C.POINTER(C.c_double)), ("g", C.POINTER(C.c_double)), ("psi", C.POINTER(C.c_double))]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("fp32_sweeps", C.c_int32),
                ("theta", C.c_double), ("dt", C.c_double),
                ("stream", C.c_void_p), ("timing", C.c_int32), ("host_only", C.c_int32),
                ("graph", C.c_int32), ("adaptive", C.c_int32), ("split_lines", C.c_int32),
                ("pivot_tol", C.c_double), ("splitting", C.c_int32), ("stabilize", C.c_int32),
                ("krylov", C.c_int32), ("transfer", C.c_int32), ("increments", C.c_int32)]


_lib = None


def load():
    """Load libadr.so (built in-tree); raise if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built: run paper_2411_11041_amd/build.py")
    # torch's HIP runtime must be the one in the process: import it first so
    # that the library binds to the already loaded runtime
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    i32, i64, dbl, vp = C.c_int32, C.c_int64, C.c_double, C.c_void_p
    P = C.POINTER
    lib.adr_setup.argtypes = [P(Problem), i32, P(Options), P(vp)]
    lib.adr_layout.argtypes = [vp, P(i64)]
    lib.adr_counts.argtypes = [vp, P(i64), P(i64), P(i64), P(i64), P(i64)]
    lib.adr_update.argtypes = [vp, P(Problem), i32]
    lib.adr_split_iterate.argtypes = [vp, vp, i32, dbl, P(i32), P(dbl)]
    lib.adr_split_iterate_judged.argtypes = [vp, vp, vp, i32, dbl, P(i32), P(dbl), P(i32)]
    lib.adr_autotune.argtypes = [vp, vp, i32, dbl, P(i32), P(i32), P(dbl), P(i32), P(i32), P(i32), P(i32)]
    lib.adr_set_line_shapes.argtypes = [vp, P(i32)]
    lib.adr_set_graph.argtypes = [vp, i32]
    lib.adr_set_timing.argtypes = [vp, i32]
    lib.adr_time_step.argtypes = [vp, vp, dbl, dbl, i32, i32, dbl, P(i32)]
    lib.adr_residual.argtypes = [vp, vp, P(dbl)]
    lib.adr_initial_guess.argtypes = [vp, vp]
    lib.adr_export_lines.argtypes = [vp, i32, i32, P(i64), P(i64), P(i64), P(dbl), P(dbl)]
    lib.adr_export_scatter.argtypes = [vp, i32, i32, P(i64), P(i32), P(i32), P(dbl), P(dbl), P(dbl)]
    lib.adr_export_direct.argtypes = [vp, i32, i32, P(i64), P(i32), P(dbl)]
    lib.adr_export_direct_packed.argtypes = [vp, i32, i32, P(i64), P(i32), P(C.c_int16), P(C.c_uint32)]
    lib.adr_export_scatter_factors.argtypes = [vp, i32, i32, P(i64), P(dbl), P(dbl), P(dbl)]
    lib.adr_kernel_times.argtypes = [vp, i32, P(dbl), P(i64), P(i64), i32]
    lib.adr_destroy.argtypes = [vp]
    lib.adr_copy_probe.argtypes = [vp, vp, i64, vp]
    lib.adr_line_solve.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp, vp, dbl, vp]
    lib.adr_line_solve_noalloc.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp, vp, dbl, vp]
    lib.adr_last_error.argtypes = [vp]
    lib.adr_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("adr_last_error",):
            getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _device_ptr(t):
    """Device pointer of a torch float64 CUDA tensor (contiguous)."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("u must be a contiguous float64 device tensor")
    return C.c_void_p(t.data_ptr())


def copy_probe(src, dst, stream=None):
    """dst = src (device tensors of equal byte size) by the library's plain copy
    kernel, queued on torch's current stream (measurement export)."""
    import torch
    lib = load()
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_cuda and dst.is_cuda):
        raise ValueError("copy_probe: two device tensors of equal size")
    st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    code = lib.adr_copy_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, C.c_void_p(st))
    if code != ADR_OK:
        raise ADRError(code, "adr_copy_probe failed")


def line_solve(off, lo, di, up, rhs, x=None, singular=None, pivot_tol=0.0, stream=None, entry="adr_line_solve"):
    """Batched tridiagonal solve on given rows (include/adr.h adr_line_solve):
    off int64 device tensor (n_lines + 1), lo/di/up/rhs float64 device tensors;
    returns x (written into `x` when given), queued on torch's current stream."""
    import torch
    lib = load()
    for t in (off, lo, di, up, rhs):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("line_solve: contiguous device tensors")
    if off.dtype != torch.int64 or any(t.dtype != torch.float64 for t in (lo, di, up, rhs)):
        raise ValueError("line_solve: int64 offsets and float64 rows")
    n_lines = off.numel() - 1
    n_rows = rhs.numel()
    if x is None:
        x = torch.empty_like(rhs)
    st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    code = getattr(lib, entry)(n_lines, n_rows, C.c_void_p(off.data_ptr()), C.c_void_p(lo.data_ptr()),
                               C.c_void_p(di.data_ptr()), C.c_void_p(up.data_ptr()), C.c_void_p(rhs.data_ptr()),
                               C.c_void_p(x.data_ptr()),
                               C.c_void_p(singular.data_ptr()) if singular is not None else None,
                               float(pivot_tol), C.c_void_p(st))
    if code != ADR_OK:
        raise ADRError(code, lib.adr_last_error(None).decode())
    return x


def _kind(v):
    """options.transfer / options.increments from "grid", "direct" (or the raw value)."""
    return {"grid": 0, "direct": 1}[v] if isinstance(v, str) else int(v)


class Solver:
    """One context over a batch of problems (workloads.Problem-like objects)."""

    def __init__(self, problems, precision="fp64", theta=1.0, dt=0.05, fp32_sweeps=3,
                 stream=None, timing=False, host_only=False, graph=False, adaptive=False, split_lines=False,
                 pivot_tol=0.0, splitting="lie", stabilize=False, krylov=0, transfer="grid", increments="grid"):
        self.lib = load()
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self._keep = []
        arr = self._structs(problems)
        if stream is None and not host_only:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        prec = {"fp64": PREC_FP64, "fp32": PREC_FP32_LINES}[precision]
        opt = Options(prec, int(fp32_sweeps), float(theta), float(dt),
                      C.c_void_p(stream) if stream else None, int(bool(timing)), int(bool(host_only)),
                      int(bool(graph)), int(bool(adaptive)), int(split_lines), float(pivot_tol),
                      {"lie": 0, "strang": 1}[splitting], int(bool(stabilize)), int(krylov),
                      _kind(transfer), _kind(increments))
        self.n = len(problems)
        self.ctx = C.c_void_p()
        st = self.lib.adr_setup(arr, self.n, C.byref(opt), C.byref(self.ctx))
        if st != ADR_OK:
            raise ADRError(st, self.lib.adr_last_error(None).decode())
        self.host_only = host_only
        self.precision = precision

    def _structs(self, problems):
        arr = (Problem * len(problems))()
        def arr_or_none(v):
            if v is None:
                return None
            a = np.ascontiguousarray(v, np.float64).ravel()
            self._keep.append(a)
            return _dptr(a)

        for k, p in enumerate(problems):
            f = np.ascontiguousarray(p.f, np.float64).ravel()
            dp = np.ascontiguousarray(np.asarray(p.dom_params, np.float64).ravel())
            self._keep += [f, dp]
            a, b, c, d = p.box
            # beta as given, else (both None) from the stream function psi
            b1, b2 = arr_or_none(p.beta1), arr_or_none(p.beta2)
            psi = arr_or_none(getattr(p, "psi", None)) if (b1 is None and b2 is None) else None
            arr[k] = Problem(p.nx, p.ny, a, b, c, d, int(p.domain), int(dp.size),
                             _dptr(dp) if dp.size else None, float(p.mu), float(p.sigma),
                             b1, b2, _dptr(f), arr_or_none(getattr(p, "g", None)), psi)
        return arr

    def update(self, problems):
        """New mu, sigma, f on the same curves (same grids and domains)."""
        self._keep = []
        arr = self._structs(list(problems))
        self._check(self.lib.adr_update(self.ctx, arr, len(problems)))

    def _check(self, st, ok=(ADR_OK,)):
        if st not in ok:
            raise ADRError(st, self.lib.adr_last_error(self.ctx).decode())
        return st

    def layout(self):
        off = np.zeros(self.n + 1, np.int64)
        self._check(self.lib.adr_layout(self.ctx, off.ctypes.data_as(C.POINTER(C.c_int64))))
        return off

    def counts(self):
        v = [C.c_int64() for _ in range(5)]
        self._check(self.lib.adr_counts(self.ctx, *[C.byref(x) for x in v]))
        return dict(grid_unknowns=v[0].value, lines_b=v[1].value, lines_g=v[2].value,
                    line_unknowns_b=v[3].value, line_unknowns_g=v[4].value)

    def set_timing(self, on):
        self._check(self.lib.adr_set_timing(self.ctx, int(bool(on))))

    def autotune(self, work, max_iters, tol):
        """Times the solve with one line launch and with one per length bucket
        (in turn, and on concurrent streams), then each candidate schedule (fixed FP32-sweep counts, adaptive maxima)
        on `work` (overwritten), and keeps the fastest; returns (count or
        maximum, adaptive, ms, split_lines: 0 one launch, 1 per bucket, 2 per
        bucket on concurrent streams, shapes: the workgroup shape of each length
        bucket, krylov: 0 or the GMRES restart length, increments: 0 grid, 1
        direct-transfer increment sweeps)."""
        best = C.c_int32()
        ad = C.c_int32()
        ms = C.c_double()
        sp = C.c_int32()
        sh = (C.c_int32 * 5)()
        kr = C.c_int32()
        inc = C.c_int32()
        self._check(self.lib.adr_autotune(self.ctx, _device_ptr(work), int(max_iters), float(tol),
                                          C.byref(best), C.byref(ad), C.byref(ms), C.byref(sp), sh, C.byref(kr),
                                          C.byref(inc)))
        return best.value, bool(ad.value), ms.value, int(sp.value), list(sh), int(kr.value), int(inc.value)

    def set_graph(self, on):
        """Replay the stationary solve's blocks from HIP graphs (include/adr.h)."""
        self._check(self.lib.adr_set_graph(self.ctx, int(bool(on))))

    def set_line_shapes(self, shapes):
        """Workgroup shape of each of the 5 length buckets (include/adr.h)."""
        arr = (C.c_int32 * 5)(*[int(v) for v in shapes])
        self._check(self.lib.adr_set_line_shapes(self.ctx, arr))

    def split_iterate(self, u, max_iters, tol):
        iters = np.zeros(self.n, np.int32)
        rel = np.zeros(self.n, np.float64)
        st = self.lib.adr_split_iterate(self.ctx, _device_ptr(u), int(max_iters), float(tol),
                                        iters.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(rel))
        self._check(st, ok=(ADR_OK, ADR_ENOTCONV))
        return iters, rel, st

    def split_iterate_judged(self, u, fallback, max_iters, tol):
        """split_iterate from u; instances whose start has a residual not below
        the fallback's restart from the fallback (include/adr.h).  Returns
        iters, rel, status, used_fallback."""
        iters = np.zeros(self.n, np.int32)
        rel = np.zeros(self.n, np.float64)
        used = np.zeros(self.n, np.int32)
        st = self.lib.adr_split_iterate_judged(self.ctx, _device_ptr(u), _device_ptr(fallback), int(max_iters),
                                               float(tol), iters.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(rel),
                                               used.ctypes.data_as(C.POINTER(C.c_int32)))
        self._check(st, ok=(ADR_OK, ADR_ENOTCONV))
        return iters, rel, st, used

    def time_step(self, u, theta, dt, nsteps, inner_max=0, inner_tol=0.0):
        """nsteps time steps of eq. (7)/(10) on u; with inner_max > 0 each implicit
        Euler step is iterated to inner_tol, and the per-step sweep counts
        (nsteps x n) and the status are returned."""
        if inner_max <= 0:
            self._check(self.lib.adr_time_step(self.ctx, _device_ptr(u), float(theta), float(dt), int(nsteps),
                                               0, 0.0, None))
            return None
        it = np.zeros(max(int(nsteps), 0) * self.n, np.int32)
        st = self.lib.adr_time_step(self.ctx, _device_ptr(u), float(theta), float(dt), int(nsteps),
                                    int(inner_max), float(inner_tol), it.ctypes.data_as(C.POINTER(C.c_int32)))
        self._check(st, ok=(ADR_OK, ADR_ENOTCONV))
        return it.reshape(max(int(nsteps), 0), self.n), st

    def residual(self, u, allow_nonfinite=False):
        """Per-instance relative residual; with allow_nonfinite a non-finite
        entry is returned (as inf/nan) instead of raised."""
        rel = np.zeros(self.n, np.float64)
        ok = (ADR_OK, ADR_ENONFINITE) if allow_nonfinite else (ADR_OK,)
        self._check(self.lib.adr_residual(self.ctx, _device_ptr(u), _dptr(rel)), ok)
        return rel

    def initial_guess(self, u):
        self._check(self.lib.adr_initial_guess(self.ctx, _device_ptr(u)))

    def export_lines(self, inst, family):
        nl, nn = C.c_int64(), C.c_int64()
        self._check(self.lib.adr_export_lines(self.ctx, inst, family, C.byref(nl), C.byref(nn),
                                              None, None, None))
        off = np.zeros(nl.value + 1, np.int64)
        x = np.zeros(nn.value)
        y = np.zeros(nn.value)
        self._check(self.lib.adr_export_lines(self.ctx, inst, family, None, None,
                                              off.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(x), _dptr(y)))
        return off, x, y

    def export_scatter(self, inst, family, with_gb=False):
        """Scatter stencil rows (host-only contexts): node, k, ca, cb [, gb]."""
        nr = C.c_int64()
        self._check(self.lib.adr_export_scatter(self.ctx, inst, family, C.byref(nr), None, None, None, None, None))
        n = nr.value
        node = np.zeros(n, np.int32)
        k = np.zeros(4 * n, np.int32)
        ca = np.zeros(4 * n)
        cb = np.zeros(4 * n)
        gb = np.zeros(n)
        i32p = C.POINTER(C.c_int32)
        self._check(self.lib.adr_export_scatter(self.ctx, inst, family, None, node.ctypes.data_as(i32p),
                                                k.ctypes.data_as(i32p), _dptr(ca), _dptr(cb), _dptr(gb)))
        out = (node, k.reshape(n, 4), ca.reshape(n, 4), cb.reshape(n, 4))
        return out + (gb,) if with_gb else out

    def export_scatter_factors(self, inst, family):
        """The scatter stencil's factors (host-only contexts): wh (n), lam (n x 2), t (n x 4)."""
        nr = C.c_int64()
        self._check(self.lib.adr_export_scatter_factors(self.ctx, inst, family, C.byref(nr), None, None, None))
        n = nr.value
        wh = np.zeros(n)
        lam = np.zeros(2 * n)
        t = np.zeros(4 * n)
        self._check(self.lib.adr_export_scatter_factors(self.ctx, inst, family, None, _dptr(wh), _dptr(lam), _dptr(t)))
        return wh, lam.reshape(n, 2), t.reshape(n, 4)

    def export_direct(self, inst, family):
        """Direct-transfer records (host-only contexts with transfer="direct"):
        k (n_nodes x 2) and w (n_nodes x 4), node indices local to the instance."""
        nn = C.c_int64()
        self._check(self.lib.adr_export_direct(self.ctx, inst, family, C.byref(nn), None, None))
        n = nn.value
        k = np.zeros(2 * n, np.int32)
        w = np.zeros(4 * n)
        self._check(self.lib.adr_export_direct(self.ctx, inst, family, None, k.ctypes.data_as(C.POINTER(C.c_int32)),
                                               _dptr(w)))
        return k.reshape(n, 2), w.reshape(n, 4)

    def export_direct_packed(self, inst, family):
        """The same records as the FP32 sweeps receive them (include/adr.h):
        k0 (int32), kd (int16), wp (uint32) per node."""
        nn = C.c_int64()
        self._check(self.lib.adr_export_direct_packed(self.ctx, inst, family, C.byref(nn), None, None, None))
        n = nn.value
        k0 = np.zeros(n, np.int32)
        kd = np.zeros(n, np.int16)
        wp = np.zeros(n, np.uint32)
        self._check(self.lib.adr_export_direct_packed(self.ctx, inst, family, None,
                                                      k0.ctypes.data_as(C.POINTER(C.c_int32)),
                                                      kd.ctypes.data_as(C.POINTER(C.c_int16)),
                                                      wp.ctypes.data_as(C.POINTER(C.c_uint32))))
        return k0, kd, wp

    def kernel_times(self, precision="fp64", reset=True, work=False):
        """Per kernel class: (ms, launches), or (ms, launches, work) with work=True."""
        ms = np.zeros(5)
        cnt = np.zeros(5, np.int64)
        wk = np.zeros(5, np.int64)
        i64p = C.POINTER(C.c_int64)
        self._check(self.lib.adr_kernel_times(self.ctx, {"fp64": 0, "fp32": 1}[precision], _dptr(ms),
                                              cnt.ctypes.data_as(i64p), wk.ctypes.data_as(i64p),
                                              int(bool(reset))))
        if work:
            return {k: (float(ms[i]), int(cnt[i]), int(wk[i])) for i, k in enumerate(KERNEL_CLASSES)}
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def close(self):
        if self.ctx:
            self.lib.adr_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ----------------------------------------------------------------------------
# learned warm start (include/adrnn.h)
NN_EXPORTS = ("adrnn_param_count", "adrnn_create", "adrnn_destroy", "adrnn_set_params", "adrnn_get_params",
              "adrnn_pack", "adrnn_forward", "adrnn_grads", "adrnn_adam", "adrnn_train_step", "adrnn_loss_sum",
              "adrnn_warm_start", "adrnn_restrict", "adrnn_warm_start_prolong", "adrnn_mfma_probe",
              "adrnn_last_error")

_nn_ready = False


def _load_nn():
    global _nn_ready
    lib = load()
    if _nn_ready:
        return lib
    i32, vp, P = C.c_int32, C.c_void_p, C.POINTER
    lib.adrnn_param_count.restype = C.c_int64
    lib.adrnn_create.argtypes = [i32, i32, i32, vp, P(vp)]
    lib.adrnn_destroy.argtypes = [vp]
    lib.adrnn_set_params.argtypes = [vp, vp]
    lib.adrnn_get_params.argtypes = [vp, vp]
    lib.adrnn_pack.argtypes = [vp, i32, vp, vp, vp, P(C.c_double), vp, vp, vp, vp]
    lib.adrnn_forward.argtypes = [vp, i32, vp, vp]
    lib.adrnn_grads.argtypes = [vp, i32, vp, vp, vp, vp, P(C.c_double)]
    lib.adrnn_adam.argtypes = [vp, vp, C.c_float]
    lib.adrnn_train_step.argtypes = [vp, i32, vp, vp, vp, C.c_float, P(C.c_double)]
    lib.adrnn_loss_sum.argtypes = [vp, P(C.c_double), P(C.c_int64), i32]
    lib.adrnn_warm_start.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    lib.adrnn_restrict.argtypes = [vp, i32, i32, vp, vp]
    lib.adrnn_warm_start_prolong.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
    lib.adrnn_mfma_probe.argtypes = [vp, vp, vp, vp]
    lib.adrnn_last_error.argtypes = [vp]
    lib.adrnn_last_error.restype = C.c_char_p
    for n in NN_EXPORTS:
        if n not in ("adrnn_param_count", "adrnn_last_error"):
            getattr(lib, n).restype = i32
    _nn_ready = True
    return lib


def _dp(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Net:
    """Warm-start network context (H x W images, batches up to max_batch)."""

    def __init__(self, H, W, max_batch, stream=None):
        import torch
        self.lib = _load_nn()
        self.H, self.W, self.maxB = H, W, max_batch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.ctx = C.c_void_p()
        st = self.lib.adrnn_create(H, W, max_batch, C.c_void_p(stream) if stream else None, C.byref(self.ctx))
        if st != ADR_OK:
            raise ADRError(st, "adrnn_create failed")
        self.n_params = int(self.lib.adrnn_param_count())

    def _check(self, st):
        if st != ADR_OK:
            raise ADRError(st, self.lib.adrnn_last_error(self.ctx).decode())

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        assert p.size == self.n_params
        self._check(self.lib.adrnn_set_params(self.ctx, p.ctypes.data_as(C.c_void_p)))

    def get_params(self):
        p = np.zeros(self.n_params, np.float32)
        self._check(self.lib.adrnn_get_params(self.ctx, p.ctypes.data_as(C.c_void_p)))
        return p

    def pack(self, B, f, s, mask, mu, u_star=None):
        import torch
        HW = self.H * self.W
        x0 = torch.empty(B * HW * 4, dtype=torch.int16, device="cuda")
        tgt = torch.empty(B * HW, dtype=torch.float32, device="cuda") if u_star is not None else None
        sn = torch.empty(B, dtype=torch.float64, device="cuda")
        mu = np.ascontiguousarray(mu, np.float64)
        self._check(self.lib.adrnn_pack(self.ctx, B, _dp(f), _dp(s), _dp(mask), mu.ctypes.data_as(C.POINTER(C.c_double)),
                                        _dp(u_star), _dp(x0), _dp(tgt), _dp(sn)))
        return x0, tgt, sn

    def forward(self, B, x0, out=None):
        import torch
        if out is None:
            out = torch.empty(B * self.H * self.W, dtype=torch.float32, device="cuda")
        self._check(self.lib.adrnn_forward(self.ctx, B, _dp(x0), _dp(out)))
        return out

    def grads(self, B, x0, target, mask):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = C.c_double()
        self._check(self.lib.adrnn_grads(self.ctx, B, _dp(x0), _dp(target), _dp(mask), _dp(g), C.byref(loss)))
        return g, loss.value

    def adam(self, grads, lr):
        self._check(self.lib.adrnn_adam(self.ctx, _dp(grads), float(lr)))

    def train_step(self, B, x0, target, mask, lr, want_loss=True):
        """One Adam step; returns the batch loss (a stream synchronisation), or
        None with want_loss=False (asynchronous; see loss_sum)."""
        loss = C.c_double()
        self._check(self.lib.adrnn_train_step(self.ctx, B, _dp(x0), _dp(target), _dp(mask), float(lr),
                                              C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def loss_sum(self, reset=True):
        """(sum, count) of the losses since the last reset (synchronises)."""
        sm = C.c_double()
        n = C.c_int64()
        self._check(self.lib.adrnn_loss_sum(self.ctx, C.byref(sm), C.byref(n), int(bool(reset))))
        return sm.value, n.value

    def warm_start(self, B, s, s_norm, out, mask, u):
        self._check(self.lib.adrnn_warm_start(self.ctx, B, _dp(s), _dp(s_norm), _dp(out), _dp(mask), _dp(u)))

    def fine_shape(self, r):
        """Fine grid (rows, columns) whose every r-th node is this context's grid."""
        return r * (self.H - 1) + 1, r * (self.W - 1) + 1

    def restrict(self, B, r, fine, coarse=None):
        """Coarse FP64 grids (B*H*W) from fine FP64 grids (B*Hf*Wf); include/adrnn.h."""
        import torch
        if coarse is None:
            coarse = torch.empty(B * self.H * self.W, dtype=torch.float64, device="cuda")
        self._check(self.lib.adrnn_restrict(self.ctx, B, r, _dp(fine), _dp(coarse)))
        return coarse

    def warm_start_prolong(self, B, r, s, s_norm, out, mask, u):
        """u (fine) = s + |s|_inf * bilinear(out) on the fine mask; include/adrnn.h."""
        self._check(self.lib.adrnn_warm_start_prolong(self.ctx, B, r, _dp(s), _dp(s_norm), _dp(out), _dp(mask),
                                                      _dp(u)))

    def close(self):
        if self.ctx:
            self.lib.adrnn_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mfma_probe(A_bf16_bits, B_bf16_bits):
    """D = A @ B through the matrix-core path (16x16 BF16 bit patterns as int16 tensors)."""
    import torch
    lib = _load_nn()
    D = torch.empty(256, dtype=torch.float32, device="cuda")
    st = lib.adrnn_mfma_probe(_dp(A_bf16_bits), _dp(B_bf16_bits), _dp(D),
                              C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != ADR_OK:
        raise ADRError(st, "mfma probe failed")
    return D
