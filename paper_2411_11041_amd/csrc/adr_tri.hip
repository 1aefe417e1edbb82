// Batched tridiagonal solve on given rows (the line systems of eq. (16)-(19)
// with caller-supplied coefficients), for systems of any length.
//
// Each system is cut into chunks of kChunk consecutive rows; the last row of
// every chunk but the system's last is a separator.  Three passes:
//  1. one thread per chunk expresses the chunk's first and last interior rows
//     through the two separators around it (x = y + a S_left + g S_right): a
//     forward elimination gives the last row, a backward one the first;
//  2. the separators of a system then satisfy a reduced tridiagonal system,
//     one row per separator, solved by one thread per system (Thomas);
//  3. every chunk folds its two separators into its end rows and solves its
//     interior rows in registers.
// The chunk expressions and the reduced solution live in device scratch taken
// from the stream-ordered allocator for the call.  No pivoting (as the line
// solver of the sweeps): a pivot that is not finite or falls below pivot_tol
// times its row's scale flags the system.
#include <hip/hip_runtime.h>

#include <string>

#include "adr_internal.h"
#include "adr_tri.h"

namespace adr_tri {

constexpr int kThreads = 256;

__device__ inline bool bad_pivot(double den, double scale, double tol) {
    return !(fabs(den) > tol * scale);  // also true for NaN
}

// chunk_start[l] = chunks of systems 0..l-1 (one workgroup); flags cleared.
__global__ __launch_bounds__(kThreads) void k_tri_chunks(const int64_t *__restrict__ off, int64_t n_lines,
                                                         int64_t *__restrict__ cs, int32_t *__restrict__ singular) {
    __shared__ int64_t part[kThreads];
    const int t = threadIdx.x;
    const int64_t per = (n_lines + kThreads - 1) / kThreads;
    const int64_t l0 = t * per < n_lines ? t * per : n_lines;
    const int64_t l1 = l0 + per < n_lines ? l0 + per : n_lines;
    int64_t s = 0;
    for (int64_t l = l0; l < l1; ++l) {
        s += (off[l + 1] - off[l] + kChunk - 1) / kChunk;
        if (singular) singular[l] = 0;
    }
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int k = 0; k < kThreads; ++k) {
            const int64_t v = part[k];
            part[k] = acc;
            acc += v;
        }
        cs[n_lines] = acc;
    }
    __syncthreads();
    int64_t acc = part[t];
    for (int64_t l = l0; l < l1; ++l) {
        cs[l] = acc;
        acc += (off[l + 1] - off[l] + kChunk - 1) / kChunk;
    }
}

// the system of chunk c: the last l with cs[l] <= c (cs is non-decreasing)
__device__ inline int64_t line_of(const int64_t *__restrict__ cs, int64_t n_lines, int64_t c) {
    int64_t lo = 0, hi = n_lines - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (cs[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct Chunk {
    int64_t r0, r1, e;  // rows r0 .. r1-1; interior rows r0 .. e-1 (e = r1 - 1 with a separator)
    bool first, last;
};

__device__ inline Chunk chunk_rows(const int64_t *__restrict__ off, const int64_t *__restrict__ cs, int64_t l,
                                   int64_t c) {
    const int64_t q = c - cs[l], nq = cs[l + 1] - cs[l];
    Chunk k;
    k.r0 = off[l] + q * kChunk;
    k.first = q == 0;
    k.last = q + 1 == nq;
    k.r1 = k.last ? off[l + 1] : k.r0 + kChunk;
    k.e = k.last ? k.r1 : k.r1 - 1;
    return k;
}

// Pass 1.  Forward over the interior rows: x_r + cp_r x_{r+1} = y_r + a_r S_left,
// so the last interior row is y + a S_left - cp S_right.  Backward: x_r + bp_r
// x_{r-1} = z_r + h_r S_right, so the first is z - bp S_left + h S_right.  The
// system's own first row has no left neighbour and its last no right one.
__global__ __launch_bounds__(kThreads) void k_tri_reduce(const int64_t *__restrict__ off, int64_t n_lines,
                                                         int64_t bound, const int64_t *__restrict__ cs,
                                                         const double *__restrict__ lo, const double *__restrict__ di,
                                                         const double *__restrict__ up, const double *__restrict__ rhs,
                                                         double *__restrict__ expr, int32_t *__restrict__ singular,
                                                         double tol) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t total = cs[n_lines];
    if (total > bound || c >= total) return;
    const int64_t l = line_of(cs, n_lines, c);
    const Chunk k = chunk_rows(off, cs, l, c);
    bool ok = true;
    double pc = 0.0, py = 0.0, pa = 0.0;
    for (int64_t r = k.r0; r < k.e; ++r) {
        const double lr = (r == k.r0 && k.first) ? 0.0 : lo[r];
        const double ur = (r == k.r1 - 1 && k.last) ? 0.0 : up[r];
        const double den = di[r] - lr * pc;
        if (bad_pivot(den, fabs(di[r]) + fabs(lr * pc), tol)) ok = false;
        const double inv = 1.0 / den;
        const double cp = ur * inv, y = (rhs[r] - lr * py) * inv, a = (r == k.r0 ? -lr : -lr * pa) * inv;
        pc = cp; py = y; pa = a;
    }
    double bp = 0.0, z = 0.0, h = 0.0;
    for (int64_t r = k.e - 1; r >= k.r0; --r) {
        const double lr = (r == k.r0 && k.first) ? 0.0 : lo[r];
        const double ur = (r == k.r1 - 1 && k.last) ? 0.0 : up[r];
        const double den = di[r] - ur * bp;
        if (bad_pivot(den, fabs(di[r]) + fabs(ur * bp), tol)) ok = false;
        const double inv = 1.0 / den;
        const double nz = (rhs[r] - ur * z) * inv, nh = (r == k.e - 1 ? -ur : -ur * h) * inv;
        bp = lr * inv; z = nz; h = nh;
    }
    double *x = expr + kExpr * c;
    x[0] = z; x[1] = -bp; x[2] = h;    // first interior row
    x[3] = py; x[4] = pa; x[5] = -pc;  // last interior row
    if (!k.last) {
        const int64_t s = k.r1 - 1;
        x[6] = lo[s]; x[7] = di[s]; x[8] = up[s]; x[9] = rhs[s];
    } else {
        x[6] = 0.0; x[7] = 1.0; x[8] = 0.0; x[9] = 0.0;
    }
    if (!ok && singular) singular[l] = 1;
}

// Pass 2.  Separator q (the last row s of chunk q) couples to chunk q's last
// interior row (yL + aL S_{q-1} + gL S_q) and chunk q+1's first (fy + fa S_q +
// fg S_{q+1}):
//   (lo aL) S_{q-1} + (di + lo gL + up fa) S_q + (up fg) S_{q+1} = rhs - lo yL - up fy.
// Thomas on one thread per system; S[c] holds chunk c's separator.
__global__ __launch_bounds__(kThreads) void k_tri_separators(int64_t n_lines, int64_t bound,
                                                             const int64_t *__restrict__ cs,
                                                             double *__restrict__ expr, double *__restrict__ S,
                                                             int32_t *__restrict__ singular, double tol) {
    const int64_t l = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (l >= n_lines || cs[n_lines] > bound) return;
    const int64_t c0 = cs[l], R = cs[l + 1] - c0 - 1;
    if (R <= 0) return;
    bool ok = true;
    double pc = 0.0, py = 0.0;
    for (int64_t q = 0; q < R; ++q) {
        double *e = expr + kExpr * (c0 + q);
        const double *en = expr + kExpr * (c0 + q + 1);
        const double a = q > 0 ? e[6] * e[4] : 0.0;
        const double b = e[7] + e[6] * e[5] + e[8] * en[1];
        const double cc = q + 1 < R ? e[8] * en[2] : 0.0;
        const double d = e[9] - e[6] * e[3] - e[8] * en[0];
        const double den = b - a * pc;
        if (bad_pivot(den, fabs(b) + fabs(a * pc), tol)) ok = false;
        const double inv = 1.0 / den;
        pc = cc * inv;
        py = (d - a * py) * inv;
        S[c0 + q] = py;
        e[6] = pc;  // the separator row is read: its slot keeps the forward factor
    }
    double xs = 0.0;
    for (int64_t q = R - 1; q >= 0; --q) {
        xs = S[c0 + q] - (q + 1 < R ? expr[kExpr * (c0 + q) + 6] * xs : 0.0);
        S[c0 + q] = xs;
    }
    if (!ok && singular) singular[l] = 1;
}

// Pass 3.  The separators folded into the end rows' right-hand sides, the
// chunk's interior rows are one small tridiagonal system, eliminated and
// substituted back in registers (fully unrolled over kChunk rows).
__global__ __launch_bounds__(kThreads) void k_tri_back(const int64_t *__restrict__ off, int64_t n_lines,
                                                       int64_t bound, const int64_t *__restrict__ cs,
                                                       const double *__restrict__ lo, const double *__restrict__ di,
                                                       const double *__restrict__ up, const double *__restrict__ rhs,
                                                       const double *__restrict__ S, double *__restrict__ x) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    const int64_t total = cs[n_lines];
    if (total > bound || c >= total) return;
    const int64_t l = line_of(cs, n_lines, c);
    const Chunk k = chunk_rows(off, cs, l, c);
    const double SL = k.first ? 0.0 : S[c - 1];
    const double SR = k.last ? 0.0 : S[c];
    const int ni = static_cast<int>(k.e - k.r0);
    double cpv[kChunk], yv[kChunk];
    double pc = 0.0, py = 0.0;
#pragma unroll
    for (int i = 0; i < kChunk; ++i) {
        if (i < ni) {
            const int64_t r = k.r0 + i;
            const double lr = i == 0 ? 0.0 : lo[r];
            const double ur = i == ni - 1 ? 0.0 : up[r];
            double d = rhs[r];
            if (i == 0 && !k.first) d -= lo[r] * SL;
            if (i == ni - 1 && !k.last) d -= up[r] * SR;
            const double inv = 1.0 / (di[r] - lr * pc);
            pc = ur * inv;
            py = (d - lr * py) * inv;
            cpv[i] = pc;
            yv[i] = py;
        }
    }
    double xn = 0.0;
#pragma unroll
    for (int i = kChunk - 1; i >= 0; --i) {
        if (i < ni) {
            xn = yv[i] - (i == ni - 1 ? 0.0 : cpv[i] * xn);
            x[k.r0 + i] = xn;
        }
    }
    if (!k.last) x[k.r1 - 1] = SR;
}

adr_status fail(adr_status code, const std::string &m) {
    adr::set_thread_error(m);
    return code;
}

adr_status check(int64_t n_lines, int64_t n_rows, const int64_t *off, const double *lo, const double *di,
                 const double *up, const double *rhs, double *x) {
    if (n_lines < 0 || n_rows < 0 || n_lines > (int64_t(1) << 31) || n_rows > (int64_t(1) << 40))
        return fail(ADR_EINVAL, "adr_line_solve: n_lines or n_rows out of range");
    if (n_lines > 0 && (!off || !lo || !di || !up || !rhs || !x))
        return fail(ADR_EINVAL, "adr_line_solve: null array");
    return ADR_OK;
}

adr_status run(int64_t n_lines, int64_t n_rows, const int64_t *off, const double *lo, const double *di,
               const double *up, const double *rhs, double *x, int32_t *singular, double pivot_tol,
               hipStream_t st, void *base) {
    const int64_t bound = n_rows / kChunk + n_lines;  // at most one partial chunk per system
    unsigned char *b = static_cast<unsigned char *>(base);
    int64_t *cs = reinterpret_cast<int64_t *>(b);
    double *expr = reinterpret_cast<double *>(b + sizeof(int64_t) * (n_lines + 1));
    double *S = expr + kExpr * bound;
    const double tol = pivot_tol > 0.0 ? pivot_tol : 64.0 * 2.220446049250313e-16;
    const unsigned gc = static_cast<unsigned>((bound + kThreads - 1) / kThreads);
    const unsigned gl = static_cast<unsigned>((n_lines + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_tri_chunks, dim3(1), dim3(kThreads), 0, st, off, n_lines, cs, singular);
    hipLaunchKernelGGL(k_tri_reduce, dim3(gc), dim3(kThreads), 0, st, off, n_lines, bound, cs, lo, di, up, rhs, expr,
                       singular, tol);
    hipLaunchKernelGGL(k_tri_separators, dim3(gl), dim3(kThreads), 0, st, n_lines, bound, cs, expr, S, singular, tol);
    hipLaunchKernelGGL(k_tri_back, dim3(gc), dim3(kThreads), 0, st, off, n_lines, bound, cs, lo, di, up, rhs, S, x);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ADR_EDEVICE, std::string("adr_line_solve: launch: ") + hipGetErrorString(e));
    return ADR_OK;
}

}  // namespace adr_tri

extern "C" adr_status adr_line_solve(int64_t n_lines, int64_t n_rows, const int64_t *off, const double *lo,
                                     const double *di, const double *up, const double *rhs, double *x,
                                     int32_t *singular, double pivot_tol, void *stream) {
    using namespace adr_tri;
    adr_status s = check(n_lines, n_rows, off, lo, di, up, rhs, x);
    if (s != ADR_OK || n_lines == 0) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    void *p = nullptr;
    hipError_t e = hipMallocAsync(&p, scratch_bytes(n_lines, n_rows), st);
    if (e != hipSuccess) return fail(ADR_ENOMEM, std::string("adr_line_solve: hipMallocAsync: ") + hipGetErrorString(e));
    s = run(n_lines, n_rows, off, lo, di, up, rhs, x, singular, pivot_tol, st, p);
    e = hipFreeAsync(p, st);
    if (s == ADR_OK && e != hipSuccess)
        return fail(ADR_EDEVICE, std::string("adr_line_solve: hipFreeAsync: ") + hipGetErrorString(e));
    return s;
}
