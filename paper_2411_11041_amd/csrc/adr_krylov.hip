// Vector kernels of the GMRES acceleration of the stationary iteration: per
// instance dot products and linear combinations of FP64 grid fields in the
// blocked layout (all of an instance's entries, the ones outside its interior
// being zero in every Krylov vector).  Each instance's range is cut into
// chunks of kKChunk entries; a workgroup takes one chunk, partial sums go to
// per-chunk slots and are summed per instance in a fixed order (the results
// do not depend on scheduling).
#include <hip/hip_runtime.h>

#include "adr_kernels.h"

namespace adr {

namespace {
constexpr int kKThreads = 256;
constexpr int kKPer = 8;                       // entries per thread
constexpr int kKChunk = kKThreads * kKPer;     // entries per chunk

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// block sum of the 4 wavefronts' values (one per wave in lds[0..3]); valid in thread 0
__device__ inline double block_sum(double v, double *lds) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    return (lds[0] + lds[1]) + (lds[2] + lds[3]);
}
}  // namespace

// partial[c * kmax + i] = (z, V_i) over chunk c, i < nv
__global__ __launch_bounds__(kKThreads) void k_kdot(const double *__restrict__ z, const double *__restrict__ V,
                                                    int64_t stride, int nv, int kmax, const KChunks ch,
                                                    const int *__restrict__ done, double *__restrict__ partial) {
    __shared__ double lds[4];
    const int c = blockIdx.x;
    const int inst = ch.inst[c];
    if (done[inst]) return;
    const int64_t b = ch.begin[c], e = ch.end[c];
    double zv[kKPer];
#pragma unroll
    for (int q = 0; q < kKPer; ++q) {
        const int64_t k = b + threadIdx.x + static_cast<int64_t>(q) * kKThreads;
        zv[q] = k < e ? z[k] : 0.0;
    }
    for (int i = 0; i < nv; ++i) {
        const double *vi = V + static_cast<int64_t>(i) * stride;
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < kKPer; ++q) {
            const int64_t k = b + threadIdx.x + static_cast<int64_t>(q) * kKThreads;
            s += k < e ? zv[q] * vi[k] : 0.0;
        }
        s = block_sum(s, lds);
        if (threadIdx.x == 0) partial[static_cast<int64_t>(c) * kmax + i] = s;
    }
}

// out[inst * kmax + i] = sum over the instance's chunks (fixed order) of partial[c * kmax + i]
__global__ __launch_bounds__(kKThreads) void k_kreduce(const double *__restrict__ partial, int nv, int kmax,
                                                       const int *__restrict__ inst_chunk,
                                                       const int *__restrict__ done, double *__restrict__ out) {
    __shared__ double lds[4];
    const int inst = blockIdx.x;
    if (done[inst]) return;
    const int c0 = inst_chunk[inst], c1 = inst_chunk[inst + 1];
    for (int i = 0; i < nv; ++i) {
        double s = 0.0;
        for (int c = c0 + threadIdx.x; c < c1; c += kKThreads) s += partial[static_cast<int64_t>(c) * kmax + i];
        s = block_sum(s, lds);
        if (threadIdx.x == 0) out[static_cast<int64_t>(inst) * kmax + i] = s;
    }
}

// Arnoldi update: w = V_j - z - sum_{i < nv} coef[inst][i] V_i written to z
// (z holds T V_j on entry), with |w|^2 per chunk in partial[c * kmax].
__global__ __launch_bounds__(kKThreads) void k_kupdate(double *__restrict__ z, const double *__restrict__ V,
                                                       int64_t stride, int j, int nv, int kmax,
                                                       const double *__restrict__ coef, const KChunks ch,
                                                       const int *__restrict__ done, double *__restrict__ partial) {
    __shared__ double lds[4];
    const int c = blockIdx.x;
    const int inst = ch.inst[c];
    if (done[inst]) return;
    const int64_t b = ch.begin[c], e = ch.end[c];
    const double *cf = coef + static_cast<int64_t>(inst) * kmax;
    const double *vj = V + static_cast<int64_t>(j) * stride;
    double w[kKPer];
#pragma unroll
    for (int q = 0; q < kKPer; ++q) {
        const int64_t k = b + threadIdx.x + static_cast<int64_t>(q) * kKThreads;
        w[q] = k < e ? vj[k] - z[k] : 0.0;
    }
    for (int i = 0; i < nv; ++i) {
        const double a = cf[i];
        const double *vi = V + static_cast<int64_t>(i) * stride;
#pragma unroll
        for (int q = 0; q < kKPer; ++q) {
            const int64_t k = b + threadIdx.x + static_cast<int64_t>(q) * kKThreads;
            if (k < e) w[q] -= a * vi[k];
        }
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kKPer; ++q) {
        const int64_t k = b + threadIdx.x + static_cast<int64_t>(q) * kKThreads;
        if (k < e) {
            z[k] = w[q];
            s += w[q] * w[q];
        }
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) partial[static_cast<int64_t>(c) * kmax] = s;
}

// x += sum_{i < nv} coef[inst][i] V_i  (coef[inst][i] = 0 leaves x alone)
__global__ __launch_bounds__(kKThreads) void k_kcombine(double *__restrict__ x, const double *__restrict__ V,
                                                        int64_t stride, int nv, int kmax,
                                                        const double *__restrict__ coef, const KChunks ch,
                                                        const int *__restrict__ done) {
    const int c = blockIdx.x;
    const int inst = ch.inst[c];
    if (done[inst]) return;
    const int64_t b = ch.begin[c], e = ch.end[c];
    const double *cf = coef + static_cast<int64_t>(inst) * kmax;
#pragma unroll
    for (int q = 0; q < kKPer; ++q) {
        const int64_t k = b + threadIdx.x + static_cast<int64_t>(q) * kKThreads;
        if (k >= e) continue;
        double acc = x[k];
        for (int i = 0; i < nv; ++i) acc += cf[i] * V[static_cast<int64_t>(i) * stride + k];
        x[k] = acc;
    }
}

// v *= scale[inst * kmax] over the instance's chunks
__global__ __launch_bounds__(kKThreads) void k_kscale(double *__restrict__ v, const double *__restrict__ scale,
                                                      int kmax, const KChunks ch, const int *__restrict__ done) {
    const int c = blockIdx.x;
    const int inst = ch.inst[c];
    if (done[inst]) return;
    const int64_t b = ch.begin[c], e = ch.end[c];
    const double s = scale[static_cast<int64_t>(inst) * kmax];
#pragma unroll
    for (int q = 0; q < kKPer; ++q) {
        const int64_t k = b + threadIdx.x + static_cast<int64_t>(q) * kKThreads;
        if (k < e) v[k] *= s;
    }
}

// r[gb[s]] = phi[gb[s]] - u[gb[s]] on the interior nodes (scatter slots s < npad)
__global__ void k_kresidual(const int *__restrict__ gb, int npad, const double *__restrict__ phi,
                            const double *__restrict__ u, double *__restrict__ r) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= npad) return;
    const int g = gb[s];
    if (g < 0) return;
    r[g] = phi[g] - u[g];
}

int krylov_chunk() { return kKChunk; }

hipError_t launch_kdot(const double *z, const double *V, int64_t stride, int nv, int kmax, const KChunks &ch,
                       const int *done, double *partial, double *out, hipStream_t st) {
    if (ch.n == 0 || nv == 0) return hipSuccess;
    hipLaunchKernelGGL(k_kdot, dim3(ch.n), dim3(kKThreads), 0, st, z, V, stride, nv, kmax, ch, done, partial);
    hipLaunchKernelGGL(k_kreduce, dim3(ch.n_inst), dim3(kKThreads), 0, st, partial, nv, kmax, ch.inst_chunk, done,
                       out);
    return hipGetLastError();
}

hipError_t launch_kupdate(double *z, const double *V, int64_t stride, int j, int nv, int kmax, const double *coef,
                          const KChunks &ch, const int *done, double *partial, double *out, hipStream_t st) {
    if (ch.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_kupdate, dim3(ch.n), dim3(kKThreads), 0, st, z, V, stride, j, nv, kmax, coef, ch, done,
                       partial);
    hipLaunchKernelGGL(k_kreduce, dim3(ch.n_inst), dim3(kKThreads), 0, st, partial, 1, kmax, ch.inst_chunk, done,
                       out);
    return hipGetLastError();
}

hipError_t launch_kcombine(double *x, const double *V, int64_t stride, int nv, int kmax, const double *coef,
                           const KChunks &ch, const int *done, hipStream_t st) {
    if (ch.n == 0 || nv == 0) return hipSuccess;
    hipLaunchKernelGGL(k_kcombine, dim3(ch.n), dim3(kKThreads), 0, st, x, V, stride, nv, kmax, coef, ch, done);
    return hipGetLastError();
}

hipError_t launch_kscale(double *v, const double *scale, int kmax, const KChunks &ch, const int *done,
                         hipStream_t st) {
    if (ch.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_kscale, dim3(ch.n), dim3(kKThreads), 0, st, v, scale, kmax, ch, done);
    return hipGetLastError();
}

hipError_t launch_kresidual(const int *gb, int npad, const double *phi, const double *u, double *r,
                            hipStream_t st) {
    if (npad <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_kresidual, dim3((npad + 255) / 256), dim3(256), 0, st, gb, npad, phi, u, r);
    return hipGetLastError();
}

}  // namespace adr
