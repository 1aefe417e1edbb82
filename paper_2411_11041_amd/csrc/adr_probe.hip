// Measurement export: a plain device copy for the HBM roofline (the measured
// counterpart of the vendor bandwidth).  Not part of the solver path.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/adr.h"

namespace {

// dst = src, n 16-byte words, one word per thread (a grid of n / 256
// workgroups: on gfx950 this streams faster than grid-stride loops, 6.2 TB/s
// against 4.0-5.4 measured for those)
__global__ __launch_bounds__(256) void k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n) {
    const size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace

extern "C" adr_status adr_copy_probe(const void *src, void *dst, int64_t bytes, void *stream) {
    if (!src || !dst || bytes < 0 || (bytes & 15) || (reinterpret_cast<uintptr_t>(src) & 15) ||
        (reinterpret_cast<uintptr_t>(dst) & 15))
        return ADR_EINVAL;
    if (bytes == 0) return ADR_OK;
    const size_t n = static_cast<size_t>(bytes) / 16;
    const size_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffffu) return ADR_EINVAL;
    hipLaunchKernelGGL(k_copy, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n);
    return hipGetLastError() == hipSuccess ? ADR_OK : ADR_EDEVICE;
}
