// adr_line_solve without allocation: the same three passes with their scratch
// in a fixed device array of this file, for callers that cannot allocate
// (work captured into a graph, serving loops that forbid it).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "adr_tri.h"

namespace adr_tri {
namespace {

constexpr size_t kScratchMax = size_t(16) << 20;  // bytes per device, held until the process ends
constexpr int kMaxDevices = 64;

// One copy per device.  In host code the name stands for a host-side symbol,
// not a device address: kernels get the address looked up per device below.
static __device__ __align__(256) unsigned char scratch[kScratchMax];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// The current device's copy of scratch; looked up once per device, with that
// device current.
hipError_t scratch_on_current_device(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace adr_tri

extern "C" adr_status adr_line_solve_noalloc(int64_t n_lines, int64_t n_rows, const int64_t *off, const double *lo,
                                             const double *di, const double *up, const double *rhs, double *x,
                                             int32_t *singular, double pivot_tol, void *stream) {
    using namespace adr_tri;
    adr_status s = check(n_lines, n_rows, off, lo, di, up, rhs, x);
    if (s != ADR_OK || n_lines == 0) return s;
    const size_t need = scratch_bytes(n_lines, n_rows);
    if (need > kScratchMax)
        return fail(ADR_EINVAL, "adr_line_solve_noalloc: needs " + std::to_string(need) +
                                    " bytes of scratch, more than its fixed " + std::to_string(kScratchMax) +
                                    " (about 88 B per 32 rows and 8 B per system)");
    void *p = nullptr;
    const hipError_t e = scratch_on_current_device(&p);
    if (e != hipSuccess)
        return fail(ADR_EDEVICE, std::string("adr_line_solve_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
    return run(n_lines, n_rows, off, lo, di, up, rhs, x, singular, pivot_tol, static_cast<hipStream_t>(stream), p);
}
