// Internal interface of the batched tridiagonal solver on given rows (adr_tri.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/adr.h"

namespace adr_tri {

constexpr int kChunk = 32;  // rows per chunk (>= 2); the back-substitution holds them in registers
constexpr int kExpr = 10;   // doubles per chunk expression

// Scratch layout: chunk_start (n_lines + 1 int64), then per chunk kExpr
// doubles (first interior row y, a, g; last interior row y, a, g; the
// separator row lo, di, up, rhs), then one double per chunk (its separator's
// value in the reduced solution), for the chunk bound n_rows / kChunk +
// n_lines.  Nothing in it needs to start at zero.
inline size_t scratch_bytes(int64_t n_lines, int64_t n_rows) {
    const int64_t bound = n_rows / kChunk + n_lines;
    return sizeof(int64_t) * (n_lines + 1) + sizeof(double) * (kExpr + 1) * bound;
}

// Argument checks (no device call).
adr_status check(int64_t n_lines, int64_t n_rows, const int64_t *off, const double *lo, const double *di,
                 const double *up, const double *rhs, double *x);
// Queues the three passes on `stream` with the scratch at device address
// `base` (scratch_bytes(n_lines, n_rows) bytes).  No allocation.
adr_status run(int64_t n_lines, int64_t n_rows, const int64_t *off, const double *lo, const double *di,
               const double *up, const double *rhs, double *x, int32_t *singular, double pivot_tol,
               hipStream_t stream, void *base);
// Sets the thread's error message and returns code.
adr_status fail(adr_status code, const std::string &msg);

}  // namespace adr_tri
