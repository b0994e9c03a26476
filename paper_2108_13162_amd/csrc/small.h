// The one-launch solve of a small system (small.hip) and its sizing rules.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "kernels.h"

namespace ss {

// ---- one-launch solve of a small system (small.hip) --------------------------
// One workgroup of kSmallThreads threads runs the whole CG (M = I, FP64):
// each thread owns `rows` rows (t, t + kSmallThreads, ...) of the
// block-diagonal matrix, their `width` (5 or 7) value slots, column
// positions and r held in registers (the largest kernels, 6 rows of 5 and 5
// of 7, spill 52 and 92 bytes a thread); x, p, the interface products and
// the interface copy lists live in LDS.
constexpr int kSmallThreads = 768;

struct SmallMat {
    int32_t n_loc;
    int32_t n_copies;      // entries of the interface copy lists
    int32_t rows, width;   // rows per thread (see small_rows), value slots per row
    const double *val;     // [width][n_loc] slot-major, device position order, 0 past a row's length
    const uint32_t *colw;  // [(width+1)/2][n_loc] two 16-bit column positions per word (padding: the
                           // row itself); the upper half of the last word holds the row's length
};

inline size_t small_lds_bytes(int32_t n_loc, int32_t n_if, int32_t ngamma, int32_t n_copies)
{
    return sizeof(double) * (2 * (size_t)n_loc + (size_t)n_if + 2 * (kSmallThreads / 64) + 256) +
           sizeof(int32_t) * ((size_t)n_if + (size_t)ngamma + 1 + (size_t)n_copies);
}
// Rows per thread of the kernel for `rows_needed` rows of `width` slots, 0
// if none is built: width 5 up to 6 rows per thread (4608 positions), width
// 7 up to 5 (3840) -- what fits in a thread's registers without spilling at
// three waves per SIMD.
int32_t small_rows(int32_t rows_needed, int32_t width);
// The solve from the gathered b and x0 (x updated in place) to the final
// status, iteration count, (r, r), (b, b) and restart count in `state`
// (whose tol, kmax, hist and hist_cap the host set).
void launch_cg_small(hipStream_t s, const SmallMat &M, const Iface &I, const double *b, double *x,
                     DevState *state);

}  // namespace ss
