// Launch-shape constants shared by the kernels and the host-side layout
// builder (no HIP types: the layout builder is plain C++).
#pragma once

namespace ss {

constexpr int kBS = 256;    // workgroup size of every kernel
constexpr int kUI = 2;      // positions per thread per batch in the update / residual kernels
constexpr int kNumXcd = 8;  // MI355X: workgroups are dealt round-robin to 8 XCDs

// Grid size for `work` items remapped so that each XCD gets a contiguous range.
inline int xcd_grid(int work) { return ((work + kNumXcd - 1) / kNumXcd) * kNumXcd; }

enum { FMT_SELL = 0, FMT_CSR = 1 };

}  // namespace ss
