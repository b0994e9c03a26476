// Device kernels of the sub-structured CG and their host-side launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ss {

// Status of the device-resident CG run.
enum : int32_t {
    ST_RUNNING = 0,
    ST_CONVERGED = 1,
    ST_MAXIT = 2,
    ST_BREAKDOWN = 3,
    ST_ZERO_RHS = 4,
};

// Scalars of one CG run, kept in device memory so that a whole iteration runs
// without the host: the kernels read alpha / beta / status from here and the
// finishing workgroup of every reduction writes them.
struct DevState {
    double rr;        // (r, r) of the current residual (weighted local dot)
    double bb;        // (b, b)
    double pAp;       // (p, A p)
    double alpha;
    double beta;
    double tol;       // relative tolerance of the run
    double stop;      // CG continues while sqrt(rr) > stop
    double scale;     // IR: norm of the outer residual the inner solve started from
    int32_t iter;     // iterations done (all runs of this solve)
    int32_t kmax;     // iteration limit of the current run
    int32_t status;   // ST_*
    int32_t hist_cap; // entries of hist
    double *hist;     // ||r_k|| / ||b||, device, or nullptr
    uint32_t cnt[4];  // arrival counters of the fused reductions
};

// One workgroup of the update / residual kernels: `count` consecutive
// positions starting at `start`, all of one kind: 0 interior (owned, no
// assembly), 1 owned interface copy, 2 other interface copy.  `ifbase`
// indexes pos_grp for the first position of an interface block.
struct UpdBlock {
    int32_t start, count, kind, ifbase;
};

constexpr int kBS = 256;     // workgroup size of all streaming kernels
constexpr int kUI = 4;       // positions per thread in the update kernels
constexpr int kNumXcd = 8;   // MI355X: workgroups are dealt round-robin to 8 XCDs

// Grid size for `work` items remapped so that each XCD gets a contiguous range.
inline int xcd_grid(int work) { return ((work + kNumXcd - 1) / kNumXcd) * kNumXcd; }

struct Csr {
    const int32_t *rowptr, *colidx, *tile_row;
    const void *val;  // double or float
    int32_t ntiles, tile_nnz;
};

struct Iface {
    const UpdBlock *blk;
    int32_t nblk;
    const int32_t *pos_grp, *copy_ptr, *copy_pos;
    int32_t ngamma;
};

// ---- launchers (all asynchronous on `st`) --------------------------------
// Local copies of a global vector (each copy gets the node's value).
template <typename XT>
void launch_gather(hipStream_t s, int32_t n_loc, const int32_t *l2g, const double *src, XT *dst);
// Global vector from the owned copies; zero == true writes zeros instead.
template <typename XT>
void launch_scatter(hipStream_t s, int32_t n, const int32_t *g2own, const XT *src, double *dst, const DevState *dst_state);

// q = A_bd x (no assembly).
template <typename VT, typename XT>
void launch_spmv(hipStream_t s, const Csr &A, const XT *x, XT *q);
// CG step: pout = r + beta * pin (beta from state), q = A_bd pout,
// partial (pout, q) -> alpha.
template <typename VT, typename XT>
void launch_spmv_cg(hipStream_t s, const Csr &A, const XT *pin, const XT *r, XT *pout, XT *q, double *partial,
                    DevState *state, bool fused);
// Interface assembly in place: every copy of an interface node gets the sum of
// all its copies (ascending sub-domain).
template <typename XT>
void launch_iface_sum(hipStream_t s, const Iface &I, XT *q);
// Assembly + x += alpha p, r -= alpha q, partial (r, r) -> beta, convergence.
template <typename XT>
void launch_update(hipStream_t s, const Iface &I, XT *x, const XT *p, XT *r, const XT *q, double *partial,
                   DevState *state, bool fused);
// Fresh residual: r = b - assemble(q), p0 = r, partial (r, r) [and (b, b)].
template <typename XT>
void launch_residual(hipStream_t s, const Iface &I, const XT *b, const XT *q, XT *r, XT *p0, double *partial,
                     DevState *state, bool first, bool fused);

// Adjoint gradient on the pattern and value updates through the entry map.
void launch_grad_vals(hipStream_t s, int32_t n_loc, const int32_t *rowptr, const int32_t *colidx, const int32_t *nzmap,
                      const int32_t *l2g, const double *lambda, const double *x, double *dvals);
void launch_set_values(hipStream_t s, int64_t nnz, const int32_t *nzmap, const double *val_glob, double *val64,
                       float *val32);

}  // namespace ss
