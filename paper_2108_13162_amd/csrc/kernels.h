// Device kernels of the sub-structured CG and their host-side launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch_shape.h"

namespace ss {

// Status of the device-resident CG run.
enum : int32_t {
    ST_RUNNING = 0,
    ST_CONVERGED = 1,
    ST_MAXIT = 2,
    ST_BREAKDOWN = 3,
    ST_ZERO_RHS = 4,
};

// Scalars of one CG run, in device memory, so that iterations run without
// the host.  (r, r) and the iteration count live in two slots: the kernel of
// a step reads slot c and its workgroup 0 writes slot 1 - c, so no workgroup
// ever reads a value that another workgroup of the same kernel is writing.
// `status` is accessed with atomic loads / stores inside kernels.
struct DevState {
    double rr[2];      // (r, r) of the current residual (weighted local dot), by slot
    double rz[2];      // (r, z), z = M^{-1} r (equal to (r, r) without preconditioner), by slot
    int32_t iter[2];   // completed CG iterations, by slot
    double bb;         // (b, b)
    double tol;        // relative tolerance of the run
    double stop;       // CG continues while sqrt(rr) > stop
    double alpha[2];   // alpha of the update of slot c, for the x update of the step of slot c
                       // (0 when the run had stopped before that update)
    double beta, pAp;  // last scalars (report only)
    double rr_last;    // latest (r, r) (report; read by the host and the next residual step)
    int32_t iter_last; // latest iteration count (same)
    int32_t kmax;      // iteration limit
    int32_t status;    // ST_*
    int32_t hist_cap;  // entries of hist
    double *hist;      // ||r_k|| / ||b||, device, or nullptr
    // residual replacement (FP32 CG of an SS_FP32_RU solve)
    double rref;       // ||b - A x|| at the last replacement (or start)
    double delta;      // replace once sqrt(rr) <= delta * rref
    int32_t refresh;   // decision of the current chunk end
    int32_t nrefresh;  // replacements made
    int32_t restarts;  // residual recomputations that restarted CG (one-launch solve)
};


// The block-diagonal matrix of all local matrices in device position order.
//  SELL-64: rows in chunks of 64 consecutive positions (one row per lane of a
//    wave), entry j of the chunk's rows stored contiguously (column-major
//    inside the chunk), chunk length = longest row of the chunk, padded
//    entries masked by the row length.  Chunks are stored in processing order
//    (cpos = first position of each), which spreads the interface chunks
//    evenly over the persistent workgroups.
//  CSR tiles: plain CSR cut into row tiles of at most tile_nnz entries.
//  SELL column positions are stored per chunk either in 16 bits (col16: bit
//  15 picks one of the chunk's two window bases, bits 0-14 the offset from
//  it; used when every entry of the chunk falls in the two 32768-position
//  windows) or as int32 positions (col).
struct Mat {
    int32_t fmt;
    int32_t nrows;
    int32_t grid;                 // persistent grid of the SpMV kernels (multiple of 8)
    const int32_t *col;           // column positions (CSR order; SELL: wide chunks)
    const void *val;              // values, double or float, same order
    // SELL-64
    int32_t nchunks;
    int32_t unroll;               // entries per lane loaded before use: 5, 7, 8 or 9
    int32_t one_batch;            // 1: no chunk longer than unroll (chunks pipelined)
    int32_t band_m, nbands;       // nbands > 1: band-column product, bands of band_m columns
    const int32_t *cptr;          // [nchunks+1] start of each chunk in val
    const int32_t *ccol;          // [nchunks] >= 0: start in col16; < 0: ~start in col
    const uint16_t *col16;        // window offsets of the narrow chunks
    const int2 *cbase;            // [nchunks] the two window bases of a narrow chunk
    const int32_t *cpos;          // [nchunks] first row position of each chunk
    const uint8_t *clen;          // [nchunks] entries per row slot of the chunk
    const uint8_t *rlen;          // [nrows] entries of each row (by position)
    // offset dictionaries (one-batch matrices of at most 8 entries a row):
    // cdict[c] >= 0 names chunk c's block b, whose 16 column - row offsets are
    // dtab[16 b ..] and whose lane l holds the 4-bit offset indices of slots
    // 0..U-1 in dword[64 b + l] (with U <= 7 its top 4 bits hold the row's
    // length); inside each SpMV workgroup's range these chunks come first.
    // nullptr: none.
    // Rows of several load batches (dict_batches > 0): the wide kind, 64
    // offsets a block (dtab[64 b ..]), and for batch j of block b lane l's two
    // words of 6-bit indices of the batch's slots at dword[2 ((b
    // dict_batches + j) 64 + l) ..].
    const int32_t *cdict;
    const int32_t *dtab;
    const uint32_t *dword;
    int32_t dict_batches;
    // CSR tiles
    const int32_t *rowptr;        // [nrows+1]
    const int32_t *tile_row;      // [ntiles+1]
    int32_t ntiles, tile_nnz;
};

// The CG step is split (p formed by k_pstep, then the SpMV on it) for SELL
// storage whose rows take several load batches; one-batch matrices keep the
// fused, pipelined step.
inline bool split_step(const Mat &A) { return A.fmt == FMT_SELL && !A.one_batch; }

// Device position order: [0, n_own) owned interface copies, [n_own, n_if)
// the other interface copies, [n_if, n_loc) the interior positions of every
// sub-domain.  pos_grp[c] = interface node of copy c (c < n_if).  The update
// and residual kernels give one batch of kUI * kBS positions to each
// workgroup, interface batches first.
struct Iface {
    int32_t n_loc, n_own, n_if;
    int32_t grid;                 // workgroups of the update kernels (one per kUI * kBS positions)
    const int32_t *pos_grp, *copy_ptr, *copy_pos;
    int32_t ngamma;
    const double *dinv;           // Jacobi: 1 / a_ii of every position, or nullptr (no preconditioner)
};

// Partial sums of the reductions of a CG iteration.
struct Partials {
    double *a;   // (p, A_s p), one per SpMV workgroup (count = Mat::grid)
    double *b;   // (r, r), one per update workgroup (count = Iface::grid)
    int32_t na, nb;
    double *b2;  // (r, z) with the Jacobi preconditioner (same count as b), else nullptr
};

// ---- launchers (all asynchronous on the given stream) ---------------------
// Local copies of a global vector (each copy gets the node's value, converted
// to XT with round-to-nearest-even).
template <typename ST, typename XT>
void launch_gather(hipStream_t s, int32_t n_loc, const int32_t *l2g, const ST *src, XT *dst);
// Global vector from the owned copies; writes zeros if `state` says b = 0.
template <typename XT, typename DT>
void launch_scatter(hipStream_t s, int32_t n, const int32_t *g2own, const XT *src, DT *dst,
                    const DevState *state);

// q = A_bd x (no assembly).
template <typename VT, typename XT>
void launch_spmv(hipStream_t s, const Mat &A, const XT *x, XT *q);
// First CG step after a fresh residual: pout = r (p_1 = r_1), q = A_bd pout,
// partials (pout, q) -> P.a.
template <typename VT, typename XT>
void launch_spmv_first(hipStream_t s, const Mat &A, const XT *pin, const XT *r, XT *pout, XT *q, Partials P,
                       DevState *state);
// Later CG steps: each workgroup finishes (r, r) from P.b (and (r, z) from
// P.b2 when preconditioned), records the iteration (workgroup 0), tests for
// convergence, applies the previous iteration's x += alpha pin (also when
// the run stops here), then pout = r + beta pin (pass z as r when
// preconditioned), q = A_bd pout, partials -> P.a.
template <typename VT, typename XT>
void launch_spmv_step(hipStream_t s, const Mat &A, const XT *pin, const XT *r, XT *pout, XT *q, XT *x, Partials P,
                      DevState *state, int slot);
// Interface assembly in place: every copy of an interface node gets the sum of
// all its copies (ascending sub-domain).
template <typename XT>
void launch_iface_sum(hipStream_t s, const Iface &I, XT *q);
// Each workgroup finishes (p, A p) from P.a -> alpha (recorded in the state
// for the next step's x update), then assembly, r -= alpha q and partials
// (r, r) -> P.b; with I.dinv also z = D^{-1} r and (r, z) -> P.b2.
template <typename XT>
void launch_update(hipStream_t s, const Iface &I, XT *r, XT *z, const XT *q, Partials P, DevState *state, int slot);
// Fresh residual r = b - assemble(q), z = D^{-1} r (with I.dinv), p0 = z
// (= r without preconditioner), then one workgroup finishes (r, r), (r, z)
// [and (b, b) when `first`] and sets the status.  partial: 3 * I.grid.
template <typename XT>
void launch_residual(hipStream_t s, const Iface &I, const XT *b, const XT *q, XT *r, XT *z, XT *p0,
                     double *partial, DevState *state, bool first);

// FP32-value iterative refinement.  ir_prepare: inner right-hand side
// rin = (XT)(r64 / s) with s = sqrt(outer (r, r)), p0 = rin, d = 0, then one
// workgroup sets up the inner run's state (stop = inner_tol * ||rin||, limit
// min(iterations + inner_maxit, maxit), history scaled to ||r|| / ||b||).
template <typename XT>
void launch_ir_prepare(hipStream_t s, const Iface &I, const double *r64, XT *rin, XT *p0, XT *d, double *partial,
                       const DevState *outer, DevState *inner, double inner_tol, int32_t inner_maxit, int32_t maxit);
// x64 += s * d (every copy), iteration count back to the outer state; an
// inner breakdown skips the correction and marks the outer state.
template <typename XT>
void launch_ir_accumulate(hipStream_t s, int32_t n_loc, double *x64, const XT *d, const DevState *inner,
                          DevState *outer);

// FP32 CG with FP64 residual replacement.  Start (after a fresh FP64
// residual r64 in the outer state): rin = (XT) r64, d = 0, inner state from
// the outer one (unscaled: same stop and (b, b)), rref = ||r64||.
template <typename XT>
void launch_ru_start(hipStream_t s, const Iface &I, const double *r64, XT *rin, XT *d, double *partial,
                     const DevState *outer, DevState *inner, double delta);
// Chunk end (graph-captured): decide whether to replace; if so x64 += d,
// d = 0, q64 = A x64 (FP64 values), r64 = b - assemble(q64), rin = (XT) r64,
// (rin, rin) -> inner slot 0, true residual -> stopping test (CONVERGED ends
// the run).  Every launch returns at once when no replacement is due.
template <typename XT>
void launch_ru_refresh(hipStream_t s, const Iface &I, const Mat &A64, double *x64, XT *d, const double *b64,
                       double *q64, double *r64, XT *rin, double *partial, DevState *inner, DevState *outer);
// After the run: x64 += d, d = 0, iteration count to the outer state, a
// breakdown propagated.
template <typename XT>
void launch_ru_fold(hipStream_t s, int32_t n_loc, double *x64, XT *d, const DevState *inner, DevState *outer);

// Adjoint gradient on the pattern: dvals[nzmap[k]] = -lambda[row] x[col] for
// every stored (non-padding) entry k of A in device order.
void launch_grad_vals(hipStream_t s, const Mat &A, const int32_t *nzmap, const int32_t *l2g, const double *lambda,
                      const double *x, double *dvals);
// dinv[c] = 1 / val_glob[dnz[c]] (the Jacobi preconditioner from new values).
void launch_set_dinv(hipStream_t s, int32_t n_loc, const int32_t *dnz, const double *val_glob, double *dinv);
// val64[k] = val_glob[nzmap[k]] (0 for padding, nzmap < 0), val32 its FP32 rounding
// (val32 may be nullptr).
void launch_set_values(hipStream_t s, int64_t len, const int32_t *nzmap, const double *val_glob, double *val64,
                       float *val32);

}  // namespace ss
