/*
 * ss.h -- C-ABI of the sub-structured Conjugate Gradient library (libss.so)
 * for AMD Instinct MI355X (gfx950).
 *
 * Method: "Parallel Sub-Structuring Methods for solving Sparse Linear Systems
 * on a cluster of GPU" (Cheik Ahamed, Magoules).  A sparse symmetric
 * positive-definite system A x = b stored in CSR (Section 2.2) is split into
 * sub-domains (sub-structuring splitting, Section 3.4) and solved by CG
 * (Algorithm 3).  Every product by A is a local SpMV in each sub-domain
 * followed by the assembly of the interface contributions (Section 4.4.1,
 * Algorithms 4 and 5); dot products are weighted local sums followed by a
 * global sum (Section 4.4.2).  All sub-domains of a partition are resident on
 * one GPU: the interface exchange is an on-device gather-sum and the global
 * sums are on-device reductions.
 *
 * Conventions for every entry point:
 *  - 0-based int32 indices; FP64 values unless stated.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are GPU
 *    memory of the device that was current when the solver was set up.
 *  - Inputs are borrowed for the duration of the call only; the library
 *    copies what it keeps.  The caller owns every buffer it passes.
 *  - Device work is ordered on the HIP stream given to the setup call;
 *    device input buffers must be ready on that stream, device outputs are
 *    complete when the call returns (the call synchronises the stream).
 *  - Handles are not thread-safe; use one handle per host thread / stream.
 *  - Return value: one of the SS_* status codes below.  On a negative code
 *    no output is valid unless stated; ss_strerror() gives a message and
 *    ss_last_error() the detail of the last failure on the calling thread.
 */
#ifndef SS_H
#define SS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
#define SS_OK 0            /* success                                        */
#define SS_NOT_CONVERGED 1 /* maxit reached; outputs hold the last iterate   */
#define SS_EINVAL (-1)     /* invalid argument or matrix (see ss_last_error) */
#define SS_ENOMEM (-2)     /* host or device allocation failed               */
#define SS_EDEVICE (-3)    /* HIP runtime error                              */
#define SS_EBREAKDOWN (-4) /* (p, A p) <= 0 or a non-finite scalar: A is not
                              SPD or the data holds NaN/Inf; x holds the last
                              finite iterate                                 */
#define SS_EUNSUPPORTED (-5)

/* ------------------------------------------------------------ matrices */
/* Global sparse matrix in CSR, host memory: rowptr[n+1] with rowptr[0] = 0
 * and rowptr[n] = nnz, colidx[nnz] strictly increasing inside each row,
 * val[nnz].  The paper's IA/JA/AA (Section 2.2), 0-based.  Solver entry
 * points require a structurally and bitwise-numerically symmetric matrix
 * (Section 3.4: S is symmetric positive-definite); violations give
 * SS_EINVAL. */
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t *rowptr;
    const int32_t *colidx;
    const double *val;
} ss_csr;

/* ---------------------------------------------------------- partitions */
enum {
    SS_PART_BOX = 0,  /* structured grid cut into boxes                    */
    SS_PART_RCB = 1,  /* weighted recursive coordinate bisection           */
    SS_PART_USER = 2, /* node -> sub-domain array given by the caller      */
    SS_PART_GRAPH = 3 /* multilevel bisection of the adjacency graph of A  */
};

typedef struct ss_part ss_part;     /* opaque, host memory */
typedef struct ss_solver ss_solver; /* opaque, owns device buffers */

/*
 * ss_partition -- pre-processing step, run once per matrix and independent
 * of the solver (Section 3: data distribution is a separate step; Section
 * 3.4: sub-structuring splitting).
 *
 * 1. Node partition P(i) in [0, nparts):
 *    BOX : grid[dim] = nodes per axis (node id = x + Mx*(y + My*z), x
 *          fastest, n must equal the product), boxes[dim] = boxes per axis,
 *          nparts must equal their product.  Box b along an axis of M nodes
 *          and B boxes starts at floor(b*M/B).  Part = bx + Bx*(by + By*bz).
 *    RCB : coords[n*dim] (row-major, host) and weights[nparts] (target
 *          relative sizes, > 0; NULL = equal).  A node set for the part range
 *          [lo,hi) is split along its widest axis (ties: lowest axis); nodes
 *          ordered by (coordinate, id); the first
 *          floor(|S| * W[lo,mid) / W[lo,hi) + 0.5) go to [lo, mid),
 *          mid = (lo+hi)/2; weight sums are sequential left to right.
 *    USER: user_part[n] with values in [0, nparts).
 *    GRAPH: no geometry needed: multilevel recursive bisection of the
 *          adjacency graph of A (off-diagonal entries = edges of weight 1):
 *          heavy-edge coarsening, a grown bisection of the coarsest graph,
 *          Fiduccia-Mattheyses refinement on the way back; each bisection
 *          splits the part range [lo,hi) at mid = lo + (hi-lo)/2 with target
 *          weights W[lo,mid) : W[mid,hi) (weights as RCB) and lets a side
 *          exceed its target by 1%.  Deterministic.
 *    Unused pointer arguments may be NULL.
 * 2. Split of the matrix into local matrices A_s (the paper's S_s, whose
 *    interface block is a partial sum, S_33 = sum_s S_33^(s)): every stored
 *    entry (i,j) goes to one sub-domain, o(i,j) = P(i) if i == j else
 *    min(P(i), P(j)), so that sum_s R_s^T A_s R_s == A exactly.
 *    V_s = {i : P(i) = s} U {i, j : o(i,j) = s}; multiplicity m_i = number
 *    of sub-domains holding i; interface Gamma = {i : m_i > 1}.
 * 3. Local numbering, concatenated over sub-domains: sub-domain s occupies
 *    positions [sub_off[s], sub_off[s+1]) ordered as interior nodes (m = 1),
 *    then interface nodes it owns (P(i) = s), then the other interface nodes
 *    it holds, each group ascending by global id.
 *
 * Errors: SS_EINVAL for an invalid CSR (see ss_csr), a non-symmetric matrix,
 * n < 1, nparts outside [1, n], inconsistent grid/boxes, a non-positive or
 * non-finite weight, a user part out of range.  *out is set only on SS_OK
 * and is released with ss_part_destroy.
 */
int ss_partition(const ss_csr *A, int32_t method, int32_t nparts, int32_t dim, const int32_t *grid,
                 const int32_t *boxes, const double *coords, const double *weights,
                 const int32_t *user_part, ss_part **out);

/* Sizes of the maps below (any pointer may be NULL).  n_loc = sum_s |V_s|,
 * n_copies = sum over interface nodes of m_i, nnz = stored entries (equal
 * to the sum of the local nnz). */
int ss_part_sizes(const ss_part *p, int32_t *nparts, int32_t *n, int32_t *n_loc, int32_t *n_gamma,
                  int32_t *n_copies, int64_t *nnz);

/* Copies the partition maps into caller-provided host arrays (any may be
 * NULL): part[n], sub_off[nparts+1], n_int[nparts] (interior count),
 * n_own[nparts] (owned interface count), l2g[n_loc] (global id of each
 * concatenated position), gamma[n_gamma] (interface nodes ascending),
 * copy_ptr[n_gamma+1] and copy_pos[n_copies] (positions of the copies of
 * gamma[g], ascending sub-domain).  These are the lists Algorithms 4 and 5
 * walk (list_s), flattened for one address space. */
int ss_part_export(const ss_part *p, int32_t *part, int32_t *sub_off, int32_t *n_int, int32_t *n_own,
                   int32_t *l2g, int32_t *gamma, int32_t *copy_ptr, int32_t *copy_pos);

/* Copies the block-diagonal CSR of all local matrices (host arrays, any may
 * be NULL): bd_rowptr[n_loc+1], bd_colidx[nnz] (concatenated positions,
 * ascending inside each row) and bd_nzmap[nnz] (index of the global stored
 * entry each local entry takes its value from). */
int ss_part_export_local(const ss_part *p, int32_t *bd_rowptr, int32_t *bd_colidx, int32_t *bd_nzmap);

void ss_part_destroy(ss_part *p);

/* --------------------------------------------------------------- solver */
typedef void *(*ss_alloc_fn)(void *ctx, size_t bytes); /* device memory, 256-byte aligned, or NULL */
typedef void (*ss_free_fn)(void *ctx, void *ptr);

enum { SS_FP64 = 0, SS_FP32_IR = 1, SS_FP32_RU = 2 };

/* Preconditioner M of Algorithm 3. */
enum {
    SS_PRECOND_NONE = 0,  /* M = I                                                */
    SS_PRECOND_JACOBI = 1 /* M = diag(A) (every copy of a node uses the node's
                             global diagonal entry, which must be positive);
                             SS_FP64 only                                        */
};

/* Solve of a small system in one launch (SS_FP64, M = I): one workgroup
 * runs every CG iteration, with the matrix in registers and p in LDS, instead
 * of two launches per iteration.  Used for systems whose local rows hold at
 * most 7 entries and number at most 4608 (rows of at most 5 entries) or 3840
 * (at most 7), within the LDS a workgroup may take.  Same method, stopping rule and outputs as the general path. */
enum {
    SS_SMALL_AUTO = 0, /* use it when the system qualifies (default) */
    SS_SMALL_OFF = 1   /* always the general path                    */
};

/* Device storage of the block-diagonal matrix of all local matrices. */
enum {
    SS_MAT_AUTO = 0, /* SELL-64 unless rows are too uneven, else CSR row tiles */
    SS_MAT_SELL = 1, /* chunks of 64 rows, one row per lane, column-major
                        (rows of at most 255 entries and fewer than 2^29 local
                        positions; otherwise CSR row tiles)                  */
    SS_MAT_CSR = 2   /* CSR cut into row tiles of tile_nnz entries             */
};

typedef struct {
    int32_t precision;   /* SS_FP64; SS_FP32_IR: FP32 values and vectors in
                            the inner CG, FP64 dots, FP64 residuals and an
                            outer iterative-refinement loop; SS_FP32_RU: the
                            same FP32 CG with FP64 residual replacement that
                            keeps the search direction                         */
    double inner_tol;    /* IR: inner relative tolerance, in (0, 1); 1e-6     */
    double ru_delta;     /* RU: replace the residual once the recursive one
                            has dropped by this factor, in [0, 1]; 0.1        */
    int32_t inner_maxit; /* IR: inner iteration cap (<= 0: unlimited)          */
    int32_t max_outer;   /* IR: outer iteration cap (<= 0: 50)                 */
    int32_t check_every; /* CG iterations between host polls (<= 0: 32)        */
    int32_t use_graph;   /* 1: replay polled chunks as HIP graphs (default);
                            0: plain launches                                  */
    int32_t tile_nnz;    /* CSR tiles: entries per tile, 0 = 2048, else one of
                            1024, 2048, 4096                                  */
    int32_t matrix_format; /* SS_MAT_*                                        */
    int32_t spmv_grid;   /* persistent SpMV workgroups, 0 = tuned default      */
    int32_t precond;     /* SS_PRECOND_*                                       */
    ss_alloc_fn alloc;   /* device allocator; NULL = hipMalloc                 */
    ss_free_fn free;     /* matching release; NULL = hipFree                   */
    void *alloc_ctx;
    int32_t small_solver; /* SS_SMALL_*                                        */
} ss_opts;

/* Fills *o with the defaults. */
void ss_opts_default(ss_opts *o);

typedef struct {
    int32_t status;           /* same as the return value of the solve      */
    int32_t iterations;       /* CG iterations (IR: inner iterations, total) */
    int32_t outer_iterations; /* IR outer iterations (0 for SS_FP64)         */
    int32_t restarts;         /* recomputed-residual restarts               */
    double relres;            /* ||b - A x|| / ||b|| recomputed at exit      */
    double true_relres;       /* same quantity, FP64 values and vectors      */
} ss_result;

/*
 * ss_cg_setup -- uploads the local matrices, maps and work vectors of
 * partition p of A to the current HIP device and prepares the kernels.
 * A must be the matrix p was built from (same n, nnz and pattern -- checked:
 * SS_EINVAL otherwise; the values may differ).  hip_stream is a hipStream_t (NULL = default
 * stream).  o may be NULL (defaults).  Device memory comes from o->alloc
 * when given.  *out is released with ss_cg_destroy.
 * Errors: SS_EINVAL (A does not match p, bad options), SS_ENOMEM,
 * SS_EDEVICE.
 */
int ss_cg_setup(const ss_csr *A, const ss_part *p, const ss_opts *o, void *hip_stream, ss_solver **out);

/*
 * ss_cg_solve -- CG (Algorithm 3; M = I, or M = diag(A) with
 * SS_PRECOND_JACOBI: z = M^{-1} r, alpha = (z, r) / (A p, p),
 * beta = (r', z') / (r, z), p = z + beta p) for A x = b.
 * b_dev[n], x_dev[n]: device, global numbering; x_dev holds the initial
 * guess x_1 on entry and the solution on return.  Stopping rule (the paper
 * states none): ||r|| <= tol ||b||, with r recomputed as b - A x whenever the
 * recurrence reports convergence (restarting CG from it if needed).  At most
 * maxit CG iterations.  b = 0 returns x = 0 after 0 iterations.
 * With precision SS_FP32_IR the same stopping rule applies to the FP64
 * residual of the outer loop: r = b - A x (FP64 values and vectors), inner CG
 * on the FP32 values with FP32 vectors for r / ||r|| (FP64 dots and scalars)
 * until its residual drops by inner_tol (or inner_maxit iterations), then
 * x += ||r|| d; at most max_outer corrections (SS_NOT_CONVERGED beyond).
 * With precision SS_FP32_RU, CG runs on the FP32 values with FP32 vectors
 * (FP64 dots and scalars) and accumulates its solution change d; at the end
 * of every polled chunk of check_every iterations, if the recursive ||r||
 * has dropped to ru_delta times the last true residual, x += d (FP64), the
 * residual is replaced by b - A x computed with the FP64 values and CG
 * continues with the same search direction; the stopping test is taken on
 * that true residual (and, when the recursion meets it, on a final
 * replacement, restarting from it if needed).  outer_iterations reports the
 * replacements made inside the iteration.
 * res (host, may be NULL) receives the result (iterations = all inner
 * iterations for SS_FP32_IR); hist_host (host, may be NULL, capacity
 * maxit+1) receives ||r_k||/||b|| for k = 0..iterations (FP32_IR: inner
 * estimates, replaced by the FP64 value at every outer step; at most the
 * first 4194304 entries are recorded).
 * Returns SS_OK, SS_NOT_CONVERGED, SS_EBREAKDOWN, SS_EINVAL (tol < 0,
 * maxit < 0), SS_EDEVICE.
 */
int ss_cg_solve(ss_solver *s, const double *b_dev, double *x_dev, double tol, int32_t maxit, ss_result *res,
                double *hist_host);

/*
 * ss_cg_solve_noalloc -- ss_cg_solve for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  Same method, arguments and results as ss_cg_solve for a
 * solver set up with SS_FP64 (any preconditioner and path), but the run
 * state and the residual history live in a fixed device array of the library
 * (256 bytes + SS_NOALLOC_HIST_MAX doubles per GPU, held until the process
 * ends) instead of the solver's buffers, no graph is instantiated (the polled
 * chunks are launched kernel by kernel), and nothing is allocated: no
 * hipMalloc, hipFree or allocator callback.
 * hist_host: NULL (no history), or capacity maxit+1 with maxit + 1 <=
 * SS_NOALLOC_HIST_MAX.
 * Every call on one GPU uses that GPU's array: calls that overlap on one GPU
 * (through any solver, on any stream or thread) race and must not be made.
 * Returns as ss_cg_solve; also SS_EINVAL (history longer than the maximum),
 * SS_EUNSUPPORTED (precision other than SS_FP64).
 */
#define SS_NOALLOC_HIST_MAX 32768
int ss_cg_solve_noalloc(ss_solver *s, const double *b_dev, double *x_dev, double tol, int32_t maxit,
                        ss_result *res, double *hist_host);

/* y_dev = A x_dev through the sub-structured path (local SpMV in every
 * sub-domain, then interface assembly; Section 4.4.1).  Device, global
 * numbering, length n; y must not alias x. */
int ss_cg_apply(ss_solver *s, const double *x_dev, double *y_dev);

/* y_dev = A32 x_dev in FP32, the product the inner CG of the SS_FP32_*
 * modes uses: A32 = the values rounded to FP32 (nearest even), every row
 * summed left to right in column order with each product and sum rounded to
 * FP32 (no fused multiply-add), then the interface copies added in ascending
 * sub-domain order in FP32 (Section 4.4.1, Algorithms 4 and 5).  x_dev[n],
 * y_dev[n]: device, FP32, global numbering; y must not alias x.
 * Errors: SS_EINVAL (NULL argument), SS_EUNSUPPORTED (solver set up with
 * SS_FP64: it holds no FP32 values), SS_EDEVICE. */
int ss_cg_apply_f32(ss_solver *s, const float *x_dev, float *y_dev);

/* Replaces the matrix values (same pattern): val_dev[nnz], device, global
 * stored-entry order.  The values must keep A symmetric positive-definite;
 * symmetry is not re-checked.  Every copy the solver keeps follows: the FP64
 * and FP32 values, the one-launch solve's values and, with
 * SS_PRECOND_JACOBI, the inverse diagonal (a non-positive diagonal then ends
 * the next solve with SS_EBREAKDOWN or a non-finite scalar). */
int ss_cg_set_values(ss_solver *s, const double *val_dev);

/* Adjoint gradient on the stored pattern: with x = A^{-1} b and
 * lambda = A^{-1} dL/dx (a second solve with the same symmetric A),
 * dvals_dev[k] = -lambda[row_k] * x[col_k] for every stored entry k, in
 * global stored-entry order.  lambda_dev[n], x_dev[n], dvals_dev[nnz]:
 * device.  dL/db equals lambda itself. */
int ss_cg_grad_vals(ss_solver *s, const double *lambda_dev, const double *x_dev, double *dvals_dev);

/* Average duration in milliseconds of one CG step (beta, p = r + beta p,
 * the local SpMV, (p, A p); the FP32 inner step for the SS_FP32_* modes):
 * one launch, or for matrices whose rows take several load batches (rows of
 * more than 9 entries) two launches -- p formed, then the SpMV on it -- timed
 * with one HIP event pair around `reps` back-to-back steps on the solver
 * stream.  Leaves the solver state unchanged except for scratch vectors.
 * Also reports the algorithmic bytes a step moves (values and column data of
 * the stored entries, row structure, one read of r, p and x, writes of p, q
 * and x; the two-launch step also reads p back). */
int ss_cg_time_spmv(ss_solver *s, int32_t reps, double *ms_per_launch, double *bytes_per_launch);

/* Measurement: the rate at which the current device streams the bytes of the
 * CG step without its gathers.  rows (>= 64, rounded down to a multiple of
 * 64) rows in chunks of 64 with `slots` (5, 7, 9 or 27) FP64 values per row
 * stored as the SELL-64 matrix stores them, one read each of three FP64
 * vectors and one write each of three, on the CG step's persistent grid;
 * reps timed back-to-back launches on hip_stream (NULL = default stream).
 * *ms_per_launch: average launch time; *bytes_per_launch (may be NULL):
 * rows * (8 slots + 48).  Allocates and frees its own buffers.
 * Errors: SS_EINVAL, SS_ENOMEM, SS_EDEVICE. */
int ss_stream_rate(int64_t rows, int32_t slots, int32_t reps, void *hip_stream, double *ms_per_launch,
                   double *bytes_per_launch);

/* Sizes of the device problem (any pointer may be NULL): matrix_format is
 * the SS_MAT_SELL / SS_MAT_CSR storage chosen, stored the entries it holds
 * (SELL: including the chunk padding). */
int ss_cg_info(const ss_solver *s, int32_t *n, int32_t *n_loc, int64_t *nnz, int32_t *matrix_format,
               int64_t *stored);

/* How ss_cg_solve runs on this solver: SS_PATH_STREAM, two streaming
 * launches per CG iteration replayed in graph chunks; SS_PATH_SMALL, the
 * whole solve in one launch (see SS_SMALL_AUTO). */
enum { SS_PATH_STREAM = 0, SS_PATH_SMALL = 1 };
int ss_cg_path(const ss_solver *s, int32_t *path);

void ss_cg_destroy(ss_solver *s);

/* --------------------------------------------------------- band splittings */
/*
 * The paper's other two decompositions (Section 3.1, Algorithm 1; Section
 * 3.2, Algorithm 2), for comparison with the sub-structuring.  n is cut into
 * nbands bands of m = n / nbands consecutive indices, the last band taking
 * the remainder n - (nbands-1) m.
 *   SS_BAND_ROW: band p holds rows [p m, p m + N_p) with all (global) columns.
 *   SS_BAND_COL: band p holds every row restricted to the columns
 *                [p m, p m + N_p), renumbered from 0.
 */
#define SS_BAND_ROW 0
#define SS_BAND_COL 1

/* Shape of band p: *nrows, *ncols and *nnz (stored entries).  Any pointer may
 * be NULL.  Errors: SS_EINVAL (invalid CSR, unknown kind, nbands outside
 * [1, n], p outside [0, nbands)). */
int ss_band_size(const ss_csr *A, int32_t kind, int32_t nbands, int32_t p, int32_t *nrows, int32_t *ncols,
                 int64_t *nnz);

/* Band p as CSR in caller-provided host arrays sized by ss_band_size:
 * rowptr[nrows+1], colidx[nnz], val[nnz]; columns ascending inside each row
 * as in A.  Errors as ss_band_size. */
int ss_band_extract(const ss_csr *A, int32_t kind, int32_t nbands, int32_t p, int32_t *rowptr, int32_t *colidx,
                    double *val);

/*
 * ss_band_setup -- CG (Algorithm 3) on A with the band splitting `kind` into
 * nbands bands, all bands on the current HIP device; solved, applied, timed
 * and released with the ss_cg_* calls of a solver from ss_cg_setup.
 * On one device the band-row splitting's collection of the whole x before
 * each product (Section 4.2.1) is the shared vector itself, so its product is
 * the global one; the band-column product (Section 4.3.1) adds the bands'
 * partial products y = sum_p A_p x_p, band by band in ascending order, which
 * is done per row: each row's sum is split where its columns cross into the
 * next band.  Dot products and the stopping rule as ss_cg_solve.
 * o: SS_FP64 only (SS_EUNSUPPORTED otherwise); the band-column product needs
 * the SELL layout (rows of at most 255 entries, fewer than 2^29 rows;
 * SS_EUNSUPPORTED otherwise).
 * Errors: SS_EINVAL (invalid CSR, unknown kind, nbands outside [1, n]),
 * SS_EUNSUPPORTED, SS_ENOMEM, SS_EDEVICE.
 */
int ss_band_setup(const ss_csr *A, int32_t kind, int32_t nbands, const ss_opts *o, void *hip_stream,
                  ss_solver **out);

/* ------------------------------------------------------- batched solver */
/*
 * Many independent SPD systems, each with nrhs right-hand sides, solved
 * together: one pass of the batched update and SpMV code over a system's
 * tiles advances all of its (system, right-hand side) pairs by one CG
 * iteration, so one read of each matrix serves all its right-hand sides, and
 * all systems share the launches (two per iteration, or one for all
 * iterations; see the schedules below).  Each pair runs exactly the CG of ss_cg_solve on its own
 * (Algorithm 3, M = I, one sub-domain): own scalars, own stopping test,
 * recomputed-residual restarts, own iteration count; a pair that stops keeps
 * its x while the others go on, and a system whose pairs have all stopped
 * drops out.  Only the summation order of the dot products
 * differs from one-by-one solves.
 *
 * Vector layout at the boundary (b_dev, x_dev): device, FP64, the systems'
 * rows concatenated in batch order, the nrhs values of a row adjacent:
 * element (system s, row i, rhs j) at (row_offset[s] + i) * nrhs + j, where
 * row_offset[s] = n_0 + ... + n_{s-1}.
 */
typedef struct ss_batch ss_batch;

/* Schedules of the batched iterations.
 * SS_BATCH_CHUNKED: every iteration is two launches over the tiles of all
 *   systems still running, captured in graphs of check_every iterations; the
 *   host polls between graphs and the list of running systems is rebuilt.
 * SS_BATCH_PERSISTENT: all iterations in one launch.  Each system moves
 *   through its own update / SpMV phases; a free workgroup claims the next
 *   tile of the first system (largest first) that has one, and the
 *   workgroup finishing a phase's last tile starts the system's next phase,
 *   so no system waits for the others and no launch boundary drains the
 *   device.  Every hand-over of a phase between workgroups costs a
 *   device-scope release and acquire (an L2 write-back and invalidation on
 *   this multi-XCD device), which makes it slower than the chunked
 *   schedule on large batches; the autotuner times both.  check_every is not
 *   used.
 * SS_BATCH_GRAPH: the chunked schedule's launches, with the whole solve
 *   captured as one HIP graph and launched once: as many check_every-
 *   iteration chunks as the longest solve of this batch so far took before
 *   its residual check (each chunk followed by the rebuild of the running
 *   list), the residual check and the restart it may start, as many chunks
 *   as that solve's restart took, and a last check.  Each check runs only
 *   once no pair runs any more (else its kernels return at once), and chunks
 *   past the end find no running system and return at once, so the results
 *   are bitwise those of the chunked schedule.  The host polls only after
 *   the graph.  The first solve of a batch runs chunk by chunk and sets the
 *   lengths; a solve that outruns the graph goes on chunk by chunk, and the
 *   next one sets the lengths again.  The graph's checks read the solve's
 *   right-hand sides from a copy that every solve makes (one more vector of
 *   the batch's size on the device). */
enum { SS_BATCH_CHUNKED = 0, SS_BATCH_PERSISTENT = 1, SS_BATCH_GRAPH = 2 };

/* Launch shape of the batched kernels.  It changes timing only: results are
 * bitwise the same for every choice (all partial sums are taken over fixed
 * 512-row granules, each system's phases run in the same order). */
typedef struct {
    int32_t tile_granules; /* 512-row granules per workgroup tile: 1, 2, 4, 8;
                              0 = per system, the fewest of those for which
                              the 2h rows around a tile that the staged SpMV
                              reads twice (h: the system's largest
                              |column - row|) are at most a quarter of it  */
    int32_t grid;          /* workgroups per launch, a multiple of 8 in
                              [8, 65536]; 0 = one per tile (chunked) or as
                              many as are resident at once (persistent)     */
    int32_t unroll;        /* matrix entries loaded per lane before use: 4, 5, 8 */
    int32_t check_every;   /* CG iterations between host polls, even, 2..1024  */
    int32_t schedule;      /* SS_BATCH_CHUNKED, SS_BATCH_PERSISTENT or
                              SS_BATCH_GRAPH                                */
} ss_batch_tuning;

typedef struct {
    ss_batch_tuning tuning;
    double ms_per_iteration; /* all pairs running */
} ss_batch_trial;

/*
 * ss_batch_setup -- uploads nsys systems (host CSR, n >= 1, columns sorted
 * and in range, pattern and values symmetric) for nrhs right-hand sides each (1, 2 or 4; pad to 4 with zero columns otherwise: a zero
 * right-hand side costs nothing) to the current HIP device.  Rows may hold at
 * most 255 entries.  o: NULL or options (only the allocator fields and
 * check_every are used).  Default tuning: 2 granules per tile, chunked, one
 * workgroup per tile, unroll 8, check_every 32.
 * Errors: SS_EINVAL, SS_EUNSUPPORTED (nrhs, row length), SS_ENOMEM,
 * SS_EDEVICE.
 */
int ss_batch_setup(int32_t nsys, const ss_csr *systems, int32_t nrhs, const ss_opts *o, void *hip_stream,
                   ss_batch **out);

/*
 * ss_batch_solve -- solves A_s x_sj = b_sj for every pair.  x_dev holds the
 * initial guesses on entry and the solutions on return; b_dev and x_dev must
 * not overlap.  tol, maxit: as ss_cg_solve, per pair.  res (host, may be
 * NULL): nsys * nrhs results, pair (s, j) at s * nrhs + j (outer_iterations
 * 0).  summary (host, may be NULL): the worst status, the largest iteration
 * count, restart count and relative residual over the pairs.
 * Returns SS_OK when every pair converged (or had b = 0), else
 * SS_EBREAKDOWN if any pair broke down, else SS_NOT_CONVERGED.
 */
int ss_batch_solve(ss_batch *bt, const double *b_dev, double *x_dev, double tol, int32_t maxit, ss_result *res,
                   ss_result *summary);

/* Sets / reads the launch shape (SS_EINVAL for values outside the ranges). */
int ss_batch_set_tuning(ss_batch *bt, const ss_batch_tuning *t);
int ss_batch_get_tuning(const ss_batch *bt, ss_batch_tuning *t);

/*
 * ss_batch_tune -- the autotuner.  Times each candidate launch shape (tile
 * granules per system/1/2/4/8 x unroll 4/5/8 x {chunked with grid one-per-tile
 * / 2048 / 1024, persistent with the resident grid}: 60 shapes) over `iters` CG
 * iterations (<= 0: 8) of this batch with right-hand sides b_dev, every pair
 * running from x = 0 (x_dev is not touched), and keeps the fastest.
 * The choice is remembered for the process, keyed by the batch structure
 * (row counts, entry counts, nrhs, device): a later call for a batch of the
 * same structure takes it without timing, unless force is nonzero.
 * chosen (may be NULL) receives the shape in use; trials (may be NULL,
 * capacity cap) the timings, *ntrials their count (0 when cached).
 */
int ss_batch_tune(ss_batch *bt, const double *b_dev, int32_t iters, int32_t force, ss_batch_tuning *chosen,
                  ss_batch_trial *trials, int32_t cap, int32_t *ntrials);

/* Sizes (any pointer may be NULL): systems, right-hand sides, total rows,
 * stored entries of the systems and the device storage incl. padding. */
int ss_batch_info(const ss_batch *bt, int32_t *nsys, int32_t *nrhs, int64_t *nrows, int64_t *nnz,
                  int64_t *stored);

/* Host-side launches of the last ss_batch_solve: *graphs = launches of the
 * whole-solve graph (SS_BATCH_GRAPH), *chunks = launches of single-chunk
 * graphs, *kernels = launches of the persistent kernel (SS_BATCH_PERSISTENT).
 * Any pointer may be NULL.  Errors: SS_EINVAL (bt NULL). */
int ss_batch_launches(const ss_batch *bt, int32_t *graphs, int32_t *chunks, int32_t *kernels);

void ss_batch_destroy(ss_batch *bt);

/* --------------------------------------------------------------- errors */
const char *ss_strerror(int code);
const char *ss_last_error(void); /* detail of the last failure on this thread */
int ss_version(void);            /* 100 * major + minor */

#ifdef __cplusplus
}
#endif

#endif /* SS_H */
