/*
 * Plain C99 client of libss: 2D 5-point Poisson problem on an m x m grid,
 * split into 2 x 2 boxes, solved through the C-ABI alone (hipMalloc'd device
 * buffers, library-owned work memory).  Prints the iteration count and the
 * relative residual recomputed on the host; then the product A x against
 * the host's, the allocation-free solve against the first one, and a batch
 * of three copies of the system with two right-hand sides each, solved as
 * one whole-solve graph launch.  Exits non-zero on any failure.
 *
 *   usage: poisson_c_abi [m]
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "ss.h"

#define CHECK_SS(call)                                                                  \
    do {                                                                                \
        int rc_ = (call);                                                               \
        if (rc_ != SS_OK) {                                                             \
            fprintf(stderr, "%s: %s (%s)\n", #call, ss_strerror(rc_), ss_last_error()); \
            return 1;                                                                   \
        }                                                                               \
    } while (0)

#define CHECK_HIP(call)                                              \
    do {                                                             \
        if ((call) != hipSuccess) {                                  \
            fprintf(stderr, "%s failed\n", #call);                   \
            return 1;                                                \
        }                                                            \
    } while (0)

/* An allocator whose blocks are 64 bytes past a 256-byte boundary: the
 * library must refuse them (SS_ENOMEM) and hand every block back. */
static int n_live = 0;
static void *offset_alloc(void *ctx, size_t bytes)
{
    (void)ctx;
    void *p = NULL;
    if (hipMalloc(&p, bytes + 256) != hipSuccess) return NULL;
    ++n_live;
    return (char *)p + 64;
}
static void offset_free(void *ctx, void *p)
{
    (void)ctx;
    if (p && hipFree((char *)p - 64) == hipSuccess) --n_live;
}

int main(int argc, char **argv)
{
    const int m = argc > 1 ? atoi(argv[1]) : 48;
    const int n = m * m;
    int32_t *rowptr = malloc(sizeof(int32_t) * (n + 1));
    int32_t *colidx = malloc(sizeof(int32_t) * 5 * n);
    double *val = malloc(sizeof(double) * 5 * n);
    double *b = malloc(sizeof(double) * n), *x = malloc(sizeof(double) * n), *ax = malloc(sizeof(double) * n);
    if (!rowptr || !colidx || !val || !b || !x || !ax) return 1;
    int nnz = 0;
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
            const int r = i + m * j;
            rowptr[r] = nnz;
            if (j > 0) { colidx[nnz] = r - m; val[nnz++] = -1.0; }
            if (i > 0) { colidx[nnz] = r - 1; val[nnz++] = -1.0; }
            colidx[nnz] = r; val[nnz++] = 4.0;
            if (i < m - 1) { colidx[nnz] = r + 1; val[nnz++] = -1.0; }
            if (j < m - 1) { colidx[nnz] = r + m; val[nnz++] = -1.0; }
            b[r] = (double)((r * 7919) % 2001 - 1000) / 1000.0;
            x[r] = 0.0;
        }
    rowptr[n] = nnz;
    ss_csr A = {n, nnz, rowptr, colidx, val};

    ss_part *part = NULL;
    const int32_t grid[2] = {m, m}, boxes[2] = {2, 2};
    CHECK_SS(ss_partition(&A, SS_PART_BOX, 4, 2, grid, boxes, NULL, NULL, NULL, &part));
    ss_solver *solver = NULL;
    CHECK_SS(ss_cg_setup(&A, part, NULL, NULL, &solver));

    double *b_dev = NULL, *x_dev = NULL;
    CHECK_HIP(hipMalloc((void **)&b_dev, sizeof(double) * n));
    CHECK_HIP(hipMalloc((void **)&x_dev, sizeof(double) * n));
    CHECK_HIP(hipMemcpy(b_dev, b, sizeof(double) * n, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(x_dev, x, sizeof(double) * n, hipMemcpyHostToDevice));
    ss_result res;
    CHECK_SS(ss_cg_solve(solver, b_dev, x_dev, 1e-10, 10000, &res, NULL));
    CHECK_HIP(hipMemcpy(x, x_dev, sizeof(double) * n, hipMemcpyDeviceToHost));

    double rr = 0.0, bb = 0.0;
    for (int r = 0; r < n; ++r) {
        double s = 0.0;
        for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) s += val[k] * x[colidx[k]];
        rr += (b[r] - s) * (b[r] - s);
        bb += b[r] * b[r];
    }
    const double rel = sqrt(rr / bb);
    printf("m=%d iterations=%d relres=%.3e host_relres=%.3e\n", m, res.iterations, res.relres, rel);

    /* the product A x through the sub-structured path, against the host's */
    double *y_dev = NULL;
    CHECK_HIP(hipMalloc((void **)&y_dev, sizeof(double) * n));
    CHECK_SS(ss_cg_apply(solver, x_dev, y_dev));
    CHECK_HIP(hipMemcpy(ax, y_dev, sizeof(double) * n, hipMemcpyDeviceToHost));
    double dmax = 0.0, amax = 0.0;
    for (int r = 0; r < n; ++r) {
        double s = 0.0;
        for (int k = rowptr[r]; k < rowptr[r + 1]; ++k) s += val[k] * x[colidx[k]];
        dmax = fmax(dmax, fabs(ax[r] - s));
        amax = fmax(amax, fabs(s));
    }
    printf("apply: max difference %.3e of %.3e\n", dmax, amax);
    if (!(dmax <= 1e-13 * amax)) return 4;

    /* the allocation-free solve: the same iterations and bits */
    double *x2_dev = NULL, *x2 = malloc(sizeof(double) * n);
    if (!x2) return 1;
    CHECK_HIP(hipMalloc((void **)&x2_dev, sizeof(double) * n));
    CHECK_HIP(hipMemset(x2_dev, 0, sizeof(double) * n));
    ss_result res2;
    CHECK_SS(ss_cg_solve_noalloc(solver, b_dev, x2_dev, 1e-10, 10000, &res2, NULL));
    CHECK_HIP(hipMemcpy(x2, x2_dev, sizeof(double) * n, hipMemcpyDeviceToHost));
    int same = res2.iterations == res.iterations;
    for (int r = 0; r < n; ++r) same = same && x2[r] == x[r];
    printf("noalloc: iterations=%d identical=%d\n", res2.iterations, same);
    if (!same) return 5;

    /* a batch: three copies of the system, right-hand sides (b, -b), (2b, b),
     * (b, 0) interleaved per row; the whole solve as one graph launch once
     * the first solve has set its length */
    enum { NSYS = 3, NRHS = 2 };
    ss_csr sys[NSYS] = {A, A, A};
    ss_batch *bt = NULL;
    CHECK_SS(ss_batch_setup(NSYS, sys, NRHS, NULL, NULL, &bt));
    ss_batch_tuning tun;
    CHECK_SS(ss_batch_get_tuning(bt, &tun));
    tun.schedule = SS_BATCH_GRAPH;
    CHECK_SS(ss_batch_set_tuning(bt, &tun));
    const double coef[NSYS][NRHS] = {{1.0, -1.0}, {2.0, 1.0}, {1.0, 0.0}};
    const size_t nb = (size_t)NSYS * n * NRHS;
    double *bb_h = malloc(sizeof(double) * nb), *xb_h = malloc(sizeof(double) * nb);
    if (!bb_h || !xb_h) return 1;
    for (int s = 0; s < NSYS; ++s)
        for (int r = 0; r < n; ++r)
            for (int j = 0; j < NRHS; ++j) bb_h[((size_t)s * n + r) * NRHS + j] = coef[s][j] * b[r];
    double *bb_dev = NULL, *xb_dev = NULL;
    CHECK_HIP(hipMalloc((void **)&bb_dev, sizeof(double) * nb));
    CHECK_HIP(hipMalloc((void **)&xb_dev, sizeof(double) * nb));
    CHECK_HIP(hipMemcpy(bb_dev, bb_h, sizeof(double) * nb, hipMemcpyHostToDevice));
    int32_t graphs = 0, chunks = 0, kernels = 0;
    ss_result bsum;
    for (int rep = 0; rep < 2; ++rep) {
        CHECK_HIP(hipMemset(xb_dev, 0, sizeof(double) * nb));
        CHECK_SS(ss_batch_solve(bt, bb_dev, xb_dev, 1e-10, 10000, NULL, &bsum));
        CHECK_SS(ss_batch_launches(bt, &graphs, &chunks, &kernels));
    }
    CHECK_HIP(hipMemcpy(xb_h, xb_dev, sizeof(double) * nb, hipMemcpyDeviceToHost));
    double worst = 0.0;
    for (int s = 0; s < NSYS; ++s)
        for (int j = 0; j < NRHS; ++j) {
            double r2 = 0.0, b2 = 0.0;
            for (int r = 0; r < n; ++r) {
                double t = 0.0;
                for (int k = rowptr[r]; k < rowptr[r + 1]; ++k)
                    t += val[k] * xb_h[((size_t)s * n + colidx[k]) * NRHS + j];
                const double bi = bb_h[((size_t)s * n + r) * NRHS + j];
                r2 += (bi - t) * (bi - t);
                b2 += bi * bi;
            }
            worst = fmax(worst, b2 > 0.0 ? sqrt(r2 / b2) : sqrt(r2));
        }
    printf("batch: graphs=%d chunks=%d kernels=%d iterations=%d worst_host_relres=%.3e\n", graphs, chunks, kernels,
           bsum.iterations, worst);
    if (graphs != 1 || chunks != 0 || kernels != 0 || !(worst <= 1e-10)) return 6;
    ss_batch_destroy(bt);
    CHECK_HIP(hipFree(bb_dev));
    CHECK_HIP(hipFree(xb_dev));
    CHECK_HIP(hipFree(y_dev));
    CHECK_HIP(hipFree(x2_dev));
    free(bb_h); free(xb_h); free(x2);

    ss_opts o;
    ss_opts_default(&o);
    o.alloc = offset_alloc;
    o.free = offset_free;
    ss_solver *misaligned = NULL;
    const int rc_mis = ss_cg_setup(&A, part, &o, NULL, &misaligned);
    printf("misaligned allocator: %s, blocks left %d\n", ss_strerror(rc_mis), n_live);
    if (rc_mis != SS_ENOMEM || misaligned != NULL || n_live != 0) return 3;

    ss_cg_destroy(solver);
    ss_part_destroy(part);
    CHECK_HIP(hipFree(b_dev));
    CHECK_HIP(hipFree(x_dev));
    free(rowptr); free(colidx); free(val); free(b); free(x); free(ax);
    return rel <= 1e-10 && res.status == SS_OK ? 0 : 2;
}
