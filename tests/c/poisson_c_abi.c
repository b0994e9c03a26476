/*
 * Plain C99 client of libss: 2D 5-point Poisson problem on an m x m grid,
 * split into 2 x 2 boxes, solved through the C-ABI alone (hipMalloc'd device
 * buffers, library-owned work memory).  Prints the iteration count and the
 * relative residual recomputed on the host; exits non-zero on any failure.
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
