/*
 * Oracle, all-cores build (test infrastructure only): the CPU baseline of the
 * benchmark and the floor solutions its error figures are taken against.
 * Only tests/ and the bench's CPU-baseline leg load it; it shares no code with
 * the HIP library.
 *
 * The same sub-structured CG as ss_oracle.c -- Algorithm 3 with M = I, every
 * product a local CSR product per sub-domain followed by the assembly of the
 * interface copies (Section 4.4.1, Algorithms 4 and 5), dot products over the
 * owned positions (the 0/1 weights of Section 4.4.2), the residual recomputed
 * when the recurrence converges and CG restarted from it if needed -- with
 * its loops shared among OpenMP threads the way the paper's C+MPI code shares
 * sub-domains among processes: a static partition of the rows, of the
 * interface nodes and of the vectors, each thread's partial dot added in
 * thread order.  Built with -ffp-contract=off like the sequential oracle; for
 * a fixed thread count the results are reproducible run to run.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EBREAKDOWN = -4 };

/* Same layout as the sequential oracle's sub-domain description. */
typedef struct {
    int32_t P;
    int32_t n_loc;
    const int32_t *sub_off, *n_int, *n_own, *l2g;
    int32_t ngamma;
    const int32_t *copy_ptr, *copy_pos;
    const int32_t *bd_rowptr, *bd_colidx;
    const double *bd_val;
    const float *bd_val32;
} orc_sub;

/* An operator y = A x on n positions: CSR rows, then (if ngamma > 0) the
 * interface copies summed in list order; dots count the positions with
 * own[i] != 0. */
typedef struct {
    int64_t n;
    const int32_t *rowptr, *colidx;
    const double *val;
    int64_t ngamma;
    const int32_t *copy_ptr, *copy_pos;
    const unsigned char *own;
} omp_op;

static void op_apply(const omp_op *A, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < A->n; ++i) {
        double s = 0.0;
        for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
            s = s + A->val[k] * x[A->colidx[k]];
        y[i] = s;
    }
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < A->ngamma; ++g) {
        double t = 0.0;
        for (int64_t c = A->copy_ptr[g]; c < A->copy_ptr[g + 1]; ++c)
            t = t + y[A->copy_pos[c]];
        for (int64_t c = A->copy_ptr[g]; c < A->copy_ptr[g + 1]; ++c)
            y[A->copy_pos[c]] = t;
    }
}

/* Owned-position dot: each thread sums its static block left to right, the
 * thread partials are then added in thread order. */
static double op_dot(const omp_op *A, const double *u, const double *v)
{
    const int nt = omp_get_max_threads();
    double *part = (double *)calloc((size_t)nt, sizeof(double));
    if (!part) return NAN;
#pragma omp parallel
    {
        double s = 0.0;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < A->n; ++i)
            if (!A->own || A->own[i]) s = s + u[i] * v[i];
        part[omp_get_thread_num()] = s;
    }
    double t = 0.0;
    for (int i = 0; i < nt; ++i) t = t + part[i];
    free(part);
    return t;
}

/* Algorithm 3 (M = I) with the stopping rule and restarts of the sequential
 * oracle: stop when ||r|| <= tol ||b|| on the recomputed residual. */
static int cg_omp(const omp_op *A, const double *b, double *x, double tol, int32_t maxit, int32_t *iters,
                  double *relres)
{
    const int64_t n = A->n;
    const size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *r = (double *)malloc(sz), *p = (double *)malloc(sz), *q = (double *)malloc(sz);
    int status = ORC_OK;
    int32_t k = 0;
    double rr = 0.0;
    if (!r || !p || !q) { status = ORC_ENOMEM; goto done; }
    const double bb = op_dot(A, b, b);
    if (!isfinite(bb)) { status = ORC_EBREAKDOWN; goto done; }
    if (bb == 0.0) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        *relres = 0.0;
        goto done;
    }
    const double stop = tol * sqrt(bb);
    for (;;) {
        op_apply(A, x, q);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            r[i] = b[i] - q[i];
            p[i] = r[i];
        }
        rr = op_dot(A, r, r);
        if (!isfinite(rr)) { status = ORC_EBREAKDOWN; goto done; }
        if (sqrt(rr) <= stop) { status = ORC_OK; break; }
        if (k >= maxit) { status = ORC_NOT_CONVERGED; break; }
        while (sqrt(rr) > stop && k < maxit) {
            op_apply(A, p, q);
            const double pq = op_dot(A, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) { status = ORC_EBREAKDOWN; goto done; }
            const double alpha = rr / pq;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) {
                x[i] = x[i] + alpha * p[i];
                r[i] = r[i] - alpha * q[i];
            }
            const double rr1 = op_dot(A, r, r);
            if (!isfinite(rr1)) { status = ORC_EBREAKDOWN; goto done; }
            const double beta = rr1 / rr;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
            rr = rr1;
            ++k;
        }
    }
    *relres = sqrt(rr / bb);
done:
    *iters = k;
    free(r); free(p); free(q);
    return status;
}

static double true_relres_omp(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *val,
                              const double *b, const double *x)
{
    double *t = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!t) return NAN;
    omp_op G = {n, rowptr, colidx, val, 0, NULL, NULL, NULL};
    op_apply(&G, x, t);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) t[i] = b[i] - t[i];
    const double rr = op_dot(&G, t, t), bb = op_dot(&G, b, b);
    free(t);
    return bb == 0.0 ? 0.0 : sqrt(rr) / sqrt(bb);
}

/* Sub-structured CG on `threads` threads (<= 0: the OpenMP default).  x: in
 * x0, out the solution (global numbering, length n). */
int orc_ss_cg_omp(const orc_sub *S, int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *val,
                  const double *b, double *x, double tol, int32_t maxit, int32_t threads, int32_t *iters,
                  double *relres, double *true_rr)
{
    if (threads > 0) omp_set_num_threads(threads);
    const int64_t nl = S->n_loc;
    const size_t sz = (size_t)(nl > 0 ? nl : 1);
    double *bl = (double *)malloc(sizeof(double) * sz), *xl = (double *)malloc(sizeof(double) * sz);
    unsigned char *own = (unsigned char *)calloc(sz, 1);
    if (!bl || !xl || !own) { free(bl); free(xl); free(own); return ORC_ENOMEM; }
    for (int32_t s = 0; s < S->P; ++s)
        for (int64_t i = S->sub_off[s]; i < (int64_t)S->sub_off[s] + S->n_int[s] + S->n_own[s]; ++i) own[i] = 1;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nl; ++c) {
        bl[c] = b[S->l2g[c]];
        xl[c] = x[S->l2g[c]];
    }
    omp_op A = {nl, S->bd_rowptr, S->bd_colidx, S->bd_val, S->ngamma, S->copy_ptr, S->copy_pos, own};
    const int st = cg_omp(&A, bl, xl, tol, maxit, iters, relres);
    for (int64_t c = 0; c < nl; ++c)
        if (own[c]) x[S->l2g[c]] = xl[c];
    *true_rr = true_relres_omp(n, rowptr, colidx, val, b, x);
    free(bl); free(xl); free(own);
    return st;
}

/* CG on the unsplit global matrix on `threads` threads. */
int orc_cg_omp(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *val, const double *b,
               double *x, double tol, int32_t maxit, int32_t threads, int32_t *iters, double *relres,
               double *true_rr)
{
    if (threads > 0) omp_set_num_threads(threads);
    omp_op A = {n, rowptr, colidx, val, 0, NULL, NULL, NULL};
    const int st = cg_omp(&A, b, x, tol, maxit, iters, relres);
    *true_rr = true_relres_omp(n, rowptr, colidx, val, b, x);
    return st;
}

/* Threads an OpenMP region of this library gets by default. */
int orc_omp_max_threads(void) { return omp_get_max_threads(); }
