/*
 * Oracle (test infrastructure only): plain, slow, sequential FP64 reference
 * for the sub-structured Conjugate Gradient.  Only tests/, the smoke check and
 * the bench's CPU-baseline leg may load it.  It shares no code with the HIP
 * library.  Built with -O2 -ffp-contract=off: every a*b+c below is a rounded
 * product followed by a rounded sum, in the order written.
 *
 * Paper: "Parallel Sub-Structuring Methods for solving Sparse Linear Systems
 * on a cluster of GPU" (Cheik Ahamed, Magoules).
 *   - CSR storage: Section 2.2.
 *   - Sub-structured SpMV = local SpMV in every sub-domain, then assembly of
 *     the interface contributions (y_3 = y_3^(1) + y_3^(2)): Section 4.4.1.
 *   - Interface exchange "collect" (Algorithm 4) and "receive and update"
 *     (Algorithm 5); a node on several interfaces receives every contribution:
 *     Section 4.4.2.
 *   - Dot products: weighted local sums then a global sum: Section 4.4.2.
 *   - CG: Algorithm 3 with M = I.
 *   - Band-row and band-column splittings (Algorithms 1 and 2) with their
 *     products and dot products: Sections 3.1, 3.2, 4.2 and 4.3.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_OK = 0, ORC_NOT_CONVERGED = 1, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EBREAKDOWN = -4 };

/* ---------------------------------------------------------------------- */
/* CSR products (Section 2.2): row i sums a_ik * x_k left to right.        */
/* ---------------------------------------------------------------------- */

void orc_csr_matvec(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *val,
                    const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            s = s + val[k] * x[colidx[k]];
        y[i] = s;
    }
}

void orc_csr_matvec_f32(int64_t n, const int32_t *rowptr, const int32_t *colidx, const float *val,
                        const float *x, float *y)
{
    for (int64_t i = 0; i < n; ++i) {
        float s = 0.0f;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            s = s + val[k] * x[colidx[k]];
        y[i] = s;
    }
}

/* ---------------------------------------------------------------------- */
/* Interface assembly (Algorithms 4 and 5 on one address space).           */
/* For every interface node, its copies (one per sub-domain that holds it, */
/* ascending sub-domain id) are added left to right and the total is       */
/* written back to every copy, so all copies hold the assembled value.     */
/* ---------------------------------------------------------------------- */

void orc_iface_sum(int64_t ngamma, const int32_t *copy_ptr, const int32_t *copy_pos, double *q)
{
    for (int64_t g = 0; g < ngamma; ++g) {
        double t = 0.0;
        for (int64_t c = copy_ptr[g]; c < copy_ptr[g + 1]; ++c)
            t = t + q[copy_pos[c]];
        for (int64_t c = copy_ptr[g]; c < copy_ptr[g + 1]; ++c)
            q[copy_pos[c]] = t;
    }
}

void orc_iface_sum_f32(int64_t ngamma, const int32_t *copy_ptr, const int32_t *copy_pos, float *q)
{
    for (int64_t g = 0; g < ngamma; ++g) {
        float t = 0.0f;
        for (int64_t c = copy_ptr[g]; c < copy_ptr[g + 1]; ++c)
            t = t + q[copy_pos[c]];
        for (int64_t c = copy_ptr[g]; c < copy_ptr[g + 1]; ++c)
            q[copy_pos[c]] = t;
    }
}

/* ---------------------------------------------------------------------- */
/* Dot products                                                            */
/* ---------------------------------------------------------------------- */

double orc_dot(int64_t n, const double *u, const double *v)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s = s + u[i] * v[i];
    return s;
}

/* Weighted local dot: every node counts once.  The weights are the 0/1
 * owner mask: sub-domain s counts its interior and owned-interface
 * positions [sub_off[s], sub_off[s] + n_int[s] + n_own[s]). */
double orc_owned_dot(int32_t P, const int32_t *sub_off, const int32_t *n_int, const int32_t *n_own,
                     const double *u, const double *v)
{
    double s = 0.0;
    for (int32_t p = 0; p < P; ++p)
        for (int64_t i = sub_off[p]; i < (int64_t)sub_off[p] + n_int[p] + n_own[p]; ++i)
            s = s + u[i] * v[i];
    return s;
}

double orc_owned_dot_f32(int32_t P, const int32_t *sub_off, const int32_t *n_int, const int32_t *n_own,
                         const float *u, const float *v)
{
    double s = 0.0;
    for (int32_t p = 0; p < P; ++p)
        for (int64_t i = sub_off[p]; i < (int64_t)sub_off[p] + n_int[p] + n_own[p]; ++i)
            s = s + (double)u[i] * (double)v[i];
    return s;
}

/* Accurately evaluated dot products: Dot2 of Ogita, Rump and Oishi ("Accurate
 * sum and dot product", SIAM J. Sci. Comput. 26(6), 2005).  Each product is
 * split into its rounded value and exact error (TwoProduct), the rounded
 * values are summed
 * with exact error tracking (TwoSum), and all errors are added in at the end:
 * the result is as accurate as a sum in twice the working precision, then
 * rounded.  Used by the reference CG whose iteration counts stand for those of
 * CG with exactly rounded dot products. */
static void two_sum(double a, double b, double *x, double *y)
{
    *x = a + b;
    const double z = *x - a;
    *y = (a - (*x - z)) + (b - z);
}

/* Dekker's TwoProduct: a b = h + r exactly (Veltkamp's split of each factor
 * into 26-bit halves; no fused multiply-add needed). */
static void split(double a, double *hi, double *lo)
{
    const double c = 134217729.0 * a; /* 2^27 + 1 */
    const double big = c - a;
    *hi = c - big;
    *lo = a - *hi;
}

static void two_product(double a, double b, double *h, double *r)
{
    double a1, a2, b1, b2;
    *h = a * b;
    split(a, &a1, &a2);
    split(b, &b1, &b2);
    *r = a2 * b2 - (((*h - a1 * b1) - a2 * b1) - a1 * b2);
}

static void dot2_add(double u, double v, double *p, double *s)
{
    double h, r, q;
    two_product(u, v, &h, &r);
    two_sum(*p, h, p, &q);
    *s = *s + (q + r);
}

double orc_dot2(int64_t n, const double *u, const double *v)
{
    double p = 0.0, s = 0.0;
    for (int64_t i = 0; i < n; ++i) dot2_add(u[i], v[i], &p, &s);
    return p + s;
}

double orc_owned_dot2(int32_t P, const int32_t *sub_off, const int32_t *n_int, const int32_t *n_own,
                      const double *u, const double *v)
{
    double p = 0.0, s = 0.0;
    for (int32_t q = 0; q < P; ++q)
        for (int64_t i = sub_off[q]; i < (int64_t)sub_off[q] + n_int[q] + n_own[q]; ++i)
            dot2_add(u[i], v[i], &p, &s);
    return p + s;
}

/* ---------------------------------------------------------------------- */
/* Sub-domain description                                                  */
/* ---------------------------------------------------------------------- */

typedef struct {
    int32_t P;
    int32_t n_loc;
    const int32_t *sub_off, *n_int, *n_own, *l2g;
    int32_t ngamma;
    const int32_t *copy_ptr, *copy_pos;
    const int32_t *bd_rowptr, *bd_colidx;
    const double *bd_val;  /* FP64 local values */
    const float *bd_val32; /* FP32 local values (may be NULL) */
} orc_sub;

/* Sub-structured SpMV, Section 4.4.1: local products, then interface assembly. */
void orc_ss_spmv(const orc_sub *S, const double *x, double *q)
{
    orc_csr_matvec(S->n_loc, S->bd_rowptr, S->bd_colidx, S->bd_val, x, q);
    orc_iface_sum(S->ngamma, S->copy_ptr, S->copy_pos, q);
}

/* The same in FP32 (values rounded to FP32, every product and sum in FP32). */
void orc_ss_spmv_f32(const orc_sub *S, const float *x, float *q)
{
    orc_csr_matvec_f32(S->n_loc, S->bd_rowptr, S->bd_colidx, S->bd_val32, x, q);
    orc_iface_sum_f32(S->ngamma, S->copy_ptr, S->copy_pos, q);
}

/* ---------------------------------------------------------------------- */
/* CG, Algorithm 3 with M = I, on an abstract operator                     */
/* ---------------------------------------------------------------------- */

typedef struct {
    int64_t n;
    void (*apply)(const void *ctx, const double *x, double *y);
    double (*dot)(const void *ctx, const double *u, const double *v);
    const void *ctx;
} orc_op;

/*
 * Stopping rule (not stated in the paper; reading adopted): stop when
 * ||r||_2 <= tol * ||b||_2.  When the recurrence reports convergence the
 * residual is recomputed as b - A x (that is also how the first residual
 * r_1 = f - S x_1 is formed); if the recomputed residual still exceeds the
 * tolerance, CG restarts from it with p = r.  maxit bounds the total number
 * of CG iterations.  hist[k] = ||r_k|| / ||b||; when a residual is
 * recomputed at iteration k it replaces hist[k].
 */
static int cg_core(const orc_op *A, const double *b, double *x, double tol, int32_t maxit,
                   double *hist, int32_t *iters, double *relres)
{
    const int64_t n = A->n;
    double *r = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *q = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int status = ORC_OK;
    int32_t k = 0;
    double rr = 0.0;
    if (!r || !p || !q) { status = ORC_ENOMEM; goto done; }

    const double bb = A->dot(A->ctx, b, b);
    if (!isfinite(bb)) { status = ORC_EBREAKDOWN; goto done; }
    if (bb == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        if (hist) hist[0] = 0.0;
        *relres = 0.0;
        goto done;
    }
    const double stop = tol * sqrt(bb);

    for (;;) {
        /* r = b - A x, p = r */
        A->apply(A->ctx, x, q);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        for (int64_t i = 0; i < n; ++i) p[i] = r[i];
        rr = A->dot(A->ctx, r, r);
        if (!isfinite(rr)) { status = ORC_EBREAKDOWN; goto done; }
        if (hist) hist[k] = sqrt(rr / bb);
        if (sqrt(rr) <= stop) { status = ORC_OK; break; }
        if (k >= maxit) { status = ORC_NOT_CONVERGED; break; }

        while (sqrt(rr) > stop && k < maxit) {
            A->apply(A->ctx, p, q);                         /* S p_k          */
            const double pq = A->dot(A->ctx, p, q);         /* (S p_k, p_k)   */
            if (!(pq > 0.0) || !isfinite(pq)) { status = ORC_EBREAKDOWN; goto done; }
            const double alpha = rr / pq;                   /* alpha_k        */
            for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
            for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
            const double rr1 = A->dot(A->ctx, r, r);
            if (!isfinite(rr1)) { status = ORC_EBREAKDOWN; goto done; }
            const double beta = rr1 / rr;                   /* beta_k         */
            for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
            rr = rr1;
            ++k;
            if (hist) hist[k] = sqrt(rr / bb);
        }
    }
    *relres = sqrt(rr / bb);
done:
    *iters = k;
    free(r); free(p); free(q);
    return status;
}

/* global operator */
typedef struct { int64_t n; const int32_t *rowptr, *colidx; const double *val; } csr_ctx;

static void glob_apply(const void *c, const double *x, double *y)
{
    const csr_ctx *A = (const csr_ctx *)c;
    orc_csr_matvec(A->n, A->rowptr, A->colidx, A->val, x, y);
}
static double glob_dot(const void *c, const double *u, const double *v)
{
    return orc_dot(((const csr_ctx *)c)->n, u, v);
}

static double glob_dot2(const void *c, const double *u, const double *v)
{
    return orc_dot2(((const csr_ctx *)c)->n, u, v);
}

/* sub-structured operator */
static void ss_apply(const void *c, const double *x, double *y) { orc_ss_spmv((const orc_sub *)c, x, y); }
static double ss_dot(const void *c, const double *u, const double *v)
{
    const orc_sub *S = (const orc_sub *)c;
    return orc_owned_dot(S->P, S->sub_off, S->n_int, S->n_own, u, v);
}
static double ss_dot2(const void *c, const double *u, const double *v)
{
    const orc_sub *S = (const orc_sub *)c;
    return orc_owned_dot2(S->P, S->sub_off, S->n_int, S->n_own, u, v);
}

static double true_relres(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *val,
                          const double *b, const double *x)
{
    double *t = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!t) return NAN;
    orc_csr_matvec(n, rowptr, colidx, val, x, t);
    for (int64_t i = 0; i < n; ++i) t[i] = b[i] - t[i];
    const double rr = orc_dot(n, t, t), bb = orc_dot(n, b, b);
    free(t);
    return bb == 0.0 ? 0.0 : sqrt(rr) / sqrt(bb);
}

/* CG on the unsplit global matrix. */
int orc_cg(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *val,
           const double *b, double *x, double tol, int32_t maxit,
           double *hist, int32_t *iters, double *relres, double *true_rr)
{
    csr_ctx c = {n, rowptr, colidx, val};
    orc_op op = {n, glob_apply, glob_dot, &c};
    int st = cg_core(&op, b, x, tol, maxit, hist, iters, relres);
    *true_rr = true_relres(n, rowptr, colidx, val, b, x);
    return st;
}

/* ---------------------------------------------------------------------- */
/* Band splittings (Section 3.1, Algorithm 1; Section 3.2, Algorithm 2).   */
/* n is cut into nb bands of m = n / nb consecutive indices, the last band */
/* taking the remainder n - (nb-1) m.  A row band holds its rows with all  */
/* (global) columns; a column band holds every row restricted to its       */
/* columns, renumbered from the band's first column.                       */
/* ---------------------------------------------------------------------- */

static void band_range(int64_t n, int32_t nb, int32_t p, int64_t *lo, int64_t *np)
{
    const int64_t m = n / nb;
    *lo = (int64_t)p * m;
    *np = p == nb - 1 ? n - (int64_t)p * m : m;
}

/* Sizes of band p: rows, columns and stored entries.  kind 0 = row band,
 * 1 = column band. */
int orc_band_size(int64_t n, const int32_t *rowptr, const int32_t *colidx, int32_t kind, int32_t nb, int32_t p,
                  int64_t *nrows, int64_t *ncols, int64_t *nnz)
{
    if (nb < 1 || nb > n || p < 0 || p >= nb || (kind != 0 && kind != 1)) return ORC_EINVAL;
    int64_t lo, np;
    band_range(n, nb, p, &lo, &np);
    if (kind == 0) {
        *nrows = np;
        *ncols = n;
        *nnz = rowptr[lo + np] - rowptr[lo];
    } else {
        int64_t c = 0;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (colidx[k] >= lo && colidx[k] < lo + np) ++c;
        *nrows = n;
        *ncols = np;
        *nnz = c;
    }
    return ORC_OK;
}

/* Band p as CSR (arrays sized by orc_band_size). */
int orc_band_extract(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *val, int32_t kind,
                     int32_t nb, int32_t p, int32_t *browptr, int32_t *bcolidx, double *bval)
{
    if (nb < 1 || nb > n || p < 0 || p >= nb || (kind != 0 && kind != 1)) return ORC_EINVAL;
    int64_t lo, np;
    band_range(n, nb, p, &lo, &np);
    if (kind == 0) {
        /* the rows lo .. lo+np-1 as they are, row pointers shifted to 0 */
        const int32_t off = rowptr[lo];
        for (int64_t i = 0; i <= np; ++i) browptr[i] = rowptr[lo + i] - off;
        for (int64_t k = 0; k < browptr[np]; ++k) {
            bcolidx[k] = colidx[off + k];
            bval[k] = val[off + k];
        }
    } else {
        /* every row, keeping the entries whose column lies in the band */
        int32_t c = 0;
        for (int64_t i = 0; i < n; ++i) {
            browptr[i] = c;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (colidx[k] >= lo && colidx[k] < lo + np) {
                    bcolidx[c] = (int32_t)(colidx[k] - lo);
                    bval[c] = val[k];
                    ++c;
                }
        }
        browptr[n] = c;
    }
    return ORC_OK;
}

/* Band-column product (Section 4.3.1): every band computes the full-length
 * y_p = A_p x_p from its column band and its part of x; y is their sum, the
 * bands added in ascending order (y = ((y_0 + y_1) + y_2) + ...). */
void orc_band_col_spmv(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *val, int32_t nb,
                       const double *x, double *y, double *yp)
{
    for (int32_t p = 0; p < nb; ++p) {
        int64_t lo, np;
        band_range(n, nb, p, &lo, &np);
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (colidx[k] >= lo && colidx[k] < lo + np) s = s + val[k] * x[colidx[k]];
            yp[i] = s;
        }
        for (int64_t i = 0; i < n; ++i) y[i] = p == 0 ? yp[i] : y[i] + yp[i];
    }
}

/* Dot product of the band splittings (Section 4.2.2): each band sums its
 * own entries, then the band sums are added in ascending band order. */
double orc_band_dot(int64_t n, int32_t nb, const double *u, const double *v)
{
    double t = 0.0;
    for (int32_t p = 0; p < nb; ++p) {
        int64_t lo, np;
        band_range(n, nb, p, &lo, &np);
        double s = 0.0;
        for (int64_t i = lo; i < lo + np; ++i) s = s + u[i] * v[i];
        t = t + s;
    }
    return t;
}

typedef struct { int64_t n; const int32_t *rowptr, *colidx; const double *val; int32_t nb; double *tmp; } band_ctx;

/* Band-row product (Section 4.2.1): once x is complete on every band, each
 * band forms its own rows of y -- row by row, the global CSR product. */
static void band_row_apply(const void *c, const double *x, double *y)
{
    const band_ctx *B = (const band_ctx *)c;
    for (int32_t p = 0; p < B->nb; ++p) {
        int64_t lo, np;
        band_range(B->n, B->nb, p, &lo, &np);
        orc_csr_matvec(np, B->rowptr + lo, B->colidx, B->val, x, y + lo);
    }
}
static void band_col_apply(const void *c, const double *x, double *y)
{
    const band_ctx *B = (const band_ctx *)c;
    orc_band_col_spmv(B->n, B->rowptr, B->colidx, B->val, B->nb, x, y, B->tmp);
}
static double band_dot(const void *c, const double *u, const double *v)
{
    const band_ctx *B = (const band_ctx *)c;
    return orc_band_dot(B->n, B->nb, u, v);
}

/* CG (Algorithm 3, M = I) with a band splitting: kind 0 = band-row,
 * 1 = band-column; nb bands. */
int orc_band_cg(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *val, int32_t kind,
                int32_t nb, const double *b, double *x, double tol, int32_t maxit, double *hist, int32_t *iters,
                double *relres, double *true_rr)
{
    if (nb < 1 || nb > n || (kind != 0 && kind != 1)) return ORC_EINVAL;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!tmp) return ORC_ENOMEM;
    band_ctx c = {n, rowptr, colidx, val, nb, tmp};
    orc_op op = {n, kind == 0 ? band_row_apply : band_col_apply, band_dot, &c};
    int st = cg_core(&op, b, x, tol, maxit, hist, iters, relres);
    *true_rr = true_relres(n, rowptr, colidx, val, b, x);
    free(tmp);
    return st;
}

/* Local copies of a global vector: every copy of node i gets v[i]. */
static void gather(const orc_sub *S, const double *v, double *loc)
{
    for (int64_t c = 0; c < S->n_loc; ++c) loc[c] = v[S->l2g[c]];
}

/* Global vector from the owned positions (each node has exactly one). */
static void scatter_owned(const orc_sub *S, const double *loc, double *v)
{
    for (int32_t p = 0; p < S->P; ++p)
        for (int64_t c = S->sub_off[p]; c < (int64_t)S->sub_off[p] + S->n_int[p] + S->n_own[p]; ++c)
            v[S->l2g[c]] = loc[c];
}

/* Sub-structured CG: Algorithm 3 where every product by S is the
 * sub-structured SpMV and every dot product the weighted local sum. */
/* CG on the unsplit global matrix with Dot2 dot products. */
int orc_cg_dot2(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *val,
                const double *b, double *x, double tol, int32_t maxit,
                double *hist, int32_t *iters, double *relres, double *true_rr)
{
    csr_ctx c = {n, rowptr, colidx, val};
    orc_op op = {n, glob_apply, glob_dot2, &c};
    int st = cg_core(&op, b, x, tol, maxit, hist, iters, relres);
    *true_rr = true_relres(n, rowptr, colidx, val, b, x);
    return st;
}

int orc_ss_cg(const orc_sub *S, int64_t n, const int32_t *rowptr, const int32_t *colidx,
              const double *val, const double *b, double *x, double tol, int32_t maxit,
              double *hist, int32_t *iters, double *relres, double *true_rr)
{
    double *bl = (double *)malloc(sizeof(double) * (size_t)(S->n_loc > 0 ? S->n_loc : 1));
    double *xl = (double *)malloc(sizeof(double) * (size_t)(S->n_loc > 0 ? S->n_loc : 1));
    if (!bl || !xl) { free(bl); free(xl); return ORC_ENOMEM; }
    gather(S, b, bl);
    gather(S, x, xl);
    orc_op op = {S->n_loc, ss_apply, ss_dot, S};
    int st = cg_core(&op, bl, xl, tol, maxit, hist, iters, relres);
    scatter_owned(S, xl, x);
    *true_rr = true_relres(n, rowptr, colidx, val, b, x);
    free(bl); free(xl);
    return st;
}

/* The sub-structured CG with Dot2 dot products (owned positions). */
int orc_ss_cg_dot2(const orc_sub *S, int64_t n, const int32_t *rowptr, const int32_t *colidx,
              const double *val, const double *b, double *x, double tol, int32_t maxit,
              double *hist, int32_t *iters, double *relres, double *true_rr)
{
    double *bl = (double *)malloc(sizeof(double) * (size_t)(S->n_loc > 0 ? S->n_loc : 1));
    double *xl = (double *)malloc(sizeof(double) * (size_t)(S->n_loc > 0 ? S->n_loc : 1));
    if (!bl || !xl) { free(bl); free(xl); return ORC_ENOMEM; }
    gather(S, b, bl);
    gather(S, x, xl);
    orc_op op = {S->n_loc, ss_apply, ss_dot2, S};
    int st = cg_core(&op, bl, xl, tol, maxit, hist, iters, relres);
    scatter_owned(S, xl, x);
    *true_rr = true_relres(n, rowptr, colidx, val, b, x);
    free(bl); free(xl);
    return st;
}

/* ---------------------------------------------------------------------- */
/* Preconditioned CG (Algorithm 3 with M = D, the diagonal of the global   */
/* matrix): z = D^{-1} r, alpha = (z, r) / (S p, p), p = z + beta p with    */
/* beta = (r_new, z_new) / (r, z).  Stopping rule, residual recomputation */
/* and restarts as in cg_core, on the unpreconditioned ||r||.  dinv holds  */
/* 1 / a_ii of every (local) position.                                     */
/* ---------------------------------------------------------------------- */

static int pcg_core(const orc_op *A, const double *dinv, const double *b, double *x, double tol, int32_t maxit,
                    double *hist, int32_t *iters, double *relres)
{
    const int64_t n = A->n;
    double *r = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *z = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *q = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int status = ORC_OK;
    int32_t k = 0;
    double rr = 0.0, rz = 0.0;
    if (!r || !z || !p || !q) { status = ORC_ENOMEM; goto done; }

    const double bb = A->dot(A->ctx, b, b);
    if (!isfinite(bb)) { status = ORC_EBREAKDOWN; goto done; }
    if (bb == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        if (hist) hist[0] = 0.0;
        *relres = 0.0;
        goto done;
    }
    const double stop = tol * sqrt(bb);

    for (;;) {
        /* r = f - S x, z = M^{-1} r, p = z */
        A->apply(A->ctx, x, q);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
        for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        for (int64_t i = 0; i < n; ++i) p[i] = z[i];
        rr = A->dot(A->ctx, r, r);
        rz = A->dot(A->ctx, r, z);
        if (!isfinite(rr) || !isfinite(rz)) { status = ORC_EBREAKDOWN; goto done; }
        if (hist) hist[k] = sqrt(rr / bb);
        if (sqrt(rr) <= stop) { status = ORC_OK; break; }
        if (k >= maxit) { status = ORC_NOT_CONVERGED; break; }

        while (sqrt(rr) > stop && k < maxit) {
            A->apply(A->ctx, p, q);                         /* S p_k          */
            const double pq = A->dot(A->ctx, p, q);         /* (S p_k, p_k)   */
            if (!(pq > 0.0) || !isfinite(pq)) { status = ORC_EBREAKDOWN; goto done; }
            const double alpha = rz / pq;                   /* alpha_k        */
            for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
            for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
            for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
            const double rr1 = A->dot(A->ctx, r, r);
            const double rz1 = A->dot(A->ctx, r, z);
            if (!isfinite(rr1) || !isfinite(rz1)) { status = ORC_EBREAKDOWN; goto done; }
            const double beta = rz1 / rz;                   /* beta_k         */
            for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
            rr = rr1;
            rz = rz1;
            ++k;
            if (hist) hist[k] = sqrt(rr / bb);
        }
    }
    *relres = sqrt(rr / bb);
done:
    *iters = k;
    free(r); free(z); free(p); free(q);
    return status;
}

/* 1 / a_ii of the global matrix (EINVAL if a diagonal entry is missing or
 * not positive). */
static int diag_inv(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *val, double *dinv)
{
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (colidx[k] == i) d = val[k];
        if (!(d > 0.0)) return ORC_EINVAL;
        dinv[i] = 1.0 / d;
    }
    return ORC_OK;
}

int orc_pcg(int64_t n, const int32_t *rowptr, const int32_t *colidx, const double *val,
            const double *b, double *x, double tol, int32_t maxit,
            double *hist, int32_t *iters, double *relres, double *true_rr)
{
    double *dinv = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!dinv) return ORC_ENOMEM;
    int st = diag_inv(n, rowptr, colidx, val, dinv);
    if (st == ORC_OK) {
        csr_ctx c = {n, rowptr, colidx, val};
        orc_op op = {n, glob_apply, glob_dot, &c};
        st = pcg_core(&op, dinv, b, x, tol, maxit, hist, iters, relres);
        *true_rr = true_relres(n, rowptr, colidx, val, b, x);
    }
    free(dinv);
    return st;
}

/* Sub-structured PCG: every copy of a node holds the node's global 1 / a_ii. */
int orc_ss_pcg(const orc_sub *S, int64_t n, const int32_t *rowptr, const int32_t *colidx,
               const double *val, const double *b, double *x, double tol, int32_t maxit,
               double *hist, int32_t *iters, double *relres, double *true_rr)
{
    const size_t m = (size_t)(S->n_loc > 0 ? S->n_loc : 1);
    double *dg = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *dl = (double *)malloc(sizeof(double) * m);
    double *bl = (double *)malloc(sizeof(double) * m);
    double *xl = (double *)malloc(sizeof(double) * m);
    int st = ORC_ENOMEM;
    if (dg && dl && bl && xl) {
        st = diag_inv(n, rowptr, colidx, val, dg);
        if (st == ORC_OK) {
            gather(S, dg, dl);
            gather(S, b, bl);
            gather(S, x, xl);
            orc_op op = {S->n_loc, ss_apply, ss_dot, S};
            st = pcg_core(&op, dl, bl, xl, tol, maxit, hist, iters, relres);
            scatter_owned(S, xl, x);
            *true_rr = true_relres(n, rowptr, colidx, val, b, x);
        }
    }
    free(dg); free(dl); free(bl); free(xl);
    return st;
}

/* ---------------------------------------------------------------------- */
/* FP32 values + FP64 iterative refinement (project variant)              */
/*                                                                         */
/* Outer: r = b - A x with FP64 values and vectors; stop when ||r|| <=     */
/* tol ||b||.  Inner: CG on the FP32 copy of the local values with FP32    */
/* vectors, FP32 products and sums inside the SpMV and the assembly, FP64  */
/* dot products and scalars; vector updates are evaluated in FP64 and      */
/* rounded to FP32.  The inner right-hand side is r / ||r||; the inner     */
/* solve stops at ||r_in|| <= inner_tol ||r_in,0|| or inner_maxit.         */
/* ---------------------------------------------------------------------- */

int orc_ss_ir(const orc_sub *S, int64_t n, const int32_t *rowptr, const int32_t *colidx,
              const double *val, const double *b, double *x, double tol, int32_t maxit,
              double inner_tol, int32_t inner_maxit, int32_t max_outer,
              int32_t *iters, int32_t *outer, double *relres, double *true_rr)
{
    const int64_t m = S->n_loc > 0 ? S->n_loc : 1;
    double *bl = malloc(sizeof(double) * m), *xl = malloc(sizeof(double) * m), *r = malloc(sizeof(double) * m);
    float *d = malloc(sizeof(float) * m), *ri = malloc(sizeof(float) * m), *p = malloc(sizeof(float) * m),
          *q = malloc(sizeof(float) * m);
    int st = ORC_OK;
    int32_t k = 0, j = 0;
    double rr = 0.0;
    if (!bl || !xl || !r || !d || !ri || !p || !q) { st = ORC_ENOMEM; goto out; }
    gather(S, b, bl);
    gather(S, x, xl);
    const double bb = orc_owned_dot(S->P, S->sub_off, S->n_int, S->n_own, bl, bl);
    if (!isfinite(bb)) { st = ORC_EBREAKDOWN; goto out; }
    if (bb == 0.0) { for (int64_t i = 0; i < S->n_loc; ++i) xl[i] = 0.0; *relres = 0.0; goto out; }
    for (;; ++j) {
        orc_ss_spmv(S, xl, r);
        for (int64_t i = 0; i < S->n_loc; ++i) r[i] = bl[i] - r[i];
        rr = orc_owned_dot(S->P, S->sub_off, S->n_int, S->n_own, r, r);
        if (!isfinite(rr)) { st = ORC_EBREAKDOWN; goto out; }
        if (sqrt(rr) <= tol * sqrt(bb)) { st = ORC_OK; break; }
        if (j >= max_outer || k >= maxit) { st = ORC_NOT_CONVERGED; break; }
        const double s = sqrt(rr);
        for (int64_t i = 0; i < S->n_loc; ++i) {
            ri[i] = (float)(r[i] / s);
            p[i] = ri[i];
            d[i] = 0.0f;
        }
        double rr_in = orc_owned_dot_f32(S->P, S->sub_off, S->n_int, S->n_own, ri, ri);
        const double stop_in = inner_tol * sqrt(rr_in);
        int32_t kin = 0;
        while (sqrt(rr_in) > stop_in && kin < inner_maxit && k < maxit) {
            orc_ss_spmv_f32(S, p, q);
            const double pq = orc_owned_dot_f32(S->P, S->sub_off, S->n_int, S->n_own, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) { st = ORC_EBREAKDOWN; goto out; }
            const double alpha = rr_in / pq;
            for (int64_t i = 0; i < S->n_loc; ++i) {
                d[i] = (float)((double)d[i] + alpha * (double)p[i]);
                ri[i] = (float)((double)ri[i] - alpha * (double)q[i]);
            }
            const double rr1 = orc_owned_dot_f32(S->P, S->sub_off, S->n_int, S->n_own, ri, ri);
            if (!isfinite(rr1)) { st = ORC_EBREAKDOWN; goto out; }
            const double beta = rr1 / rr_in;
            for (int64_t i = 0; i < S->n_loc; ++i) p[i] = (float)((double)ri[i] + beta * (double)p[i]);
            rr_in = rr1;
            ++kin;
            ++k;
        }
        for (int64_t i = 0; i < S->n_loc; ++i) xl[i] = xl[i] + s * (double)d[i];
    }
    *relres = sqrt(rr / bb);
out:
    if (st != ORC_ENOMEM) {
        scatter_owned(S, xl, x);
        *true_rr = true_relres(n, rowptr, colidx, val, b, x);
    }
    *iters = k;
    *outer = j;
    free(bl); free(xl); free(r); free(d); free(ri); free(p); free(q);
    return st;
}

/* ---------------------------------------------------------------------- */
/* FP32 CG with FP64 residual replacement ("reliable updates", Sleijpen &  */
/* van der Vorst): CG (Algorithm 3) runs on fl32(A) with FP32 vectors, FP64 */
/* dots and scalars, and accumulates its solution change in d.  Every m    */
/* iterations after a (re)start, if the recursive ||r|| has dropped to     */
/* delta times the last true residual, the correction is folded in,        */
/* x += d, d = 0, and r is replaced by fl32(b - A x) computed in FP64 with  */
/* the FP64 values; the search direction p is kept and CG continues with   */
/* (r, r) of the new r.  When the recursion meets the tolerance (or the    */
/* iteration limit) the same replacement is made and the stopping test is  */
/* taken on the true residual; CG restarts from it (p = r) if that is still */
/* above the tolerance.  Stopping rule as in cg_core; refreshes counts the */
/* replacements made inside the iteration.                                 */
/* ---------------------------------------------------------------------- */

int orc_ss_ru(const orc_sub *S, int64_t n, const int32_t *rowptr, const int32_t *colidx,
              const double *val, const double *b, double *x, double tol, int32_t maxit,
              double delta, int32_t m, int32_t *iters, int32_t *refreshes, double *relres, double *true_rr)
{
    const int64_t nl = S->n_loc > 0 ? S->n_loc : 1;
    double *bl = malloc(sizeof(double) * nl), *xl = malloc(sizeof(double) * nl), *r64 = malloc(sizeof(double) * nl);
    float *d = malloc(sizeof(float) * nl), *r = malloc(sizeof(float) * nl), *p = malloc(sizeof(float) * nl),
          *q = malloc(sizeof(float) * nl);
    int st = ORC_OK;
    int32_t k = 0, nref = 0;
    double rr64 = 0.0;
    if (!bl || !xl || !r64 || !d || !r || !p || !q || m < 1) { st = m < 1 ? ORC_EINVAL : ORC_ENOMEM; goto out; }
    gather(S, b, bl);
    gather(S, x, xl);
    const double bb = orc_owned_dot(S->P, S->sub_off, S->n_int, S->n_own, bl, bl);
    if (!isfinite(bb)) { st = ORC_EBREAKDOWN; goto out; }
    if (bb == 0.0) { for (int64_t i = 0; i < S->n_loc; ++i) xl[i] = 0.0; *relres = 0.0; goto out; }
    const double stop = tol * sqrt(bb);
    for (int64_t i = 0; i < S->n_loc; ++i) d[i] = 0.0f;
    for (;;) {
        /* fold the correction in and take the true residual (FP64) */
        for (int64_t i = 0; i < S->n_loc; ++i) {
            xl[i] = xl[i] + (double)d[i];
            d[i] = 0.0f;
        }
        orc_ss_spmv(S, xl, r64);
        for (int64_t i = 0; i < S->n_loc; ++i) r64[i] = bl[i] - r64[i];
        rr64 = orc_owned_dot(S->P, S->sub_off, S->n_int, S->n_own, r64, r64);
        if (!isfinite(rr64)) { st = ORC_EBREAKDOWN; goto out; }
        if (sqrt(rr64) <= stop) { st = ORC_OK; break; }
        if (k >= maxit) { st = ORC_NOT_CONVERGED; break; }
        /* (re)start: p = r */
        for (int64_t i = 0; i < S->n_loc; ++i) {
            r[i] = (float)r64[i];
            p[i] = r[i];
        }
        double rr = orc_owned_dot_f32(S->P, S->sub_off, S->n_int, S->n_own, r, r);
        double rref = sqrt(rr64);
        const int32_t k0 = k;
        for (;;) {
            orc_ss_spmv_f32(S, p, q);
            const double pq = orc_owned_dot_f32(S->P, S->sub_off, S->n_int, S->n_own, p, q);
            if (!(pq > 0.0) || !isfinite(pq)) { st = ORC_EBREAKDOWN; goto out; }
            const double alpha = rr / pq;
            for (int64_t i = 0; i < S->n_loc; ++i) {
                d[i] = (float)((double)d[i] + alpha * (double)p[i]);
                r[i] = (float)((double)r[i] - alpha * (double)q[i]);
            }
            const double rr1 = orc_owned_dot_f32(S->P, S->sub_off, S->n_int, S->n_own, r, r);
            ++k;
            if (!isfinite(rr1)) { st = ORC_EBREAKDOWN; goto out; }
            if (sqrt(rr1) <= stop || k >= maxit) break; /* to the true-residual test */
            const double beta = rr1 / rr;
            for (int64_t i = 0; i < S->n_loc; ++i) p[i] = (float)((double)r[i] + beta * (double)p[i]);
            rr = rr1;
            if ((k - k0) % m == 0 && sqrt(rr) <= delta * rref) {
                /* residual replacement, p kept */
                for (int64_t i = 0; i < S->n_loc; ++i) {
                    xl[i] = xl[i] + (double)d[i];
                    d[i] = 0.0f;
                }
                orc_ss_spmv(S, xl, r64);
                for (int64_t i = 0; i < S->n_loc; ++i) r64[i] = bl[i] - r64[i];
                rr64 = orc_owned_dot(S->P, S->sub_off, S->n_int, S->n_own, r64, r64);
                if (!isfinite(rr64)) { st = ORC_EBREAKDOWN; goto out; }
                ++nref;
                if (sqrt(rr64) <= stop) { st = ORC_OK; goto done; }
                for (int64_t i = 0; i < S->n_loc; ++i) r[i] = (float)r64[i];
                rr = orc_owned_dot_f32(S->P, S->sub_off, S->n_int, S->n_own, r, r);
                rref = sqrt(rr64);
            }
        }
    }
done:
    *relres = sqrt(rr64 / bb);
out:
    if (st != ORC_ENOMEM && st != ORC_EINVAL) {
        scatter_owned(S, xl, x);
        *true_rr = true_relres(n, rowptr, colidx, val, b, x);
    }
    *iters = k;
    *refreshes = nref;
    free(bl); free(xl); free(r64); free(d); free(r); free(p); free(q);
    return st;
}

/* ---------------------------------------------------------------------- */
/* Adjoint gradient on the stored pattern: for x = A^{-1} b and            */
/* lambda = A^{-1} dL/dx, dL/da_ij = -lambda_i x_j for every stored entry  */
/* taken as an independent parameter.                                      */
/* ---------------------------------------------------------------------- */

void orc_grad_vals(int64_t n, const int32_t *rowptr, const int32_t *colidx,
                   const double *lambda, const double *x, double *dvals)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            dvals[k] = -(lambda[i] * x[colidx[k]]);
}

/* ---------------------------------------------------------------------- */
/* Dense Cholesky A = L L^T and the two triangular solves (tiny systems).  */
/* a is n*n row-major and is overwritten by L in its lower triangle.       */
/* ---------------------------------------------------------------------- */

int orc_chol_solve(int64_t n, double *a, const double *b, double *x)
{
    for (int64_t j = 0; j < n; ++j) {
        double d = a[j * n + j];
        for (int64_t k = 0; k < j; ++k) d = d - a[j * n + k] * a[j * n + k];
        if (!(d > 0.0)) return ORC_EBREAKDOWN;
        const double ljj = sqrt(d);
        a[j * n + j] = ljj;
        for (int64_t i = j + 1; i < n; ++i) {
            double s = a[i * n + j];
            for (int64_t k = 0; k < j; ++k) s = s - a[i * n + k] * a[j * n + k];
            a[i * n + j] = s / ljj;
        }
    }
    for (int64_t i = 0; i < n; ++i) { /* L y = b */
        double s = b[i];
        for (int64_t k = 0; k < i; ++k) s = s - a[i * n + k] * x[k];
        x[i] = s / a[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; --i) { /* L^T x = y */
        double s = x[i];
        for (int64_t k = i + 1; k < n; ++k) s = s - a[k * n + i] * x[k];
        x[i] = s / a[i * n + i];
    }
    return ORC_OK;
}
