// Host pre-processing: CSR validation, node partitions, owner-rule split into
// sub-domains and the concatenated local numbering (sub-structuring splitting,
// Section 3.4; partitioning is a step separate from the solver, Section 3).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>

#include "ss_internal.h"

namespace {
thread_local std::string g_last_error;
}

namespace ss {

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int validate_csr(const ss_csr *A, bool require_symmetric)
{
    if (!A) return fail(SS_EINVAL, "matrix pointer is NULL");
    if (A->n < 1) return fail(SS_EINVAL, "matrix has n < 1");
    if (A->nnz < 0) return fail(SS_EINVAL, "matrix has nnz < 0");
    if (!A->rowptr || (A->nnz > 0 && (!A->colidx || !A->val)))
        return fail(SS_EINVAL, "matrix arrays are NULL");
    const int32_t n = A->n;
    if (A->rowptr[0] != 0) return fail(SS_EINVAL, "rowptr[0] != 0");
    if (A->rowptr[n] != A->nnz) return fail(SS_EINVAL, "rowptr[n] != nnz");
    for (int32_t i = 0; i < n; ++i) {
        const int32_t a = A->rowptr[i], b = A->rowptr[i + 1];
        if (b < a) return fail(SS_EINVAL, "rowptr decreases at row " + std::to_string(i));
        for (int32_t k = a; k < b; ++k) {
            const int32_t j = A->colidx[k];
            if (j < 0 || j >= n) return fail(SS_EINVAL, "column index out of range in row " + std::to_string(i));
            if (k > a && j <= A->colidx[k - 1])
                return fail(SS_EINVAL, "columns not strictly increasing in row " + std::to_string(i));
        }
    }
    if (!require_symmetric) return SS_OK;
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            const int32_t j = A->colidx[k];
            if (j == i) continue;
            const int32_t *lo = A->colidx + A->rowptr[j], *hi = A->colidx + A->rowptr[j + 1];
            const int32_t *f = std::lower_bound(lo, hi, i);
            if (f == hi || *f != i)
                return fail(SS_EINVAL, "pattern not symmetric at (" + std::to_string(i) + "," + std::to_string(j) + ")");
            const double a = A->val[k], b = A->val[f - A->colidx];
            if (std::memcmp(&a, &b, sizeof(double)) != 0)
                return fail(SS_EINVAL, "values not symmetric at (" + std::to_string(i) + "," + std::to_string(j) + ")");
        }
    }
    return SS_OK;
}

int partition_box(int32_t n, int32_t dim, const int32_t *grid, const int32_t *boxes, int32_t nparts,
                  std::vector<int32_t> &part)
{
    if (dim < 1 || dim > 3 || !grid || !boxes) return fail(SS_EINVAL, "BOX partition needs dim in 1..3, grid and boxes");
    int64_t nodes = 1, parts = 1;
    for (int d = 0; d < dim; ++d) {
        if (grid[d] < 1 || boxes[d] < 1 || boxes[d] > grid[d])
            return fail(SS_EINVAL, "BOX partition: need 1 <= boxes[d] <= grid[d]");
        nodes *= grid[d];
        parts *= boxes[d];
    }
    if (nodes != n) return fail(SS_EINVAL, "BOX partition: product of grid != n");
    if (parts != nparts) return fail(SS_EINVAL, "BOX partition: product of boxes != nparts");
    // per axis: box of every coordinate (last box whose start floor(b*M/B) <= c)
    std::vector<std::vector<int32_t>> box_of(dim);
    for (int d = 0; d < dim; ++d) {
        const int64_t M = grid[d], B = boxes[d];
        box_of[d].resize(M);
        int64_t b = 0;
        for (int64_t c = 0; c < M; ++c) {
            while (b + 1 < B && ((b + 1) * M) / B <= c) ++b;
            box_of[d][c] = (int32_t)b;
        }
    }
    part.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t rest = i, id = 0, stride = 1;
        for (int d = 0; d < dim; ++d) {
            const int64_t c = rest % grid[d];
            rest /= grid[d];
            id += box_of[d][c] * stride;
            stride *= boxes[d];
        }
        part[i] = (int32_t)id;
    }
    return SS_OK;
}

namespace {
struct Rcb {
    int32_t dim;
    const double *coords;
    const std::vector<double> *w;
    std::vector<int32_t> *part;

    void run(std::vector<int32_t> &S, size_t begin, size_t end, int32_t lo, int32_t hi)
    {
        if (hi - lo == 1) {
            for (size_t t = begin; t < end; ++t) (*part)[S[t]] = lo;
            return;
        }
        const int32_t mid = (lo + hi) / 2;
        if (end > begin) {
            int axis = 0;
            double best = -1.0;
            for (int d = 0; d < dim; ++d) {
                double mn = coords[(size_t)S[begin] * dim + d], mx = mn;
                for (size_t t = begin + 1; t < end; ++t) {
                    const double c = coords[(size_t)S[t] * dim + d];
                    mn = c < mn ? c : mn;
                    mx = c > mx ? c : mx;
                }
                if (mx - mn > best) {
                    best = mx - mn;
                    axis = d;
                }
            }
            const double *cd = coords;
            const int dm = dim;
            std::sort(S.begin() + begin, S.begin() + end, [cd, dm, axis](int32_t a, int32_t b) {
                const double ca = cd[(size_t)a * dm + axis], cb = cd[(size_t)b * dm + axis];
                return ca < cb || (ca == cb && a < b);
            });
        }
        double wl = 0.0, wt = 0.0;
        for (int32_t t = lo; t < mid; ++t) wl = wl + (*w)[t];
        for (int32_t t = lo; t < hi; ++t) wt = wt + (*w)[t];
        const size_t cnt = end - begin;
        size_t nleft = (size_t)std::floor((double)cnt * wl / wt + 0.5);
        if (nleft > cnt) nleft = cnt;
        run(S, begin, begin + nleft, lo, mid);
        run(S, begin + nleft, end, mid, hi);
    }
};
}  // namespace

int partition_rcb(int32_t n, int32_t dim, const double *coords, const double *weights, int32_t nparts,
                  std::vector<int32_t> &part)
{
    if (dim < 1 || dim > 3 || !coords) return fail(SS_EINVAL, "RCB partition needs dim in 1..3 and coords");
    for (int64_t t = 0; t < (int64_t)n * dim; ++t)
        if (!std::isfinite(coords[t])) return fail(SS_EINVAL, "RCB partition: non-finite coordinate");
    std::vector<double> w(nparts, 1.0);
    if (weights)
        for (int32_t t = 0; t < nparts; ++t) {
            if (!(weights[t] > 0.0) || !std::isfinite(weights[t]))
                return fail(SS_EINVAL, "RCB partition: weights must be positive and finite");
            w[t] = weights[t];
        }
    part.assign(n, -1);
    std::vector<int32_t> S(n);
    std::iota(S.begin(), S.end(), 0);
    Rcb r{dim, coords, &w, &part};
    r.run(S, 0, S.size(), 0, nparts);
    return SS_OK;
}

int build_subdomains(const ss_csr *A, ss_part *p)
{
    const int32_t n = A->n, P = p->P;
    const std::vector<int32_t> &part = p->part;

    // membership list of every node: its own part and the owner of every
    // entry in its row (owners are <= P(i) by the min rule); sorted, unique
    std::vector<int64_t> mptr(n + 1, 0);
    std::vector<int32_t> mlist;
    mlist.reserve((size_t)n + (size_t)n / 4);
    std::vector<int32_t> tmp;
    for (int32_t i = 0; i < n; ++i) {
        tmp.clear();
        tmp.push_back(part[i]);
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            const int32_t j = A->colidx[k];
            if (j != i) tmp.push_back(std::min(part[i], part[j]));
        }
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        mlist.insert(mlist.end(), tmp.begin(), tmp.end());
        mptr[i + 1] = (int64_t)mlist.size();
    }
    if (mlist.size() >= (size_t)INT32_MAX) return fail(SS_EINVAL, "local problem exceeds int32 positions");
    p->mult.resize(n);
    for (int32_t i = 0; i < n; ++i) p->mult[i] = (int32_t)(mptr[i + 1] - mptr[i]);

    // per sub-domain class counts: 0 interior, 1 owned interface, 2 ghost
    std::vector<int64_t> cnt((size_t)P * 3, 0);
    for (int32_t i = 0; i < n; ++i)
        for (int64_t t = mptr[i]; t < mptr[i + 1]; ++t) {
            const int32_t s = mlist[t];
            const int cls = p->mult[i] == 1 ? 0 : (part[i] == s ? 1 : 2);
            ++cnt[(size_t)s * 3 + cls];
        }
    p->sub_off.assign(P + 1, 0);
    p->n_int.resize(P);
    p->n_own.resize(P);
    std::vector<int64_t> cursor((size_t)P * 3);
    int64_t off = 0;
    for (int32_t s = 0; s < P; ++s) {
        p->sub_off[s] = (int32_t)off;
        p->n_int[s] = (int32_t)cnt[(size_t)s * 3];
        p->n_own[s] = (int32_t)cnt[(size_t)s * 3 + 1];
        cursor[(size_t)s * 3] = off;
        cursor[(size_t)s * 3 + 1] = off + cnt[(size_t)s * 3];
        cursor[(size_t)s * 3 + 2] = off + cnt[(size_t)s * 3] + cnt[(size_t)s * 3 + 1];
        off += cnt[(size_t)s * 3] + cnt[(size_t)s * 3 + 1] + cnt[(size_t)s * 3 + 2];
    }
    p->sub_off[P] = (int32_t)off;
    const int32_t n_loc = (int32_t)off;

    // positions: ascending node id inside every (sub-domain, class) group
    std::vector<int32_t> mpos(mlist.size());
    p->l2g.resize(n_loc);
    p->g2own.resize(n);
    for (int32_t i = 0; i < n; ++i)
        for (int64_t t = mptr[i]; t < mptr[i + 1]; ++t) {
            const int32_t s = mlist[t];
            const int cls = p->mult[i] == 1 ? 0 : (part[i] == s ? 1 : 2);
            const int32_t pos = (int32_t)cursor[(size_t)s * 3 + cls]++;
            mpos[t] = pos;
            p->l2g[pos] = i;
            if (s == part[i]) p->g2own[i] = pos;
        }

    // interface nodes and their copies, ascending sub-domain
    p->gamma.clear();
    p->copy_ptr.assign(1, 0);
    p->copy_pos.clear();
    for (int32_t i = 0; i < n; ++i) {
        if (p->mult[i] < 2) continue;
        p->gamma.push_back(i);
        for (int64_t t = mptr[i]; t < mptr[i + 1]; ++t) p->copy_pos.push_back(mpos[t]);
        p->copy_ptr.push_back((int32_t)p->copy_pos.size());
    }

    auto pos_in = [&](int32_t node, int32_t s) -> int32_t {
        for (int64_t t = mptr[node]; t < mptr[node + 1]; ++t)
            if (mlist[t] == s) return mpos[t];
        return -1;
    };

    // local matrices: entry (i,j) with owner o sits in row pos(o,i), column pos(o,j)
    const int64_t nnz = A->nnz;
    p->bd_rowptr.assign((size_t)n_loc + 1, 0);
    std::vector<int32_t> erow((size_t)nnz), ecol((size_t)nnz);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            const int32_t j = A->colidx[k];
            const int32_t o = (i == j) ? part[i] : std::min(part[i], part[j]);
            erow[k] = pos_in(i, o);
            ecol[k] = pos_in(j, o);
            if (erow[k] < 0 || ecol[k] < 0) return fail(SS_EINVAL, "pattern is not symmetric");
            ++p->bd_rowptr[(size_t)erow[k] + 1];
        }
    for (int32_t c = 0; c < n_loc; ++c) p->bd_rowptr[c + 1] += p->bd_rowptr[c];
    p->bd_colidx.resize((size_t)nnz);
    p->bd_nzmap.resize((size_t)nnz);
    std::vector<int32_t> fill(p->bd_rowptr.begin(), p->bd_rowptr.end() - 1);
    for (int64_t k = 0; k < nnz; ++k) {
        const int32_t at = fill[erow[k]]++;
        p->bd_colidx[at] = ecol[k];
        p->bd_nzmap[at] = (int32_t)k;
    }
    // sort every local row by column position (insertion sort: rows are short)
    for (int32_t c = 0; c < n_loc; ++c) {
        const int32_t a = p->bd_rowptr[c], b = p->bd_rowptr[c + 1];
        for (int32_t u = a + 1; u < b; ++u) {
            const int32_t kc = p->bd_colidx[u], km = p->bd_nzmap[u];
            int32_t v = u - 1;
            while (v >= a && p->bd_colidx[v] > kc) {
                p->bd_colidx[v + 1] = p->bd_colidx[v];
                p->bd_nzmap[v + 1] = p->bd_nzmap[v];
                --v;
            }
            p->bd_colidx[v + 1] = kc;
            p->bd_nzmap[v + 1] = km;
        }
    }
    return SS_OK;
}

}  // namespace ss

// ---------------------------------------------------------------------------
// C-ABI: partitions and errors
// ---------------------------------------------------------------------------

extern "C" {

const char *ss_last_error(void) { return g_last_error.c_str(); }

const char *ss_strerror(int code)
{
    switch (code) {
    case SS_OK: return "success";
    case SS_NOT_CONVERGED: return "maximum number of iterations reached";
    case SS_EINVAL: return "invalid argument";
    case SS_ENOMEM: return "out of memory";
    case SS_EDEVICE: return "HIP runtime error";
    case SS_EBREAKDOWN: return "CG breakdown: matrix not SPD or non-finite data";
    case SS_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

int ss_version(void) { return 100; }

int ss_partition(const ss_csr *A, int32_t method, int32_t nparts, int32_t dim, const int32_t *grid,
                 const int32_t *boxes, const double *coords, const double *weights, const int32_t *user_part,
                 ss_part **out)
{
    if (!out) return ss::fail(SS_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = ss::validate_csr(A, true);
    if (rc != SS_OK) return rc;
    if (nparts < 1 || nparts > A->n) return ss::fail(SS_EINVAL, "nparts must be in [1, n]");
    ss_part *p = new (std::nothrow) ss_part;
    if (!p) return ss::fail(SS_ENOMEM, "host allocation failed");
    try {
        p->n = A->n;
        p->P = nparts;
        p->nnz = A->nnz;
        switch (method) {
        case SS_PART_BOX: rc = ss::partition_box(A->n, dim, grid, boxes, nparts, p->part); break;
        case SS_PART_RCB: rc = ss::partition_rcb(A->n, dim, coords, weights, nparts, p->part); break;
        case SS_PART_GRAPH: rc = ss::partition_graph(A, weights, nparts, p->part); break;
        case SS_PART_USER:
            if (!user_part) { rc = ss::fail(SS_EINVAL, "USER partition needs user_part"); break; }
            p->part.assign(user_part, user_part + A->n);
            for (int32_t i = 0; i < A->n; ++i)
                if (p->part[i] < 0 || p->part[i] >= nparts) {
                    rc = ss::fail(SS_EINVAL, "user_part value out of [0, nparts)");
                    break;
                }
            break;
        default: rc = ss::fail(SS_EINVAL, "unknown partition method");
        }
        if (rc == SS_OK) rc = ss::build_subdomains(A, p);
    } catch (const std::bad_alloc &) {
        rc = ss::fail(SS_ENOMEM, "host allocation failed");
    }
    if (rc != SS_OK) {
        delete p;
        return rc;
    }
    *out = p;
    return SS_OK;
}

int ss_part_sizes(const ss_part *p, int32_t *nparts, int32_t *n, int32_t *n_loc, int32_t *n_gamma,
                  int32_t *n_copies, int64_t *nnz)
{
    if (!p) return ss::fail(SS_EINVAL, "partition is NULL");
    if (nparts) *nparts = p->P;
    if (n) *n = p->n;
    if (n_loc) *n_loc = p->n_loc();
    if (n_gamma) *n_gamma = (int32_t)p->gamma.size();
    if (n_copies) *n_copies = (int32_t)p->copy_pos.size();
    if (nnz) *nnz = p->nnz;
    return SS_OK;
}

static void copy_out(int32_t *dst, const std::vector<int32_t> &src)
{
    if (dst && !src.empty()) std::memcpy(dst, src.data(), src.size() * sizeof(int32_t));
}

int ss_part_export(const ss_part *p, int32_t *part, int32_t *sub_off, int32_t *n_int, int32_t *n_own,
                   int32_t *l2g, int32_t *gamma, int32_t *copy_ptr, int32_t *copy_pos)
{
    if (!p) return ss::fail(SS_EINVAL, "partition is NULL");
    copy_out(part, p->part);
    copy_out(sub_off, p->sub_off);
    copy_out(n_int, p->n_int);
    copy_out(n_own, p->n_own);
    copy_out(l2g, p->l2g);
    copy_out(gamma, p->gamma);
    copy_out(copy_ptr, p->copy_ptr);
    copy_out(copy_pos, p->copy_pos);
    return SS_OK;
}

int ss_part_export_local(const ss_part *p, int32_t *bd_rowptr, int32_t *bd_colidx, int32_t *bd_nzmap)
{
    if (!p) return ss::fail(SS_EINVAL, "partition is NULL");
    copy_out(bd_rowptr, p->bd_rowptr);
    copy_out(bd_colidx, p->bd_colidx);
    copy_out(bd_nzmap, p->bd_nzmap);
    return SS_OK;
}

void ss_part_destroy(ss_part *p) { delete p; }

// Bands (Algorithms 1 and 2): m = n / nbands indices per band, the last
// band taking the remainder.
static int band_check(const ss_csr *A, int32_t kind, int32_t nbands, int32_t p, int64_t *lo, int64_t *width)
{
    int rc = ss::validate_csr(A, false);
    if (rc != SS_OK) return rc;
    if (kind != SS_BAND_ROW && kind != SS_BAND_COL) return ss::fail(SS_EINVAL, "unknown band kind");
    if (nbands < 1 || nbands > A->n) return ss::fail(SS_EINVAL, "nbands must be in [1, n]");
    if (p < 0 || p >= nbands) return ss::fail(SS_EINVAL, "band index out of range");
    const int64_t m = A->n / nbands;
    *lo = (int64_t)p * m;
    *width = p == nbands - 1 ? A->n - *lo : m;
    return SS_OK;
}

int ss_band_size(const ss_csr *A, int32_t kind, int32_t nbands, int32_t p, int32_t *nrows, int32_t *ncols,
                 int64_t *nnz)
{
    int64_t lo, w;
    const int rc = band_check(A, kind, nbands, p, &lo, &w);
    if (rc != SS_OK) return rc;
    int64_t cnt = 0;
    if (kind == SS_BAND_ROW) {
        cnt = A->rowptr[lo + w] - A->rowptr[lo];
    } else {
        for (int64_t k = 0; k < A->nnz; ++k) cnt += A->colidx[k] >= lo && A->colidx[k] < lo + w;
    }
    if (nrows) *nrows = kind == SS_BAND_ROW ? (int32_t)w : A->n;
    if (ncols) *ncols = kind == SS_BAND_ROW ? A->n : (int32_t)w;
    if (nnz) *nnz = cnt;
    return SS_OK;
}

int ss_band_extract(const ss_csr *A, int32_t kind, int32_t nbands, int32_t p, int32_t *rowptr, int32_t *colidx,
                    double *val)
{
    int64_t lo, w;
    const int rc = band_check(A, kind, nbands, p, &lo, &w);
    if (rc != SS_OK) return rc;
    if (!rowptr || !colidx || !val) return ss::fail(SS_EINVAL, "band arrays are NULL");
    if (kind == SS_BAND_ROW) {
        const int32_t first = A->rowptr[lo];
        for (int64_t i = 0; i <= w; ++i) rowptr[i] = A->rowptr[lo + i] - first;
        std::copy(A->colidx + first, A->colidx + A->rowptr[lo + w], colidx);
        std::copy(A->val + first, A->val + A->rowptr[lo + w], val);
    } else {
        int32_t c = 0;
        for (int32_t i = 0; i < A->n; ++i) {
            rowptr[i] = c;
            // columns ascend: the band's entries of a row are consecutive
            const int32_t *b = A->colidx + A->rowptr[i], *e = A->colidx + A->rowptr[i + 1];
            const int32_t *f = std::lower_bound(b, e, (int32_t)lo);
            for (; f != e && *f < lo + w; ++f, ++c) {
                colidx[c] = (int32_t)(*f - lo);
                val[c] = A->val[f - A->colidx];
            }
        }
        rowptr[A->n] = c;
    }
    return SS_OK;
}

}  // extern "C"
