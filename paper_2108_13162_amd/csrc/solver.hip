// Solver driver: device setup, the CG loop of Algorithm 3 with device-resident
// scalars, HIP-graph replay of polled iteration chunks, and the remaining
// C-ABI entry points of ss.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"
#include "ss_internal.h"

using namespace ss;

namespace {

constexpr int kDefaultCheck = 32;
constexpr int32_t kHistMax = 1 << 22;  // residual history entries kept on the device

struct DeviceMem {
    ss_alloc_fn alloc = nullptr;
    ss_free_fn release = nullptr;
    void *ctx = nullptr;
    std::vector<void *> blocks;

    void *get(size_t bytes)
    {
        if (bytes == 0) bytes = 16;
        bytes = (bytes + 255) & ~size_t(255);
        void *p = nullptr;
        if (alloc) {
            p = alloc(ctx, bytes);
        } else if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
        if (p) blocks.push_back(p);
        return p;
    }
    void put(void *p)
    {
        auto it = std::find(blocks.begin(), blocks.end(), p);
        if (it == blocks.end()) return;
        blocks.erase(it);
        if (release)
            release(ctx, p);
        else
            (void)hipFree(p);
    }
    void clear()
    {
        for (void *p : blocks) {
            if (release)
                release(ctx, p);
            else
                (void)hipFree(p);
        }
        blocks.clear();
    }
};

#define SS_HIP(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) return fail(SS_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

struct ss_solver {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;  // private stream used only to capture graphs
    ss_opts opts{};
    DeviceMem mem;

    int32_t n = 0, n_loc = 0, P = 0, ngamma = 0, ncopies = 0;
    int64_t nnz = 0;

    // matrix and maps
    int32_t *rowptr = nullptr, *colidx = nullptr, *tile_row = nullptr, *nzmap = nullptr;
    double *val = nullptr;
    float *val32 = nullptr;
    int32_t *l2g = nullptr, *g2own = nullptr, *copy_ptr = nullptr, *copy_pos = nullptr, *pos_grp = nullptr;
    UpdBlock *ublk = nullptr;
    int32_t ntiles = 0, nublk = 0, tile_nnz = 2048;

    // FP64 work vectors (concatenated local numbering)
    double *b = nullptr, *x = nullptr, *r = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
    double *partial = nullptr;
    size_t partial_len = 0;
    DevState *st = nullptr;
    double *hist = nullptr;
    int32_t hist_cap = 0;

    // host side
    DevState *st_pinned = nullptr;     // readback of the state
    int32_t *flag_pinned = nullptr;    // two status slots for pipelined polling
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t t0 = nullptr, t1 = nullptr;

    // graph of one polled chunk
    hipGraphExec_t chunk_exec = nullptr;
    hipGraph_t chunk_graph = nullptr;
    int32_t chunk_iters = 0;

    Csr csr64() const { return Csr{rowptr, colidx, tile_row, val, ntiles, tile_nnz}; }
    Iface iface() const { return Iface{ublk, nublk, pos_grp, copy_ptr, copy_pos, ngamma}; }
};

namespace {

// Row tiles: consecutive rows with at most tile_nnz stored entries (and at
// most 4 * workgroup rows); a longer row forms a tile of its own.
std::vector<int32_t> build_tiles(const std::vector<int32_t> &rowptr, int32_t tile_nnz)
{
    const int32_t nrows = (int32_t)rowptr.size() - 1;
    const int32_t rmax = 4 * kBS;
    std::vector<int32_t> t;
    t.push_back(0);
    int32_t r0 = 0;
    while (r0 < nrows) {
        int32_t r = r0;
        if (rowptr[r0 + 1] - rowptr[r0] > tile_nnz) {
            r = r0 + 1;
        } else {
            while (r < nrows && r - r0 < rmax && rowptr[r + 1] - rowptr[r0] <= tile_nnz) ++r;
        }
        t.push_back(r);
        r0 = r;
    }
    return t;
}

// Workgroups of the update / residual kernels: per sub-domain, the interior,
// owned-interface and other-interface ranges cut into pieces of kBS * kUI.
void build_update_blocks(const ss_part *p, std::vector<UpdBlock> &blk, std::vector<int32_t> &pos_grp)
{
    const int32_t chunk = kBS * kUI;
    const int32_t nl = p->n_loc();
    // interface index of every interface position
    std::vector<int32_t> ifidx(nl, -1);
    int32_t nif = 0;
    for (int32_t s = 0; s < p->P; ++s)
        for (int32_t c = p->sub_off[s] + p->n_int[s]; c < p->sub_off[s + 1]; ++c) ifidx[c] = nif++;
    pos_grp.assign(nif, -1);
    for (size_t g = 0; g + 1 < p->copy_ptr.size(); ++g)
        for (int32_t u = p->copy_ptr[g]; u < p->copy_ptr[g + 1]; ++u) pos_grp[ifidx[p->copy_pos[u]]] = (int32_t)g;
    blk.clear();
    for (int32_t s = 0; s < p->P; ++s) {
        const int32_t a = p->sub_off[s];
        const int32_t bounds[4] = {a, a + p->n_int[s], a + p->n_int[s] + p->n_own[s], p->sub_off[s + 1]};
        for (int kind = 0; kind < 3; ++kind)
            for (int32_t c = bounds[kind]; c < bounds[kind + 1]; c += chunk) {
                const int32_t cnt = std::min(chunk, bounds[kind + 1] - c);
                blk.push_back(UpdBlock{c, cnt, kind, kind == 0 ? -1 : ifidx[c]});
            }
    }
}

template <typename T>
int upload(ss_solver *s, T **dst, const T *src, size_t count)
{
    *dst = (T *)s->mem.get(sizeof(T) * count);
    if (!*dst) return fail(SS_ENOMEM, "device allocation failed");
    if (count) SS_HIP(hipMemcpyAsync(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice, s->stream));
    return SS_OK;
}

template <typename T>
int alloc_dev(ss_solver *s, T **dst, size_t count)
{
    *dst = (T *)s->mem.get(sizeof(T) * count);
    return *dst ? SS_OK : fail(SS_ENOMEM, "device allocation failed");
}

void destroy_graph(ss_solver *s)
{
    if (s->chunk_exec) (void)hipGraphExecDestroy(s->chunk_exec);
    if (s->chunk_graph) (void)hipGraphDestroy(s->chunk_graph);
    s->chunk_exec = nullptr;
    s->chunk_graph = nullptr;
    s->chunk_iters = 0;
}

// One CG iteration: two launches (plus two finishing launches when the
// reductions are not fused).  `odd` selects the p ping-pong direction.
void enqueue_iteration(ss_solver *s, hipStream_t stream, bool odd)
{
    double *pin = odd ? s->p1 : s->p0;
    double *pout = odd ? s->p0 : s->p1;
    const bool fused = s->opts.fused_reduce != 0;
    launch_spmv_cg<double, double>(stream, s->csr64(), pin, s->r, pout, s->q, s->partial, s->st, fused);
    launch_update<double>(stream, s->iface(), s->x, pout, s->r, s->q, s->partial, s->st, fused);
}

int ensure_chunk_graph(ss_solver *s, int32_t iters)
{
    if (s->chunk_exec && s->chunk_iters == iters) return SS_OK;
    destroy_graph(s);
    SS_HIP(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
    for (int32_t k = 0; k < iters; ++k) enqueue_iteration(s, s->cap, (k & 1) != 0);
    hipGraph_t g = nullptr;
    SS_HIP(hipStreamEndCapture(s->cap, &g));
    s->chunk_graph = g;
    SS_HIP(hipGraphInstantiate(&s->chunk_exec, g, nullptr, nullptr, 0));
    s->chunk_iters = iters;
    return SS_OK;
}

int enqueue_chunk(ss_solver *s, int32_t iters)
{
    if (s->opts.use_graph) {
        SS_HIP(hipGraphLaunch(s->chunk_exec, s->stream));
    } else {
        for (int32_t k = 0; k < iters; ++k) enqueue_iteration(s, s->stream, (k & 1) != 0);
        SS_HIP(hipGetLastError());
    }
    return SS_OK;
}

// Runs CG iterations until the device status leaves RUNNING.  Chunks of
// `check_every` iterations (even, so every chunk starts from p0) are queued
// one ahead of the status poll, so the device never idles on the host.
int iterate(ss_solver *s)
{
    int32_t chunk = s->opts.check_every > 0 ? s->opts.check_every : kDefaultCheck;
    chunk += chunk & 1;
    if (s->opts.use_graph) {
        int rc = ensure_chunk_graph(s, chunk);
        if (rc != SS_OK) return rc;
    }
    int slot = 0;
    int rc = enqueue_chunk(s, chunk);
    if (rc != SS_OK) return rc;
    SS_HIP(hipMemcpyAsync(&s->flag_pinned[slot], &s->st->status, sizeof(int32_t), hipMemcpyDeviceToHost, s->stream));
    SS_HIP(hipEventRecord(s->ev[slot], s->stream));
    for (;;) {
        const int nxt = slot ^ 1;
        rc = enqueue_chunk(s, chunk);
        if (rc != SS_OK) return rc;
        SS_HIP(hipMemcpyAsync(&s->flag_pinned[nxt], &s->st->status, sizeof(int32_t), hipMemcpyDeviceToHost,
                              s->stream));
        SS_HIP(hipEventRecord(s->ev[nxt], s->stream));
        SS_HIP(hipEventSynchronize(s->ev[slot]));
        if (s->flag_pinned[slot] != ST_RUNNING) {
            SS_HIP(hipEventSynchronize(s->ev[nxt]));
            return SS_OK;
        }
        slot = nxt;
    }
}

int read_status(ss_solver *s, int32_t *status)
{
    SS_HIP(hipMemcpyAsync(&s->flag_pinned[0], &s->st->status, sizeof(int32_t), hipMemcpyDeviceToHost, s->stream));
    SS_HIP(hipStreamSynchronize(s->stream));
    *status = s->flag_pinned[0];
    return SS_OK;
}

int ensure_hist(ss_solver *s, int32_t cap)
{
    if (s->hist_cap >= cap) return SS_OK;
    if (s->hist) s->mem.put(s->hist);
    s->hist = nullptr;
    s->hist_cap = 0;
    int rc = alloc_dev(s, &s->hist, (size_t)cap);
    if (rc != SS_OK) return rc;
    s->hist_cap = cap;
    return SS_OK;
}

}  // namespace

extern "C" {

void ss_opts_default(ss_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = SS_FP64;
    o->inner_tol = 1e-5;
    o->inner_maxit = 0;
    o->max_outer = 50;
    o->check_every = kDefaultCheck;
    o->use_graph = 1;
    o->tile_nnz = 0;
    o->fused_reduce = 1;
}

void ss_cg_destroy(ss_solver *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    destroy_graph(s);
    for (auto &e : s->ev)
        if (e) (void)hipEventDestroy(e);
    if (s->t0) (void)hipEventDestroy(s->t0);
    if (s->t1) (void)hipEventDestroy(s->t1);
    if (s->st_pinned) (void)hipHostFree(s->st_pinned);
    if (s->flag_pinned) (void)hipHostFree(s->flag_pinned);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    s->mem.clear();
    delete s;
}

int ss_cg_setup(const ss_csr *A, const ss_part *p, const ss_opts *o, void *hip_stream, ss_solver **out)
{
    if (!out) return fail(SS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return fail(SS_EINVAL, "partition is NULL");
    int rc = validate_csr(A, false);
    if (rc != SS_OK) return rc;
    if (A->n != p->n || (int64_t)A->nnz != p->nnz) return fail(SS_EINVAL, "matrix does not match the partition");
    ss_opts opts;
    ss_opts_default(&opts);
    if (o) opts = *o;
    if (opts.precision != SS_FP64 && opts.precision != SS_FP32_IR) return fail(SS_EINVAL, "unknown precision");
    if (opts.tile_nnz != 0 && opts.tile_nnz != 1024 && opts.tile_nnz != 2048 && opts.tile_nnz != 4096)
        return fail(SS_EINVAL, "tile_nnz must be 0, 1024, 2048 or 4096");
    if ((opts.alloc == nullptr) != (opts.free == nullptr)) return fail(SS_EINVAL, "alloc and free go together");
    if (opts.precision == SS_FP32_IR) return fail(SS_EUNSUPPORTED, "FP32 iterative refinement is not built yet");

    ss_solver *s = new (std::nothrow) ss_solver;
    if (!s) return fail(SS_ENOMEM, "host allocation failed");
    s->opts = opts;
    s->mem.alloc = opts.alloc;
    s->mem.release = opts.free;
    s->mem.ctx = opts.alloc_ctx;
    s->stream = (hipStream_t)hip_stream;
    auto bail = [&](int code) {
        ss_cg_destroy(s);
        return code;
    };
    if (hipGetDevice(&s->device) != hipSuccess) return bail(fail(SS_EDEVICE, "no HIP device"));
    if (hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(SS_EDEVICE, "stream creation failed"));
    for (auto &e : s->ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return bail(fail(SS_EDEVICE, "event creation failed"));
    if (hipEventCreate(&s->t0) != hipSuccess || hipEventCreate(&s->t1) != hipSuccess)
        return bail(fail(SS_EDEVICE, "event creation failed"));
    if (hipHostMalloc((void **)&s->st_pinned, sizeof(DevState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&s->flag_pinned, 4 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess)
        return bail(fail(SS_ENOMEM, "pinned host allocation failed"));

    s->n = p->n;
    s->n_loc = p->n_loc();
    s->P = p->P;
    s->nnz = p->nnz;
    s->ngamma = (int32_t)p->gamma.size();
    s->ncopies = (int32_t)p->copy_pos.size();
    s->tile_nnz = opts.tile_nnz ? opts.tile_nnz : 2048;

    std::vector<int32_t> tiles = build_tiles(p->bd_rowptr, s->tile_nnz);
    s->ntiles = (int32_t)tiles.size() - 1;
    std::vector<UpdBlock> blk;
    std::vector<int32_t> pos_grp;
    build_update_blocks(p, blk, pos_grp);
    s->nublk = (int32_t)blk.size();
    std::vector<double> val_bd((size_t)s->nnz);
    for (int64_t e = 0; e < s->nnz; ++e) val_bd[e] = A->val[p->bd_nzmap[e]];

    const size_t nl = (size_t)std::max(s->n_loc, 1);
    if ((rc = upload(s, &s->rowptr, p->bd_rowptr.data(), p->bd_rowptr.size())) ||
        (rc = upload(s, &s->colidx, p->bd_colidx.data(), p->bd_colidx.size())) ||
        (rc = upload(s, &s->nzmap, p->bd_nzmap.data(), p->bd_nzmap.size())) ||
        (rc = upload(s, &s->val, val_bd.data(), val_bd.size())) ||
        (rc = upload(s, &s->tile_row, tiles.data(), tiles.size())) ||
        (rc = upload(s, &s->l2g, p->l2g.data(), p->l2g.size())) ||
        (rc = upload(s, &s->g2own, p->g2own.data(), p->g2own.size())) ||
        (rc = upload(s, &s->copy_ptr, p->copy_ptr.data(), p->copy_ptr.size())) ||
        (rc = upload(s, &s->copy_pos, p->copy_pos.data(), p->copy_pos.size())) ||
        (rc = upload(s, &s->pos_grp, pos_grp.data(), pos_grp.size())) ||
        (rc = upload(s, &s->ublk, blk.data(), blk.size())) || (rc = alloc_dev(s, &s->b, nl)) ||
        (rc = alloc_dev(s, &s->x, nl)) || (rc = alloc_dev(s, &s->r, nl)) || (rc = alloc_dev(s, &s->p0, nl)) ||
        (rc = alloc_dev(s, &s->p1, nl)) || (rc = alloc_dev(s, &s->q, nl)) || (rc = alloc_dev(s, &s->st, 1)))
        return bail(rc);
    s->partial_len = 2 * (size_t)std::max(xcd_grid(s->ntiles), xcd_grid(s->nublk)) + 16;
    if ((rc = alloc_dev(s, &s->partial, s->partial_len))) return bail(rc);
    DevState init{};
    std::memcpy(s->st_pinned, &init, sizeof(DevState));
    if (hipMemcpyAsync(s->st, s->st_pinned, sizeof(DevState), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return bail(fail(SS_EDEVICE, "upload failed"));
    *out = s;
    return SS_OK;
}

int ss_cg_info(const ss_solver *s, int32_t *n, int32_t *n_loc, int64_t *nnz, int32_t *ntiles, int32_t *tile_nnz)
{
    if (!s) return fail(SS_EINVAL, "solver is NULL");
    if (n) *n = s->n;
    if (n_loc) *n_loc = s->n_loc;
    if (nnz) *nnz = s->nnz;
    if (ntiles) *ntiles = s->ntiles;
    if (tile_nnz) *tile_nnz = s->tile_nnz;
    return SS_OK;
}

int ss_cg_solve(ss_solver *s, const double *b_dev, double *x_dev, double tol, int32_t maxit, ss_result *res,
                double *hist_host)
{
    if (!s) return fail(SS_EINVAL, "solver is NULL");
    if (!b_dev || !x_dev) return fail(SS_EINVAL, "b or x is NULL");
    if (!(tol >= 0.0) || maxit < 0) return fail(SS_EINVAL, "need tol >= 0 and maxit >= 0");
    int rc = ensure_hist(s, std::min<int64_t>((int64_t)maxit + 1, kHistMax));
    if (rc != SS_OK) return rc;
    const bool fused = s->opts.fused_reduce != 0;

    DevState init{};
    init.tol = tol;
    init.kmax = maxit;
    init.status = ST_RUNNING;
    init.hist = s->hist;
    init.hist_cap = s->hist_cap;
    std::memcpy(s->st_pinned, &init, sizeof(DevState));
    SS_HIP(hipMemcpyAsync(s->st, s->st_pinned, sizeof(DevState), hipMemcpyHostToDevice, s->stream));
    launch_gather<double>(s->stream, s->n_loc, s->l2g, b_dev, s->b);
    launch_gather<double>(s->stream, s->n_loc, s->l2g, x_dev, s->x);

    int32_t status = ST_RUNNING;
    int32_t restarts = -1;
    for (bool first = true;; first = false) {
        ++restarts;
        // r = b - A x, p = r (Algorithm 3, first line; also the convergence check)
        launch_spmv<double, double>(s->stream, s->csr64(), s->x, s->q);
        launch_residual<double>(s->stream, s->iface(), s->b, s->q, s->r, s->p0, s->partial, s->st, first, fused);
        SS_HIP(hipGetLastError());
        if ((rc = read_status(s, &status)) != SS_OK) return rc;
        if (status != ST_RUNNING) break;
        if ((rc = iterate(s)) != SS_OK) return rc;
        if ((rc = read_status(s, &status)) != SS_OK) return rc;
        if (status == ST_BREAKDOWN) break;
    }
    launch_scatter<double>(s->stream, s->n, s->g2own, s->x, x_dev, s->st);
    SS_HIP(hipGetLastError());
    SS_HIP(hipMemcpyAsync(s->st_pinned, s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
    SS_HIP(hipStreamSynchronize(s->stream));
    const DevState &f = *s->st_pinned;
    int code;
    switch (f.status) {
    case ST_CONVERGED:
    case ST_ZERO_RHS: code = SS_OK; break;
    case ST_MAXIT: code = SS_NOT_CONVERGED; break;
    default: code = SS_EBREAKDOWN; break;
    }
    const double relres = f.status == ST_ZERO_RHS ? 0.0 : std::sqrt(f.rr / f.bb);
    if (res) {
        res->status = code;
        res->iterations = f.iter;
        res->outer_iterations = 0;
        res->restarts = restarts;
        res->relres = relres;
        res->true_relres = relres;
    }
    if (hist_host) {
        const int32_t cnt = f.status == ST_ZERO_RHS ? 1 : std::min(f.iter + 1, s->hist_cap);
        SS_HIP(hipMemcpy(hist_host, s->hist, sizeof(double) * cnt, hipMemcpyDeviceToHost));
    }
    if (code == SS_EBREAKDOWN) fail(SS_EBREAKDOWN, "CG breakdown: (p, A p) <= 0 or non-finite value");
    return code;
}

int ss_cg_apply(ss_solver *s, const double *x_dev, double *y_dev)
{
    if (!s || !x_dev || !y_dev) return fail(SS_EINVAL, "NULL argument");
    launch_gather<double>(s->stream, s->n_loc, s->l2g, x_dev, s->p0);
    launch_spmv<double, double>(s->stream, s->csr64(), s->p0, s->q);
    launch_iface_sum<double>(s->stream, s->iface(), s->q);
    launch_scatter<double>(s->stream, s->n, s->g2own, s->q, y_dev, nullptr);
    SS_HIP(hipGetLastError());
    SS_HIP(hipStreamSynchronize(s->stream));
    return SS_OK;
}

int ss_cg_set_values(ss_solver *s, const double *val_dev)
{
    if (!s || !val_dev) return fail(SS_EINVAL, "NULL argument");
    launch_set_values(s->stream, s->nnz, s->nzmap, val_dev, s->val, s->val32);
    SS_HIP(hipGetLastError());
    SS_HIP(hipStreamSynchronize(s->stream));
    return SS_OK;
}

int ss_cg_grad_vals(ss_solver *s, const double *lambda_dev, const double *x_dev, double *dvals_dev)
{
    if (!s || !lambda_dev || !x_dev || !dvals_dev) return fail(SS_EINVAL, "NULL argument");
    launch_grad_vals(s->stream, s->n_loc, s->rowptr, s->colidx, s->nzmap, s->l2g, lambda_dev, x_dev, dvals_dev);
    SS_HIP(hipGetLastError());
    SS_HIP(hipStreamSynchronize(s->stream));
    return SS_OK;
}

int ss_cg_time_spmv(ss_solver *s, int32_t reps, double *ms_per_launch, double *bytes_per_launch)
{
    if (!s || reps < 1 || !ms_per_launch) return fail(SS_EINVAL, "need a solver, reps >= 1 and an output");
    // keep the run state; time the CG-step kernel with p = r = 1 and beta = 0:
    // (1, A 1) > 0 for SPD A, so the status stays RUNNING and every launch
    // does the full work
    SS_HIP(hipMemcpyAsync(s->st_pinned, s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
    SS_HIP(hipStreamSynchronize(s->stream));
    const DevState saved = *s->st_pinned;
    DevState tmp = saved;
    tmp.status = ST_RUNNING;
    tmp.beta = 0.0;
    tmp.rr = 1.0;
    std::memcpy(s->st_pinned, &tmp, sizeof(DevState));
    SS_HIP(hipMemcpyAsync(s->st, s->st_pinned, sizeof(DevState), hipMemcpyHostToDevice, s->stream));
    std::vector<double> ones((size_t)std::max(s->n_loc, 1), 1.0);
    SS_HIP(hipMemcpyAsync(s->p0, ones.data(), sizeof(double) * (size_t)s->n_loc, hipMemcpyHostToDevice, s->stream));
    SS_HIP(hipMemcpyAsync(s->r, ones.data(), sizeof(double) * (size_t)s->n_loc, hipMemcpyHostToDevice, s->stream));
    const bool fused = s->opts.fused_reduce != 0;
    launch_spmv_cg<double, double>(s->stream, s->csr64(), s->p0, s->r, s->p1, s->q, s->partial, s->st, fused);
    SS_HIP(hipEventRecord(s->t0, s->stream));
    for (int32_t k = 0; k < reps; ++k)
        launch_spmv_cg<double, double>(s->stream, s->csr64(), s->p0, s->r, s->p1, s->q, s->partial, s->st, fused);
    SS_HIP(hipEventRecord(s->t1, s->stream));
    SS_HIP(hipGetLastError());
    SS_HIP(hipEventSynchronize(s->t1));
    float ms = 0.0f;
    SS_HIP(hipEventElapsedTime(&ms, s->t0, s->t1));
    *ms_per_launch = (double)ms / reps;
    // values + column indices, row pointers, one read of r and p_{k-1},
    // writes of p_k and q
    if (bytes_per_launch)
        *bytes_per_launch = 12.0 * (double)s->nnz + 4.0 * (double)(s->n_loc + 1) + 4.0 * 8.0 * (double)s->n_loc;
    std::memcpy(s->st_pinned, &saved, sizeof(DevState));
    SS_HIP(hipMemcpyAsync(s->st, s->st_pinned, sizeof(DevState), hipMemcpyHostToDevice, s->stream));
    SS_HIP(hipStreamSynchronize(s->stream));
    return SS_OK;
}

}  // extern "C"
