// Solver driver: device layout and setup, the CG loop of Algorithm 3 with
// device-resident scalars, HIP-graph replay of polled iteration chunks, and
// the solver entry points of ss.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "host_common.h"
#include "kernels.h"
#include "layout.h"
#include "small.h"
#include "ss_internal.h"

using namespace ss;

namespace {

constexpr int kDefaultCheck = 32;
constexpr int32_t kHistMax = 1 << 22;  // residual history entries kept on the device

// ---- device memory of ss_cg_solve_noalloc ----------------------------------
// The run state (DevState, in the first 256 bytes) and the residual history
// (SS_NOALLOC_HIST_MAX doubles) of the solve that allocates nothing: one fixed
// array per GPU, held until the process ends and shared by every such call on
// that GPU.  Host code never uses the name of the array (a host-side stand-in,
// not a device address): it takes the address hipGetSymbolAddress gives for
// the current device at set-up, kept per device below.
constexpr size_t kScratchState = 256;
constexpr size_t kScratchBytes = kScratchState + sizeof(double) * SS_NOALLOC_HIST_MAX;
static_assert(sizeof(DevState) <= kScratchState, "the run state fits its slot");
__device__ __align__(256) static unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// The device address of `scratch` on `device`, which must be current; looked
// up once per device.
int scratch_address(int device, void **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return fail(SS_EDEVICE, "device ordinal out of range");
    if (!g_scratch_dev[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[device] = ptr;
    }
    *out = g_scratch_dev[device];
    return SS_OK;
}
}  // namespace

struct ss_solver {
    int device = 0;
    int64_t col_bytes = 0;     // column data the SpMV reads (see Layout::col_bytes)
    int64_t struct_bytes = 0;  // row structure the SpMV reads (see Layout::struct_bytes)
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;  // private stream used only to capture graphs
    ss_opts opts{};
    DeviceMem mem;

    int32_t n = 0, n_loc = 0, P = 0, ngamma = 0;
    int64_t nnz = 0;

    Mat mat{};
    Iface ifc{};
    int32_t *nzmap = nullptr;  // storage order -> global stored entry (-1: padding)
    double *val = nullptr;
    int32_t *l2g = nullptr, *g2own = nullptr;
    int64_t stored = 0;

    // FP64 work vectors (device position order)
    double *b = nullptr, *x = nullptr, *r = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
    double *part_a = nullptr, *part_b = nullptr, *part_r = nullptr;  // SpMV, update, residual partials
    // Jacobi preconditioner: 1 / a_ii per position, z = D^{-1} r, (r, z) partials
    double *dinv = nullptr, *z = nullptr, *part_b2 = nullptr;
    int32_t *dnz = nullptr;  // global stored entry of each position's diagonal (for new values)
    DevState *st = nullptr;
    double *hist = nullptr;
    int32_t hist_cap = 0;
    void *scratch = nullptr;  // device address of the no-allocation solve's array on this device

    // one-launch solve of a small system (rows == 0: not used)
    SmallMat small{};
    int32_t *small_nz = nullptr;  // global stored entry of each small value slot (-1: padding)

    // FP32-value iterative refinement: FP32 copy of the values, inner vectors
    Mat mat32{};
    float *val32 = nullptr, *d32 = nullptr, *r32 = nullptr, *p32a = nullptr, *p32b = nullptr, *q32 = nullptr;
    DevState *st_in = nullptr;

    // host side
    DevState *st_pinned = nullptr;   // readback of the state
    int32_t *flag_pinned = nullptr;  // two status slots for pipelined polling
    hipEvent_t ev[2] = {nullptr, nullptr};

    // one CG run: its vectors, state and the graph of one polled chunk
    struct Run {
        bool fp32 = false;
        bool ru = false;  // chunk ends with the gated FP64 residual replacement
        void *x = nullptr, *r = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
        void *z = nullptr;  // preconditioned residual (nullptr: none)
        DevState *st = nullptr;
        hipGraphExec_t exec = nullptr;
        hipGraph_t graph = nullptr;
        int32_t pairs = 0;
    } run64, run32;

    Partials partials() const { return Partials{part_a, part_b, mat.grid, ifc.grid, part_b2}; }
};

namespace {

// count elements from the host, followed by pad zero elements
template <typename T>
int upload(ss_solver *s, T **dst, const T *src, size_t count, size_t pad = 0)
{
    *dst = (T *)s->mem.get(sizeof(T) * std::max<size_t>(count + pad, 1));
    if (!*dst) return fail(SS_ENOMEM, "device allocation failed");
    if (count) SS_HIP(hipMemcpyAsync(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice, s->stream));
    if (pad) SS_HIP(hipMemsetAsync(*dst + count, 0, sizeof(T) * pad, s->stream));
    return SS_OK;
}

// The SELL kernels read a whole batch of 64 entries at clamped indexes (a
// chunk without entries reads just past its array), and the chunk lengths
// as 32-bit words: those arrays end with this many zero elements.
constexpr size_t kSellPad = 64;

template <typename T>
int alloc_dev(ss_solver *s, T **dst, size_t count)
{
    *dst = (T *)s->mem.get(sizeof(T) * std::max<size_t>(count, 1));
    return *dst ? SS_OK : fail(SS_ENOMEM, "device allocation failed");
}

void destroy_graph(ss_solver::Run &R)
{
    if (R.exec) (void)hipGraphExecDestroy(R.exec);
    if (R.graph) (void)hipGraphDestroy(R.graph);
    R.exec = nullptr;
    R.graph = nullptr;
    R.pairs = 0;
}

// Pair j of a chunk: the update of iteration k (alpha, x, r) and the SpMV step
// of iteration k+1 (beta, p, A p).  The scalar slot and the p ping-pong
// alternate with j; chunks hold an even number of pairs, so every chunk
// starts from slot 0 with the current p in p1.
template <typename XT>
void enqueue_pair_t(ss_solver *s, const ss_solver::Run &R, const Mat &M, hipStream_t stream, int j)
{
    const int slot = j & 1;
    XT *pcur = (XT *)(slot ? R.p0 : R.p1);
    XT *pnext = (XT *)(slot ? R.p1 : R.p0);
    XT *zr = (XT *)(R.z ? R.z : R.r);  // the vector p is built from: z, or r without preconditioner
    launch_update<XT>(stream, s->ifc, (XT *)R.r, (XT *)R.z, (XT *)R.q, s->partials(), R.st, slot);
    launch_spmv_step<XT, XT>(stream, M, pcur, zr, pnext, (XT *)R.q, (XT *)R.x, s->partials(), R.st, slot);
}

void enqueue_pair(ss_solver *s, const ss_solver::Run &R, hipStream_t stream, int j)
{
    if (R.fp32)
        enqueue_pair_t<float>(s, R, s->mat32, stream, j);
    else
        enqueue_pair_t<double>(s, R, s->mat, stream, j);
}

// A polled chunk: `pairs` (update, step) pairs, then for a residual-
// replacement run the gated replacement.
void enqueue_chunk_work(ss_solver *s, const ss_solver::Run &R, hipStream_t stream, int32_t pairs)
{
    for (int32_t k = 0; k < pairs; ++k) enqueue_pair(s, R, stream, k);
    if (R.ru)
        launch_ru_refresh<float>(stream, s->ifc, s->mat, s->x, (float *)R.x, s->b, s->q, s->r, (float *)R.r,
                                 s->part_r, R.st, s->st);
}

int ensure_chunk_graph(ss_solver *s, ss_solver::Run &R, int32_t pairs)
{
    if (R.exec && R.pairs == pairs) return SS_OK;
    destroy_graph(R);
    SS_HIP(hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal));
    enqueue_chunk_work(s, R, s->cap, pairs);
    hipGraph_t g = nullptr;
    SS_HIP(hipStreamEndCapture(s->cap, &g));
    R.graph = g;
    SS_HIP(hipGraphInstantiate(&R.exec, g, nullptr, nullptr, 0));
    R.pairs = pairs;
    return SS_OK;
}

int enqueue_chunk(ss_solver *s, ss_solver::Run &R, int32_t pairs)
{
    if (s->opts.use_graph) {
        SS_HIP(hipGraphLaunch(R.exec, s->stream));
    } else {
        enqueue_chunk_work(s, R, s->stream, pairs);
        SS_HIP(hipGetLastError());
    }
    return SS_OK;
}

// Runs CG iterations of run R until its device status leaves RUNNING.
// Chunks of `check_every` iterations (even) are queued one ahead of the
// status poll, so the device does not wait for the host.
int iterate(ss_solver *s, ss_solver::Run &R)
{
    int32_t chunk = s->opts.check_every > 0 ? s->opts.check_every : kDefaultCheck;
    chunk += chunk & 1;
    if (s->opts.use_graph) {
        int rc = ensure_chunk_graph(s, R, chunk);
        if (rc != SS_OK) return rc;
    }
    int slot = 0;
    int rc = enqueue_chunk(s, R, chunk);
    if (rc != SS_OK) return rc;
    SS_HIP(hipMemcpyAsync(&s->flag_pinned[slot], &R.st->status, sizeof(int32_t), hipMemcpyDeviceToHost, s->stream));
    SS_HIP(hipEventRecord(s->ev[slot], s->stream));
    for (;;) {
        const int nxt = slot ^ 1;
        rc = enqueue_chunk(s, R, chunk);
        if (rc != SS_OK) return rc;
        SS_HIP(hipMemcpyAsync(&s->flag_pinned[nxt], &R.st->status, sizeof(int32_t), hipMemcpyDeviceToHost,
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

int read_status(ss_solver *s, const DevState *st, int32_t *status)
{
    SS_HIP(hipMemcpyAsync(&s->flag_pinned[0], &st->status, sizeof(int32_t), hipMemcpyDeviceToHost, s->stream));
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

// The setup of ss_cg_setup; band_kind >= 0: the band splitting band_kind into
// nbands bands, p being the one-part partition of A.
int setup_impl(const ss_csr *A, const ss_part *p, const ss_opts *o, void *hip_stream, ss_solver **out,
               int32_t band_kind, int32_t nbands)
{
    if (!out) return fail(SS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return fail(SS_EINVAL, "partition is NULL");
    int rc = validate_csr(A, false);
    if (rc != SS_OK) return rc;
    if (A->n != p->n || (int64_t)A->nnz != p->nnz) return fail(SS_EINVAL, "matrix does not match the partition");
    // the pattern too: every local entry names a stored entry of A in the
    // row and column of its nodes
    for (int32_t r = 0; r < p->n_loc(); ++r) {
        const int32_t gi = p->l2g[r];
        for (int32_t e = p->bd_rowptr[r]; e < p->bd_rowptr[r + 1]; ++e) {
            const int32_t k = p->bd_nzmap[e];
            if (k < A->rowptr[gi] || k >= A->rowptr[gi + 1] || A->colidx[k] != p->l2g[p->bd_colidx[e]])
                return fail(SS_EINVAL, "matrix does not match the partition's pattern (row " + std::to_string(gi) + ")");
        }
    }
    ss_opts opts;
    ss_opts_default(&opts);
    if (o) opts = *o;
    if (opts.precision != SS_FP64 && opts.precision != SS_FP32_IR && opts.precision != SS_FP32_RU)
        return fail(SS_EINVAL, "unknown precision");
    if (opts.precision == SS_FP32_RU && !(opts.ru_delta >= 0.0 && opts.ru_delta <= 1.0))
        return fail(SS_EINVAL, "ru_delta must be in [0, 1]");
    if (opts.precond != SS_PRECOND_NONE && opts.precond != SS_PRECOND_JACOBI)
        return fail(SS_EINVAL, "unknown precond");
    if (opts.precond == SS_PRECOND_JACOBI && opts.precision != SS_FP64)
        return fail(SS_EUNSUPPORTED, "the Jacobi preconditioner is available with SS_FP64 only");
    std::vector<double> diag;
    std::vector<int32_t> diag_nz;
    if (opts.precond == SS_PRECOND_JACOBI) {
        diag.assign((size_t)A->n, 0.0);
        diag_nz.assign((size_t)A->n, -1);
        for (int32_t i = 0; i < A->n; ++i)
            for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
                if (A->colidx[k] == i) {
                    diag[i] = A->val[k];
                    diag_nz[i] = k;
                }
        for (int32_t i = 0; i < A->n; ++i)
            if (!(diag[i] > 0.0) || !std::isfinite(diag[i]))
                return fail(SS_EINVAL, "Jacobi needs a positive diagonal (row " + std::to_string(i) + ")");
    }
    if (opts.tile_nnz != 0 && opts.tile_nnz != 1024 && opts.tile_nnz != 2048 && opts.tile_nnz != 4096)
        return fail(SS_EINVAL, "tile_nnz must be 0, 1024, 2048 or 4096");
    if (opts.matrix_format < SS_MAT_AUTO || opts.matrix_format > SS_MAT_CSR)
        return fail(SS_EINVAL, "unknown matrix_format");
    if ((opts.alloc == nullptr) != (opts.free == nullptr)) return fail(SS_EINVAL, "alloc and free go together");
    if (opts.spmv_grid < 0 || opts.spmv_grid > kGridLimit) return fail(SS_EINVAL, "spmv_grid must be in [0, 65536]");
    if (opts.small_solver != SS_SMALL_AUTO && opts.small_solver != SS_SMALL_OFF)
        return fail(SS_EINVAL, "unknown small_solver");
    if (opts.precision == SS_FP32_IR && !(opts.inner_tol > 0.0 && opts.inner_tol < 1.0))
        return fail(SS_EINVAL, "inner_tol must be in (0, 1)");

    const bool band_col = band_kind == SS_BAND_COL && nbands > 1;
    if (band_kind >= 0 && opts.precision != SS_FP64)
        return fail(SS_EUNSUPPORTED, "the band splittings are available with SS_FP64 only");
    if (band_col && opts.matrix_format == SS_MAT_CSR)
        return fail(SS_EUNSUPPORTED, "the band-column product needs the SELL layout");

    Layout L;
    try {
        build_order(p, L);
        build_matrix(p, L, opts.tile_nnz ? opts.tile_nnz : 2048, band_col ? SS_MAT_SELL : opts.matrix_format,
                     opts.spmv_grid);
    } catch (const std::bad_alloc &) {
        return fail(SS_ENOMEM, "host allocation failed");
    }
    if (!L.encode_ok) return fail(SS_EINVAL, "internal: column encoding check failed");
    if (band_kind >= 0) {
        // one part: every position is the global index it holds, so a
        // column position is a global column
        for (size_t c = 0; c < L.l2g.size(); ++c)
            if (L.l2g[c] != (int32_t)c) return fail(SS_EINVAL, "internal: one-part positions are not global ids");
        if (band_col && L.fmt != FMT_SELL)
            return fail(SS_EUNSUPPORTED, "the band-column product needs rows of at most 255 entries");
    }

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
    // the no-allocation solve's array: an unavailable one fails that call only
    if (scratch_address(s->device, &s->scratch) != SS_OK) {
        s->scratch = nullptr;
        (void)hipGetLastError();
    }
    if (hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(SS_EDEVICE, "stream creation failed"));
    for (auto &e : s->ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return bail(fail(SS_EDEVICE, "event creation failed"));
    if (hipHostMalloc((void **)&s->st_pinned, sizeof(DevState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&s->flag_pinned, 4 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess)
        return bail(fail(SS_ENOMEM, "pinned host allocation failed"));

    s->n = p->n;
    s->n_loc = p->n_loc();
    s->P = p->P;
    s->nnz = p->nnz;
    s->ngamma = (int32_t)p->gamma.size();
    s->stored = L.stored;
    s->col_bytes = L.col_bytes;
    s->struct_bytes = L.struct_bytes;

    std::vector<double> val_st((size_t)L.stored, 0.0);
    for (int64_t k = 0; k < L.stored; ++k)
        if (L.nzmap[k] >= 0) val_st[k] = A->val[L.nzmap[k]];

    Mat &M = s->mat;
    M.fmt = L.fmt;
    M.nrows = s->n_loc;
    M.nchunks = L.nchunks;
    M.unroll = L.unroll;
    M.one_batch = L.one_batch;
    M.band_m = band_kind >= 0 ? A->n / nbands : 0;
    M.nbands = band_col ? nbands : 0;
    M.ntiles = L.ntiles;
    M.tile_nnz = L.tile_nnz;
    M.grid = spmv_grid(L.fmt == FMT_SELL, L.fmt == FMT_SELL ? L.nchunks : L.ntiles, opts.spmv_grid);
    Iface &I = s->ifc;
    I.n_loc = s->n_loc;
    I.n_own = L.n_own;
    I.n_if = L.n_if;
    I.ngamma = s->ngamma;
    I.grid = std::max(1, (s->n_loc + kUI * kBS - 1) / (kUI * kBS));

    int32_t *d_col = nullptr, *d_cptr = nullptr, *d_cpos = nullptr, *d_rowptr = nullptr, *d_tile = nullptr, *d_pos_grp = nullptr,
            *d_copy_ptr = nullptr, *d_copy_pos = nullptr, *d_ccol = nullptr;
    uint16_t *d_col16 = nullptr;
    int32_t *d_cbase = nullptr;
    uint8_t *d_clen = nullptr, *d_rlen = nullptr;
    int32_t *d_cdict = nullptr, *d_dtab = nullptr;
    uint32_t *d_dword = nullptr;
    const size_t nl = (size_t)s->n_loc;
    if ((rc = upload(s, &d_col, L.col.data(), L.col.size(), kSellPad)) ||
        (rc = upload(s, &d_col16, L.col16.data(), L.col16.size(), kSellPad)) ||
        (rc = upload(s, &d_ccol, L.ccol.data(), L.ccol.size())) ||
        (rc = upload(s, &d_cbase, L.cbase.data(), L.cbase.size())) ||
        (rc = upload(s, &s->nzmap, L.nzmap.data(), L.nzmap.size())) ||
        (rc = upload(s, &s->val, val_st.data(), val_st.size(), kSellPad)) ||
        (rc = upload(s, &d_cptr, L.cptr.data(), L.cptr.size())) ||
        (rc = upload(s, &d_cpos, L.cpos.data(), L.cpos.size())) ||
        (rc = upload(s, &d_clen, L.clen.data(), L.clen.size(), kSellPad)) ||
        (rc = upload(s, &d_rlen, L.rlen.data(), L.rlen.size())) ||
        (rc = upload(s, &d_cdict, L.cdict.data(), L.cdict.size())) ||
        (rc = upload(s, &d_dtab, L.dtab.data(), L.dtab.size(), kSellPad)) ||
        (rc = upload(s, &d_dword, L.dword.data(), L.dword.size(), kSellPad)) ||
        (rc = upload(s, &d_rowptr, L.rowptr.data(), L.rowptr.size())) ||
        (rc = upload(s, &d_tile, L.tile_row.data(), L.tile_row.size())) ||
        (rc = upload(s, &s->l2g, L.l2g.data(), L.l2g.size())) ||
        (rc = upload(s, &s->g2own, L.g2own.data(), L.g2own.size())) ||
        (rc = upload(s, &d_copy_ptr, p->copy_ptr.data(), p->copy_ptr.size())) ||
        (rc = upload(s, &d_copy_pos, L.copy_pos.data(), L.copy_pos.size())) ||
        (rc = upload(s, &d_pos_grp, L.pos_grp.data(), L.pos_grp.size())) || (rc = alloc_dev(s, &s->b, nl)) ||
        (rc = alloc_dev(s, &s->x, nl)) || (rc = alloc_dev(s, &s->r, nl)) || (rc = alloc_dev(s, &s->p0, nl)) ||
        (rc = alloc_dev(s, &s->p1, nl)) || (rc = alloc_dev(s, &s->q, nl)) || (rc = alloc_dev(s, &s->st, 1)) ||
        (rc = alloc_dev(s, &s->part_a, (size_t)M.grid)) || (rc = alloc_dev(s, &s->part_b, (size_t)I.grid)) ||
        (rc = alloc_dev(s, &s->part_r, 3 * (size_t)I.grid)))
        return bail(rc);
    if (opts.precond == SS_PRECOND_JACOBI) {
        std::vector<double> dinv(nl);
        std::vector<int32_t> dnz(nl);
        for (size_t c = 0; c < nl; ++c) {
            dinv[c] = 1.0 / diag[(size_t)L.l2g[c]];
            dnz[c] = diag_nz[(size_t)L.l2g[c]];
        }
        if ((rc = upload(s, &s->dinv, dinv.data(), dinv.size())) || (rc = upload(s, &s->dnz, dnz.data(), dnz.size())) ||
            (rc = alloc_dev(s, &s->z, nl)) || (rc = alloc_dev(s, &s->part_b2, (size_t)I.grid)))
            return bail(rc);
        I.dinv = s->dinv;
    }
    if (opts.precision != SS_FP64) {
        std::vector<float> v32(val_st.size());
        for (size_t k = 0; k < v32.size(); ++k) v32[k] = (float)val_st[k];
        if ((rc = upload(s, &s->val32, v32.data(), v32.size(), kSellPad)) || (rc = alloc_dev(s, &s->d32, nl)) ||
            (rc = alloc_dev(s, &s->r32, nl)) || (rc = alloc_dev(s, &s->p32a, nl)) ||
            (rc = alloc_dev(s, &s->p32b, nl)) || (rc = alloc_dev(s, &s->q32, nl)) || (rc = alloc_dev(s, &s->st_in, 1)))
            return bail(rc);
    }
    M.col = d_col;
    M.col16 = d_col16;
    M.ccol = d_ccol;
    M.cbase = reinterpret_cast<const int2 *>(d_cbase);
    M.val = s->val;
    M.cptr = d_cptr;
    M.cpos = d_cpos;
    M.clen = d_clen;
    M.rlen = d_rlen;
    M.cdict = L.dtab.empty() ? nullptr : d_cdict;
    M.dtab = d_dtab;
    M.dword = d_dword;
    M.dict_batches = L.dict_batches;
    M.rowptr = d_rowptr;
    M.tile_row = d_tile;
    I.pos_grp = d_pos_grp;
    I.copy_ptr = d_copy_ptr;
    I.copy_pos = d_copy_pos;
    s->mat32 = M;
    s->mat32.val = s->val32;
    s->run64.fp32 = false;
    s->run64.x = s->x;
    s->run64.r = s->r;
    s->run64.p0 = s->p0;
    s->run64.p1 = s->p1;
    s->run64.q = s->q;
    s->run64.z = s->z;
    s->run64.st = s->st;
    s->run32.fp32 = true;
    s->run32.ru = opts.precision == SS_FP32_RU;
    s->run32.x = s->d32;
    s->run32.r = s->r32;
    s->run32.p0 = s->p32a;
    s->run32.p1 = s->p32b;
    s->run32.q = s->q32;
    s->run32.st = s->st_in;

    // A small system (FP64, M = I, rows of at most 7 entries, at most 4608
    // positions with 5-entry rows or 3840 with 7, x, r, p and the interface
    // products within the LDS a workgroup may take) is solved by one launch
    // per solve.
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, s->device) != hipSuccess)
        lds_max = 0;
    if (opts.precision == SS_FP64 && opts.precond == SS_PRECOND_NONE && band_kind < 0 &&
        opts.small_solver == SS_SMALL_AUTO && s->n_loc > 0) {
        int32_t wmax = 0;
        for (int32_t u = 0; u < s->n_loc; ++u) wmax = std::max(wmax, p->bd_rowptr[u + 1] - p->bd_rowptr[u]);
        const int32_t width = wmax <= 5 ? 5 : 7;
        const int32_t rows = small_rows((s->n_loc + kSmallThreads - 1) / kSmallThreads, width);
        if (wmax <= 7 && rows > 0 && s->n_loc <= 65536 &&
            small_lds_bytes(s->n_loc, L.n_if, s->ngamma, (int32_t)p->copy_pos.size()) <=
                (size_t)std::max(lds_max, 0)) {
            std::vector<double> sv;
            std::vector<uint32_t> sc;
            try {
                build_small(p, L, A->val, width, sv, sc);
            } catch (const std::bad_alloc &) {
                return bail(fail(SS_ENOMEM, "host allocation failed"));
            }
            // where each value slot comes from, for new values (ss_cg_set_values)
            std::vector<int32_t> snz(sv.size(), -1);
            {
                std::vector<int32_t> src(nl);
                for (int32_t u = 0; u < s->n_loc; ++u) src[L.dev_pos[u]] = u;
                for (int32_t t = 0; t < s->n_loc; ++t) {
                    const int32_t u = src[t], e0 = p->bd_rowptr[u], len = p->bd_rowptr[u + 1] - e0;
                    for (int32_t j = 0; j < len; ++j) snz[(size_t)j * nl + t] = p->bd_nzmap[e0 + j];
                }
            }
            double *d_sv = nullptr;
            uint32_t *d_sc = nullptr;
            if ((rc = upload(s, &d_sv, sv.data(), sv.size())) || (rc = upload(s, &d_sc, sc.data(), sc.size())) ||
                (rc = upload(s, &s->small_nz, snz.data(), snz.size())))
                return bail(rc);
            s->small = SmallMat{s->n_loc, (int32_t)p->copy_pos.size(), rows, width, d_sv, d_sc};
        }
    }

    DevState init{};
    std::memcpy(s->st_pinned, &init, sizeof(DevState));
    if (hipMemcpyAsync(s->st, s->st_pinned, sizeof(DevState), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return bail(fail(SS_EDEVICE, "upload failed"));
    *out = s;
    return SS_OK;
}

}  // namespace

extern "C" {

void ss_opts_default(ss_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = SS_FP64;
    o->inner_tol = 1e-6;
    o->ru_delta = 0.1;
    o->inner_maxit = 0;
    o->max_outer = 50;
    o->check_every = kDefaultCheck;
    o->use_graph = 1;
    o->tile_nnz = 0;
    o->matrix_format = SS_MAT_AUTO;
}

void ss_cg_destroy(ss_solver *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    destroy_graph(s->run64);
    destroy_graph(s->run32);
    for (auto &e : s->ev)
        if (e) (void)hipEventDestroy(e);
    if (s->st_pinned) (void)hipHostFree(s->st_pinned);
    if (s->flag_pinned) (void)hipHostFree(s->flag_pinned);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    s->mem.clear();
    delete s;
}


int ss_cg_setup(const ss_csr *A, const ss_part *p, const ss_opts *o, void *hip_stream, ss_solver **out)
{
    return setup_impl(A, p, o, hip_stream, out, -1, 0);
}

int ss_band_setup(const ss_csr *A, int32_t kind, int32_t nbands, const ss_opts *o, void *hip_stream,
                  ss_solver **out)
{
    if (!out) return fail(SS_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_csr(A, false);
    if (rc != SS_OK) return rc;
    if (kind != SS_BAND_ROW && kind != SS_BAND_COL) return fail(SS_EINVAL, "unknown band kind");
    if (nbands < 1 || nbands > A->n) return fail(SS_EINVAL, "nbands must be in [1, n]");
    std::vector<int32_t> zero;
    try {
        zero.assign((size_t)A->n, 0);
    } catch (const std::bad_alloc &) {
        return fail(SS_ENOMEM, "host allocation failed");
    }
    ss_part *p = nullptr;
    rc = ss_partition(A, SS_PART_USER, 1, 0, nullptr, nullptr, nullptr, nullptr, zero.data(), &p);
    if (rc != SS_OK) return rc;
    rc = setup_impl(A, p, o, hip_stream, out, kind, nbands);
    ss_part_destroy(p);
    return rc;
}

int ss_cg_path(const ss_solver *s, int32_t *path)
{
    if (!s || !path) return fail(SS_EINVAL, "NULL argument");
    *path = s->small.rows > 0 ? SS_PATH_SMALL : SS_PATH_STREAM;
    return SS_OK;
}

int ss_cg_info(const ss_solver *s, int32_t *n, int32_t *n_loc, int64_t *nnz, int32_t *matrix_format,
               int64_t *stored)
{
    if (!s) return fail(SS_EINVAL, "solver is NULL");
    if (n) *n = s->n;
    if (n_loc) *n_loc = s->n_loc;
    if (nnz) *nnz = s->nnz;
    if (matrix_format) *matrix_format = s->mat.fmt == FMT_SELL ? SS_MAT_SELL : SS_MAT_CSR;
    if (stored) *stored = s->stored;
    return SS_OK;
}

}  // extern "C"

namespace {

// The solve of ss_cg_solve on the solver's run state s->st, history s->hist
// (capacity s->hist_cap, or none) and the launch mode s->opts.use_graph.
int solve_core(ss_solver *s, const double *b_dev, double *x_dev, double tol, int32_t maxit, ss_result *res,
               double *hist_host)
{
    int rc = SS_OK;
    DevState init{};
    init.tol = tol;
    init.kmax = maxit;
    init.status = ST_RUNNING;
    init.hist = s->hist;
    init.hist_cap = s->hist_cap;
    std::memcpy(s->st_pinned, &init, sizeof(DevState));
    SS_HIP(hipMemcpyAsync(s->st, s->st_pinned, sizeof(DevState), hipMemcpyHostToDevice, s->stream));
    launch_gather<double, double>(s->stream, s->n_loc, s->l2g, b_dev, s->b);
    launch_gather<double, double>(s->stream, s->n_loc, s->l2g, x_dev, s->x);

    int32_t status = ST_RUNNING;
    int32_t restarts = -1, outer = 0;
    bool outer_cap = false;  // IR stopped by max_outer
    if (s->opts.precision == SS_FP64 && s->small.rows > 0) {
        // the whole solve in one launch; its restart count comes back in the state
        launch_cg_small(s->stream, s->small, s->ifc, s->b, s->x, s->st);
        SS_HIP(hipGetLastError());
        restarts = 0;
    } else if (s->opts.precision == SS_FP64) {
        for (bool first = true;; first = false) {
            ++restarts;
            // r = b - A x, p = r (Algorithm 3, first line; also the convergence check)
            launch_spmv<double, double>(s->stream, s->mat, s->x, s->q);
            launch_residual<double>(s->stream, s->ifc, s->b, s->q, s->r, s->z, s->p0, s->part_r, s->st, first);
            SS_HIP(hipGetLastError());
            if ((rc = read_status(s, s->st, &status)) != SS_OK) return rc;
            if (status != ST_RUNNING) break;
            // p_1 = r_1, A p_1, then (update, step) pairs until the status changes
            // p_1 = z_1 (= r_1 without preconditioner)
            launch_spmv_first<double, double>(s->stream, s->mat, s->p0, s->z ? s->z : s->r, s->p1, s->q,
                                              s->partials(), s->st);
            if ((rc = iterate(s, s->run64)) != SS_OK) return rc;
            if ((rc = read_status(s, s->st, &status)) != SS_OK) return rc;
            if (status == ST_BREAKDOWN) break;
        }
    } else if (s->opts.precision == SS_FP32_RU) {
        // FP32 CG with FP64 residual replacement: every (re)start takes the
        // FP64 residual; the polled chunks end with the gated replacement
        SS_HIP(hipMemsetAsync(&s->st_in->nrefresh, 0, sizeof(int32_t), s->stream));
        for (bool first = true;; first = false) {
            ++restarts;
            launch_spmv<double, double>(s->stream, s->mat, s->x, s->q);
            launch_residual<double>(s->stream, s->ifc, s->b, s->q, s->r, s->z, s->p0, s->part_r, s->st, first);
            SS_HIP(hipGetLastError());
            if ((rc = read_status(s, s->st, &status)) != SS_OK) return rc;
            if (status != ST_RUNNING) break;
            launch_ru_start<float>(s->stream, s->ifc, s->r, s->r32, s->d32, s->part_r, s->st, s->st_in,
                                   s->opts.ru_delta);
            launch_spmv_first<float, float>(s->stream, s->mat32, s->r32, s->r32, s->p32b, s->q32, s->partials(),
                                            s->st_in);
            if ((rc = iterate(s, s->run32)) != SS_OK) return rc;
            launch_ru_fold<float>(s->stream, s->n_loc, s->x, s->d32, s->st_in, s->st);
            SS_HIP(hipGetLastError());
            if ((rc = read_status(s, s->st, &status)) != SS_OK) return rc;
            if (status == ST_BREAKDOWN) break;
        }
        int32_t nref = 0;
        SS_HIP(hipMemcpyAsync(&s->flag_pinned[0], &s->st_in->nrefresh, sizeof(int32_t), hipMemcpyDeviceToHost,
                              s->stream));
        SS_HIP(hipStreamSynchronize(s->stream));
        nref = s->flag_pinned[0];
        outer = nref;
    } else {
        // outer: FP64 residual of the FP64 matrix; inner: CG on the FP32 values
        // with FP32 vectors for the scaled residual; x += ||r|| d
        const int32_t max_outer = s->opts.max_outer > 0 ? s->opts.max_outer : 50;
        restarts = 0;
        for (;; ++outer) {
            launch_spmv<double, double>(s->stream, s->mat, s->x, s->q);
            launch_residual<double>(s->stream, s->ifc, s->b, s->q, s->r, s->z, s->p0, s->part_r, s->st, outer == 0);
            SS_HIP(hipGetLastError());
            if ((rc = read_status(s, s->st, &status)) != SS_OK) return rc;
            if (status != ST_RUNNING) break;
            if (outer >= max_outer) {
                outer_cap = true;
                break;
            }
            launch_ir_prepare<float>(s->stream, s->ifc, s->r, s->r32, s->p32a, s->d32, s->part_r, s->st, s->st_in,
                                     s->opts.inner_tol, s->opts.inner_maxit, maxit);
            int32_t si = ST_RUNNING;
            if ((rc = read_status(s, s->st_in, &si)) != SS_OK) return rc;
            if (si == ST_RUNNING) {
                launch_spmv_first<float, float>(s->stream, s->mat32, s->p32a, s->r32, s->p32b, s->q32, s->partials(),
                                                s->st_in);
                if ((rc = iterate(s, s->run32)) != SS_OK) return rc;
            }
            launch_ir_accumulate<float>(s->stream, s->n_loc, s->x, s->d32, s->st_in, s->st);
            SS_HIP(hipGetLastError());
            if ((rc = read_status(s, s->st, &status)) != SS_OK) return rc;
            if (status == ST_BREAKDOWN) break;
        }
    }
    launch_scatter<double, double>(s->stream, s->n, s->g2own, s->x, x_dev, s->st);
    SS_HIP(hipGetLastError());
    SS_HIP(hipMemcpyAsync(s->st_pinned, s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
    SS_HIP(hipStreamSynchronize(s->stream));
    const DevState &f = *s->st_pinned;
    int code;
    switch (f.status) {
    case ST_CONVERGED:
    case ST_ZERO_RHS: code = SS_OK; break;
    case ST_MAXIT: code = SS_NOT_CONVERGED; break;
    case ST_RUNNING: code = SS_NOT_CONVERGED; break;  // IR stopped by max_outer
    default: code = SS_EBREAKDOWN; break;
    }
    (void)outer_cap;
    const double relres = f.status == ST_ZERO_RHS ? 0.0 : std::sqrt(f.rr_last / f.bb);
    if (s->opts.precision == SS_FP64 && s->small.rows > 0) restarts = f.restarts;
    if (res) {
        res->status = code;
        res->iterations = f.iter_last;
        res->outer_iterations = outer;
        res->restarts = restarts;
        res->relres = relres;
        res->true_relres = relres;
    }
    if (hist_host && s->hist) {
        const int32_t cnt = f.status == ST_ZERO_RHS ? 1 : std::min(f.iter_last + 1, s->hist_cap);
        SS_HIP(hipMemcpy(hist_host, s->hist, sizeof(double) * cnt, hipMemcpyDeviceToHost));
    }
    if (code == SS_EBREAKDOWN) fail(SS_EBREAKDOWN, "CG breakdown: (p, A p) <= 0 or non-finite value");
    return code;
}

}  // namespace

extern "C" {

int ss_cg_solve(ss_solver *s, const double *b_dev, double *x_dev, double tol, int32_t maxit, ss_result *res,
                double *hist_host)
{
    if (!s) return fail(SS_EINVAL, "solver is NULL");
    if (!b_dev || !x_dev) return fail(SS_EINVAL, "b or x is NULL");
    if (!(tol >= 0.0) || maxit < 0) return fail(SS_EINVAL, "need tol >= 0 and maxit >= 0");
    const int rc = ensure_hist(s, std::min<int64_t>((int64_t)maxit + 1, kHistMax));
    if (rc != SS_OK) return rc;
    return solve_core(s, b_dev, x_dev, tol, maxit, res, hist_host);
}

int ss_cg_solve_noalloc(ss_solver *s, const double *b_dev, double *x_dev, double tol, int32_t maxit,
                        ss_result *res, double *hist_host)
{
    if (!s) return fail(SS_EINVAL, "solver is NULL");
    if (!b_dev || !x_dev) return fail(SS_EINVAL, "b or x is NULL");
    if (!(tol >= 0.0) || maxit < 0) return fail(SS_EINVAL, "need tol >= 0 and maxit >= 0");
    if (s->opts.precision != SS_FP64)
        return fail(SS_EUNSUPPORTED, "the no-allocation solve is available with SS_FP64 only");
    if (hist_host && (int64_t)maxit + 1 > SS_NOALLOC_HIST_MAX)
        return fail(SS_EINVAL, "with a history, maxit + 1 must not exceed SS_NOALLOC_HIST_MAX (" +
                                   std::to_string(SS_NOALLOC_HIST_MAX) + ")");
    if (!s->scratch)
        return fail(SS_EDEVICE, "the device array of the no-allocation solve was not found at set-up");
    // the run state and history in the device's fixed array, chunks launched
    // one by one (no graph is instantiated); the whole state is written at
    // the start of the solve, history entries before they are read
    DevState *const st = reinterpret_cast<DevState *>(s->scratch);
    double *const hist = hist_host ? reinterpret_cast<double *>(static_cast<char *>(s->scratch) + kScratchState)
                                   : nullptr;
    DevState *const st0 = s->st;
    double *const hist0 = s->hist;
    const int32_t cap0 = s->hist_cap, graph0 = s->opts.use_graph;
    s->st = st;
    s->run64.st = st;
    s->hist = hist;
    s->hist_cap = hist ? maxit + 1 : 0;
    s->opts.use_graph = 0;
    const int rc = solve_core(s, b_dev, x_dev, tol, maxit, res, hist_host);
    s->st = st0;
    s->run64.st = st0;
    s->hist = hist0;
    s->hist_cap = cap0;
    s->opts.use_graph = graph0;
    return rc;
}

int ss_cg_apply(ss_solver *s, const double *x_dev, double *y_dev)
{
    if (!s || !x_dev || !y_dev) return fail(SS_EINVAL, "NULL argument");
    launch_gather<double, double>(s->stream, s->n_loc, s->l2g, x_dev, s->p0);
    launch_spmv<double, double>(s->stream, s->mat, s->p0, s->q);
    launch_iface_sum<double>(s->stream, s->ifc, s->q);
    launch_scatter<double, double>(s->stream, s->n, s->g2own, s->q, y_dev, nullptr);
    SS_HIP(hipGetLastError());
    SS_HIP(hipStreamSynchronize(s->stream));
    return SS_OK;
}

int ss_cg_apply_f32(ss_solver *s, const float *x_dev, float *y_dev)
{
    if (!s || !x_dev || !y_dev) return fail(SS_EINVAL, "NULL argument");
    if (!s->val32) return fail(SS_EUNSUPPORTED, "the FP32 product needs a solver set up with an FP32 precision");
    launch_gather<float, float>(s->stream, s->n_loc, s->l2g, x_dev, s->p32a);
    launch_spmv<float, float>(s->stream, s->mat32, s->p32a, s->q32);
    launch_iface_sum<float>(s->stream, s->ifc, s->q32);
    launch_scatter<float, float>(s->stream, s->n, s->g2own, s->q32, y_dev, nullptr);
    SS_HIP(hipGetLastError());
    SS_HIP(hipStreamSynchronize(s->stream));
    return SS_OK;
}

int ss_cg_set_values(ss_solver *s, const double *val_dev)
{
    if (!s || !val_dev) return fail(SS_EINVAL, "NULL argument");
    launch_set_values(s->stream, s->stored, s->nzmap, val_dev, s->val, s->val32);
    if (s->small.rows > 0)
        launch_set_values(s->stream, (int64_t)s->small.width * s->n_loc, s->small_nz, val_dev,
                          const_cast<double *>(s->small.val), nullptr);
    if (s->dinv) launch_set_dinv(s->stream, s->n_loc, s->dnz, val_dev, s->dinv);
    SS_HIP(hipGetLastError());
    SS_HIP(hipStreamSynchronize(s->stream));
    return SS_OK;
}

int ss_cg_grad_vals(ss_solver *s, const double *lambda_dev, const double *x_dev, double *dvals_dev)
{
    if (!s || !lambda_dev || !x_dev || !dvals_dev) return fail(SS_EINVAL, "NULL argument");
    launch_grad_vals(s->stream, s->mat, s->nzmap, s->l2g, lambda_dev, x_dev, dvals_dev);
    SS_HIP(hipGetLastError());
    SS_HIP(hipStreamSynchronize(s->stream));
    return SS_OK;
}

int ss_cg_time_spmv(ss_solver *s, int32_t reps, double *ms_per_launch, double *bytes_per_launch)
{
    if (!s || reps < 1 || !ms_per_launch) return fail(SS_EINVAL, "need a solver, reps >= 1 and an output");
    // Keep the run state; time the CG-step SpMV as it runs inside the loop
    // (the FP32 inner step for an FP32_IR solver): p = r = 1, update partials
    // of 1 each, (r, r) slot 0 = 1, no stopping (stop = 0, unbounded
    // iterations, no history), so every launch finishes the reduction, reads
    // slot 0, writes slot 1 and does the full work.
    const bool f32 = s->opts.precision != SS_FP64;
    DevState *st = f32 ? s->st_in : s->st;
    SS_HIP(hipMemcpyAsync(s->st_pinned, st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
    SS_HIP(hipStreamSynchronize(s->stream));
    const DevState saved = *s->st_pinned;
    DevState tmp{};
    tmp.rr[0] = 1.0;
    tmp.rz[0] = 1.0;
    tmp.iter[0] = 0;
    tmp.bb = 1.0;
    tmp.stop = 0.0;
    tmp.kmax = INT32_MAX;
    tmp.status = ST_RUNNING;
    std::memcpy(s->st_pinned, &tmp, sizeof(DevState));
    SS_HIP(hipMemcpyAsync(st, s->st_pinned, sizeof(DevState), hipMemcpyHostToDevice, s->stream));
    const Partials P = s->partials();
    const size_t nl = (size_t)s->n_loc;
    std::vector<double> ones((size_t)std::max({s->n_loc, P.nb, 1}), 1.0);
    std::vector<float> onesf(std::max<size_t>(nl, 1), 1.0f);
    if (f32) {
        SS_HIP(hipMemcpyAsync(s->p32b, onesf.data(), sizeof(float) * nl, hipMemcpyHostToDevice, s->stream));
        SS_HIP(hipMemcpyAsync(s->r32, onesf.data(), sizeof(float) * nl, hipMemcpyHostToDevice, s->stream));
    } else {
        SS_HIP(hipMemcpyAsync(s->p1, ones.data(), sizeof(double) * nl, hipMemcpyHostToDevice, s->stream));
        SS_HIP(hipMemcpyAsync(s->r, ones.data(), sizeof(double) * nl, hipMemcpyHostToDevice, s->stream));
    }
    SS_HIP(hipMemcpyAsync(P.b, ones.data(), sizeof(double) * (size_t)P.nb, hipMemcpyHostToDevice, s->stream));
    if (P.b2) SS_HIP(hipMemcpyAsync(P.b2, ones.data(), sizeof(double) * (size_t)P.nb, hipMemcpyHostToDevice, s->stream));
    auto launch = [&]() {
        if (f32)
            launch_spmv_step<float, float>(s->stream, s->mat32, s->p32b, s->r32, s->p32a, s->q32, s->d32, P, st, 0);
        else
            launch_spmv_step<double, double>(s->stream, s->mat, s->p1, s->r, s->p0, s->q, s->x, P, st, 0);
    };
    launch();
    // one event pair around `reps` back-to-back launches: the average
    // includes the (sub-microsecond) dispatch gaps, as inside the CG loop
    hipEvent_t ev[2] = {nullptr, nullptr};
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &f : ev)
                if (f) (void)hipEventDestroy(f);
            return fail(SS_EDEVICE, "event creation failed");
        }
    (void)hipEventRecord(ev[0], s->stream);
    for (int32_t k = 0; k < reps; ++k) launch();
    (void)hipEventRecord(ev[1], s->stream);
    hipError_t err = hipGetLastError();
    if (err == hipSuccess) err = hipEventSynchronize(ev[1]);
    float total = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&total, ev[0], ev[1]);
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (err != hipSuccess) return fail(SS_EDEVICE, std::string("SpMV timing: ") + hipGetErrorString(err));
    *ms_per_launch = total / reps;
    // values and column data of the stored entries, the row structure the
    // format reads, one read of r, p_(k-1) and x, writes of p_k, q and x (the
    // split step also reads p_k back for the SpMV)
    const double sv = f32 ? 4.0 : 8.0;
    if (bytes_per_launch)
        *bytes_per_launch = sv * (double)s->nnz + (double)s->col_bytes + (double)s->struct_bytes +
                            (split_step(f32 ? s->mat32 : s->mat) ? 7.0 : 6.0) * sv * (double)s->n_loc;
    std::memcpy(s->st_pinned, &saved, sizeof(DevState));
    SS_HIP(hipMemcpyAsync(st, s->st_pinned, sizeof(DevState), hipMemcpyHostToDevice, s->stream));
    SS_HIP(hipStreamSynchronize(s->stream));
    return SS_OK;
}

}  // extern "C"
