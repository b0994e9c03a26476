// HIP kernels of the sub-structured CG for gfx950 (MI355X).
//
// Hot path of one CG iteration (Algorithm 3, M = I) with every sub-domain
// resident on the device, two launches:
//   k_spmv  (CG mode): p_k = r_k + beta p_{k-1} recomputed on the fly, the
//           local SpMV of every sub-domain on the block-diagonal CSR
//           (Section 4.4.1, first step) and the partial (p, A_s p) sums;
//           the finishing workgroup forms alpha = (r, r) / (p, A p).
//   k_update: interface assembly (Algorithms 4 and 5: every copy of an
//           interface node reads all copies and adds them in ascending
//           sub-domain order), x += alpha p, r -= alpha q and the weighted
//           local (r, r) (Section 4.4.2); the finishing workgroup forms beta
//           and the convergence flag.
// Reductions are fixed-order (per-thread sequential, 64-lane butterfly, then
// a sequential sum over waves and over workgroup partials), hence bitwise
// reproducible run to run.  The file is compiled with -ffp-contract=off:
// products and sums are rounded separately, as the expressions are written.
#include "kernels.h"

#include <cmath>

namespace ss {
namespace {

__device__ __forceinline__ int xcd_remap(int b, int grid)
{
    // workgroup b runs on XCD b % 8; give each XCD a contiguous range of work
    const int per = grid / kNumXcd;
    return (b % kNumXcd) * per + b / kNumXcd;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = v + __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup; result valid in thread 0.  ws: kBS/64 slots.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *ws)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) ws[w] = v;
    __syncthreads();
    T t = T(0);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kBS / 64; ++i) t = t + ws[i];
    }
    __syncthreads();
    return t;
}

__device__ __forceinline__ double sum_partials(const double *partial, int n, double *ws)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += kBS) v = v + partial[i];
    return block_sum(v, ws);
}

// Publishes this workgroup's partial(s); true in every thread of the
// workgroup that arrives last.  Agent-scope fences make the partials of all
// XCDs visible to it.
template <int NV>
__device__ __forceinline__ bool arrive(const double (&v)[NV], double *partial, uint32_t *counter)
{
    __shared__ int last;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int t = 0; t < NV; ++t) partial[t * gridDim.x + blockIdx.x] = v[t];
        __threadfence();
        const uint32_t prev = atomicAdd(counter, 1u);
        last = (prev == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    const bool is_last = last != 0;
    if (is_last) {
        __threadfence();
        if (threadIdx.x == 0) *counter = 0u;
    }
    return is_last;
}

// ---- finishing steps (one workgroup) ---------------------------------------

__device__ void finish_alpha(DevState *st, const double *partial, int n, double *ws)
{
    const double pAp = sum_partials(partial, n, ws);
    if (threadIdx.x == 0) {
        st->pAp = pAp;
        if (!(pAp > 0.0) || !isfinite(pAp))
            st->status = ST_BREAKDOWN;
        else
            st->alpha = st->rr / pAp;
    }
}

__device__ void finish_beta(DevState *st, const double *partial, int n, double *ws)
{
    const double rr1 = sum_partials(partial, n, ws);
    if (threadIdx.x == 0) {
        if (!isfinite(rr1)) {
            st->status = ST_BREAKDOWN;
            return;
        }
        st->beta = rr1 / st->rr;
        st->rr = rr1;
        const int k = ++st->iter;
        if (st->hist && k < st->hist_cap) st->hist[k] = sqrt(rr1 / st->bb);
        if (sqrt(rr1) <= st->stop)
            st->status = ST_CONVERGED;
        else if (k >= st->kmax)
            st->status = ST_MAXIT;
    }
}

__device__ void finish_residual(DevState *st, const double *partial, int n, bool first, double *ws)
{
    const double rr = sum_partials(partial, n, ws);
    const double bb = first ? sum_partials(partial + n, n, ws) : 0.0;
    if (threadIdx.x == 0) {
        if (first) {
            st->bb = bb;
            if (!isfinite(bb)) {
                st->status = ST_BREAKDOWN;
                return;
            }
            if (bb == 0.0) {
                st->status = ST_ZERO_RHS;
                if (st->hist && st->hist_cap > 0) st->hist[0] = 0.0;
                return;
            }
            st->stop = st->tol * sqrt(bb);
        }
        if (!isfinite(rr)) {
            st->status = ST_BREAKDOWN;
            return;
        }
        st->rr = rr;
        st->beta = 0.0;
        const int k = st->iter;
        if (st->hist && k < st->hist_cap) st->hist[k] = sqrt(rr / st->bb);
        if (sqrt(rr) <= st->stop)
            st->status = ST_CONVERGED;
        else if (k >= st->kmax)
            st->status = ST_MAXIT;
        else
            st->status = ST_RUNNING;
    }
}

// p_k = r_k + beta p_{k-1}, evaluated in FP64 and rounded to the vector type.
template <typename XT>
__device__ __forceinline__ XT pupd(XT r, XT p, double beta)
{
    return (XT)((double)r + beta * (double)p);
}

// ---- local SpMV on the block-diagonal CSR ----------------------------------
//
// One workgroup per row tile (consecutive rows holding at most TN nonzeros,
// or a single longer row).  Stage 1 streams the tile's values and column
// indices with coalesced non-temporal loads (they are read once per
// iteration, the vectors should stay in L2 / MALL) and stores the products
// in LDS; stage 2 gives each row to one thread, which adds its products left
// to right -- the same order as a sequential CSR row sum.

template <typename VT, typename XT, int TN, bool CG, bool FUSED>
__global__ __launch_bounds__(kBS) void k_spmv(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                                              const VT *__restrict__ val, const int32_t *__restrict__ tile_row,
                                              int32_t ntiles, const XT *__restrict__ pin, const XT *__restrict__ r,
                                              XT *__restrict__ pout, XT *__restrict__ q, double *__restrict__ partial,
                                              DevState *__restrict__ st)
{
    __shared__ XT prod[TN];
    __shared__ XT wsx[kBS / 64];
    __shared__ double ws[kBS / 64];
    if (CG && st->status != ST_RUNNING) return;
    const double beta = CG ? st->beta : 0.0;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    double acc = 0.0;
    if (tile < ntiles) {
        const int r0 = tile_row[tile], r1 = tile_row[tile + 1];
        const int k0 = rowptr[r0], k1 = rowptr[r1];
        if (k1 - k0 <= TN) {
            if (k1 > k0) {
                // Every load uses an index clamped into [k0, k1) so that all
                // of them are issued back to back; only the stores are masked.
                constexpr int NI = TN / kBS;
                int jj[NI];
                VT vv[NI];
                XT xx[NI];
#pragma unroll
                for (int i = 0; i < NI; ++i)
                    jj[i] = __builtin_nontemporal_load(colidx + min(k0 + (int)threadIdx.x + i * kBS, k1 - 1));
#pragma unroll
                for (int i = 0; i < NI; ++i)
                    vv[i] = __builtin_nontemporal_load(val + min(k0 + (int)threadIdx.x + i * kBS, k1 - 1));
#pragma unroll
                for (int i = 0; i < NI; ++i) xx[i] = CG ? pupd(r[jj[i]], pin[jj[i]], beta) : pin[jj[i]];
#pragma unroll
                for (int i = 0; i < NI; ++i) {
                    const int k = k0 + (int)threadIdx.x + i * kBS;
                    if (k < k1) prod[k - k0] = (XT)vv[i] * xx[i];
                }
            }
            __syncthreads();
            for (int row = r0 + (int)threadIdx.x; row < r1; row += kBS) {
                const int a = rowptr[row] - k0, e = rowptr[row + 1] - k0;
                XT s = XT(0);
                for (int t = a; t < e; ++t) s = s + prod[t];
                q[row] = s;
                if (CG) {
                    const XT pr = pupd(r[row], pin[row], beta);
                    pout[row] = pr;
                    acc = acc + (double)pr * (double)s;
                }
            }
        } else {
            // a single row longer than a tile: strided partial sums, then a
            // fixed-order workgroup sum
            XT s = XT(0);
            for (int k = k0 + (int)threadIdx.x; k < k1; k += kBS) {
                const int j = colidx[k];
                const XT xj = CG ? pupd(r[j], pin[j], beta) : pin[j];
                s = s + (XT)val[k] * xj;
            }
            s = block_sum(s, wsx);
            if (threadIdx.x == 0) {
                q[r0] = s;
                if (CG) {
                    const XT pr = pupd(r[r0], pin[r0], beta);
                    pout[r0] = pr;
                    acc = (double)pr * (double)s;
                }
            }
        }
    }
    if (CG) {
        const double part = block_sum(acc, ws);
        if (FUSED) {
            const double v[1] = {part};
            if (arrive(v, partial, &st->cnt[0])) finish_alpha(st, partial, gridDim.x, ws);
        } else if (threadIdx.x == 0) {
            partial[blockIdx.x] = part;
        }
    }
}

// ---- interface assembly ------------------------------------------------------

template <typename XT>
__device__ __forceinline__ XT assembled(const XT *__restrict__ q, int g, const int32_t *__restrict__ copy_ptr,
                                        const int32_t *__restrict__ copy_pos)
{
    const int a = copy_ptr[g], e = copy_ptr[g + 1];
    XT t = XT(0);
    for (int u = a; u < e; ++u) t = t + q[copy_pos[u]];
    return t;
}

template <typename XT>
__global__ __launch_bounds__(kBS) void k_iface_sum(int32_t ngamma, const int32_t *__restrict__ copy_ptr,
                                                   const int32_t *__restrict__ copy_pos, XT *__restrict__ q)
{
    const int g = blockIdx.x * kBS + threadIdx.x;
    if (g >= ngamma) return;
    const XT t = assembled(q, g, copy_ptr, copy_pos);
    for (int u = copy_ptr[g]; u < copy_ptr[g + 1]; ++u) q[copy_pos[u]] = t;
}

// ---- fused assembly + x / r update + (r, r) ----------------------------------

template <typename XT, bool FUSED>
__global__ __launch_bounds__(kBS) void k_update(const UpdBlock *__restrict__ blk, int32_t nblk,
                                                const int32_t *__restrict__ pos_grp,
                                                const int32_t *__restrict__ copy_ptr,
                                                const int32_t *__restrict__ copy_pos, XT *__restrict__ x,
                                                const XT *__restrict__ p, XT *__restrict__ r,
                                                const XT *__restrict__ q, double *__restrict__ partial,
                                                DevState *__restrict__ st)
{
    __shared__ double ws[kBS / 64];
    if (st->status != ST_RUNNING) return;
    const int bi = xcd_remap(blockIdx.x, gridDim.x);
    double acc = 0.0;
    if (bi < nblk) {
        const UpdBlock d = blk[bi];
        const double alpha = st->alpha;
        if (d.kind == 0) {
            // interior positions: no assembly; clamped loads, masked stores
            XT xv[kUI], pv[kUI], rv[kUI], qv[kUI];
#pragma unroll
            for (int i = 0; i < kUI; ++i) {
                const int c = d.start + min((int)threadIdx.x + i * kBS, d.count - 1);
                xv[i] = x[c];
                pv[i] = p[c];
                rv[i] = r[c];
                qv[i] = q[c];
            }
#pragma unroll
            for (int i = 0; i < kUI; ++i) {
                const int o = (int)threadIdx.x + i * kBS;
                if (o < d.count) {
                    const int c = d.start + o;
                    x[c] = (XT)((double)xv[i] + alpha * (double)pv[i]);
                    const XT rc = (XT)((double)rv[i] - alpha * (double)qv[i]);
                    r[c] = rc;
                    acc = acc + (double)rc * (double)rc;
                }
            }
        } else {
            for (int i = 0; i < kUI; ++i) {
                const int o = (int)threadIdx.x + i * kBS;
                if (o < d.count) {
                    const int c = d.start + o;
                    const XT qc = assembled(q, pos_grp[d.ifbase + o], copy_ptr, copy_pos);
                    x[c] = (XT)((double)x[c] + alpha * (double)p[c]);
                    const XT rc = (XT)((double)r[c] - alpha * (double)qc);
                    r[c] = rc;
                    if (d.kind != 2) acc = acc + (double)rc * (double)rc;
                }
            }
        }
    }
    const double part = block_sum(acc, ws);
    if (FUSED) {
        const double v[1] = {part};
        if (arrive(v, partial, &st->cnt[1])) finish_beta(st, partial, gridDim.x, ws);
    } else if (threadIdx.x == 0) {
        partial[blockIdx.x] = part;
    }
}

// ---- fresh residual r = b - A x (assembly of q = A_bd x included) -----------

template <typename XT, bool FIRST, bool FUSED>
__global__ __launch_bounds__(kBS) void k_residual(const UpdBlock *__restrict__ blk, int32_t nblk,
                                                  const int32_t *__restrict__ pos_grp,
                                                  const int32_t *__restrict__ copy_ptr,
                                                  const int32_t *__restrict__ copy_pos, const XT *__restrict__ b,
                                                  const XT *__restrict__ q, XT *__restrict__ r, XT *__restrict__ p0,
                                                  double *__restrict__ partial, DevState *__restrict__ st)
{
    __shared__ double ws[kBS / 64];
    const int bi = xcd_remap(blockIdx.x, gridDim.x);
    double arr = 0.0, abb = 0.0;
    if (bi < nblk) {
        const UpdBlock d = blk[bi];
#pragma unroll
        for (int i = 0; i < kUI; ++i) {
            const int o = (int)threadIdx.x + i * kBS;
            if (o < d.count) {
                const int c = d.start + o;
                const XT qc = d.kind == 0 ? q[c] : assembled(q, pos_grp[d.ifbase + o], copy_ptr, copy_pos);
                const XT bc = b[c];
                const XT rc = bc - qc;
                r[c] = rc;
                p0[c] = rc;
                if (d.kind != 2) {
                    arr = arr + (double)rc * (double)rc;
                    if (FIRST) abb = abb + (double)bc * (double)bc;
                }
            }
        }
    }
    const double prr = block_sum(arr, ws);
    const double pbb = FIRST ? block_sum(abb, ws) : 0.0;
    if (FUSED) {
        const double v[2] = {prr, pbb};
        if (arrive(v, partial, &st->cnt[2])) finish_residual(st, partial, gridDim.x, FIRST, ws);
    } else if (threadIdx.x == 0) {
        partial[blockIdx.x] = prr;
        partial[gridDim.x + blockIdx.x] = pbb;
    }
}

// ---- separate finishing kernels (one workgroup) ------------------------------

__global__ __launch_bounds__(kBS) void k_finish_alpha(DevState *st, const double *partial, int n)
{
    __shared__ double ws[kBS / 64];
    if (st->status != ST_RUNNING) return;
    finish_alpha(st, partial, n, ws);
}

__global__ __launch_bounds__(kBS) void k_finish_beta(DevState *st, const double *partial, int n)
{
    __shared__ double ws[kBS / 64];
    if (st->status != ST_RUNNING) return;
    finish_beta(st, partial, n, ws);
}

__global__ __launch_bounds__(kBS) void k_finish_residual(DevState *st, const double *partial, int n, int first)
{
    __shared__ double ws[kBS / 64];
    finish_residual(st, partial, n, first != 0, ws);
}

// ---- gathers, scatters, gradient -------------------------------------------

template <typename XT>
__global__ __launch_bounds__(kBS) void k_gather(int32_t n_loc, const int32_t *__restrict__ l2g,
                                                const double *__restrict__ src, XT *__restrict__ dst)
{
    const int c = blockIdx.x * kBS + threadIdx.x;
    if (c < n_loc) dst[c] = (XT)src[l2g[c]];
}

template <typename XT>
__global__ __launch_bounds__(kBS) void k_scatter(int32_t n, const int32_t *__restrict__ g2own,
                                                 const XT *__restrict__ src, double *__restrict__ dst,
                                                 const DevState *__restrict__ st)
{
    const int i = blockIdx.x * kBS + threadIdx.x;
    if (i >= n) return;
    const bool zero = st && st->status == ST_ZERO_RHS;
    dst[i] = zero ? 0.0 : (double)src[g2own[i]];
}

__global__ __launch_bounds__(kBS) void k_grad_vals(int32_t n_loc, const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ colidx,
                                                   const int32_t *__restrict__ nzmap, const int32_t *__restrict__ l2g,
                                                   const double *__restrict__ lambda, const double *__restrict__ x,
                                                   double *__restrict__ dvals)
{
    const int c = blockIdx.x * kBS + threadIdx.x;
    if (c >= n_loc) return;
    const double li = lambda[l2g[c]];
    for (int e = rowptr[c]; e < rowptr[c + 1]; ++e) dvals[nzmap[e]] = -(li * x[l2g[colidx[e]]]);
}

__global__ __launch_bounds__(kBS) void k_set_values(int64_t nnz, const int32_t *__restrict__ nzmap,
                                                    const double *__restrict__ src, double *__restrict__ v64,
                                                    float *__restrict__ v32)
{
    const int64_t e = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (e >= nnz) return;
    const double v = src[nzmap[e]];
    v64[e] = v;
    if (v32) v32[e] = (float)v;
}

inline int nblocks(int64_t n) { return (int)((n + kBS - 1) / kBS); }

}  // namespace

// ---- launchers -----------------------------------------------------------------

template <typename XT>
void launch_gather(hipStream_t s, int32_t n_loc, const int32_t *l2g, const double *src, XT *dst)
{
    if (n_loc > 0) hipLaunchKernelGGL(k_gather<XT>, dim3(nblocks(n_loc)), dim3(kBS), 0, s, n_loc, l2g, src, dst);
}

template <typename XT>
void launch_scatter(hipStream_t s, int32_t n, const int32_t *g2own, const XT *src, double *dst, const DevState *st)
{
    if (n > 0) hipLaunchKernelGGL(k_scatter<XT>, dim3(nblocks(n)), dim3(kBS), 0, s, n, g2own, src, dst, st);
}

template <typename VT, typename XT, int TN, bool CG, bool FUSED>
static void spmv_tn(hipStream_t s, const Csr &A, const XT *pin, const XT *r, XT *pout, XT *q, double *partial,
                    DevState *st)
{
    hipLaunchKernelGGL((k_spmv<VT, XT, TN, CG, FUSED>), dim3(xcd_grid(A.ntiles)), dim3(kBS), 0, s, A.rowptr, A.colidx,
                       (const VT *)A.val, A.tile_row, A.ntiles, pin, r, pout, q, partial, st);
}

template <typename VT, typename XT, bool CG, bool FUSED>
static void spmv_dispatch(hipStream_t s, const Csr &A, const XT *pin, const XT *r, XT *pout, XT *q, double *partial,
                          DevState *st)
{
    if (A.ntiles == 0) return;
    switch (A.tile_nnz) {
    case 1024: spmv_tn<VT, XT, 1024, CG, FUSED>(s, A, pin, r, pout, q, partial, st); break;
    case 4096: spmv_tn<VT, XT, 4096, CG, FUSED>(s, A, pin, r, pout, q, partial, st); break;
    default: spmv_tn<VT, XT, 2048, CG, FUSED>(s, A, pin, r, pout, q, partial, st); break;
    }
}

template <typename VT, typename XT>
void launch_spmv(hipStream_t s, const Csr &A, const XT *x, XT *q)
{
    spmv_dispatch<VT, XT, false, false>(s, A, x, nullptr, nullptr, q, nullptr, nullptr);
}

template <typename VT, typename XT>
void launch_spmv_cg(hipStream_t s, const Csr &A, const XT *pin, const XT *r, XT *pout, XT *q, double *partial,
                    DevState *st, bool fused)
{
    if (fused) {
        spmv_dispatch<VT, XT, true, true>(s, A, pin, r, pout, q, partial, st);
    } else {
        spmv_dispatch<VT, XT, true, false>(s, A, pin, r, pout, q, partial, st);
        hipLaunchKernelGGL(k_finish_alpha, dim3(1), dim3(kBS), 0, s, st, partial, xcd_grid(A.ntiles));
    }
}

template <typename XT>
void launch_iface_sum(hipStream_t s, const Iface &I, XT *q)
{
    if (I.ngamma > 0)
        hipLaunchKernelGGL(k_iface_sum<XT>, dim3(nblocks(I.ngamma)), dim3(kBS), 0, s, I.ngamma, I.copy_ptr,
                           I.copy_pos, q);
}

template <typename XT>
void launch_update(hipStream_t s, const Iface &I, XT *x, const XT *p, XT *r, const XT *q, double *partial,
                   DevState *st, bool fused)
{
    const int grid = xcd_grid(I.nblk);
    if (fused) {
        hipLaunchKernelGGL((k_update<XT, true>), dim3(grid), dim3(kBS), 0, s, I.blk, I.nblk, I.pos_grp, I.copy_ptr,
                           I.copy_pos, x, p, r, q, partial, st);
    } else {
        hipLaunchKernelGGL((k_update<XT, false>), dim3(grid), dim3(kBS), 0, s, I.blk, I.nblk, I.pos_grp, I.copy_ptr,
                           I.copy_pos, x, p, r, q, partial, st);
        hipLaunchKernelGGL(k_finish_beta, dim3(1), dim3(kBS), 0, s, st, partial, grid);
    }
}

template <typename XT>
void launch_residual(hipStream_t s, const Iface &I, const XT *b, const XT *q, XT *r, XT *p0, double *partial,
                     DevState *st, bool first, bool fused)
{
    const int grid = xcd_grid(I.nblk);
#define SS_RES(F, U)                                                                                              \
    hipLaunchKernelGGL((k_residual<XT, F, U>), dim3(grid), dim3(kBS), 0, s, I.blk, I.nblk, I.pos_grp, I.copy_ptr, \
                       I.copy_pos, b, q, r, p0, partial, st)
    if (fused) {
        if (first) SS_RES(true, true);
        else SS_RES(false, true);
    } else {
        if (first) SS_RES(true, false);
        else SS_RES(false, false);
        hipLaunchKernelGGL(k_finish_residual, dim3(1), dim3(kBS), 0, s, st, partial, grid, first ? 1 : 0);
    }
#undef SS_RES
}

void launch_grad_vals(hipStream_t s, int32_t n_loc, const int32_t *rowptr, const int32_t *colidx, const int32_t *nzmap,
                      const int32_t *l2g, const double *lambda, const double *x, double *dvals)
{
    if (n_loc > 0)
        hipLaunchKernelGGL(k_grad_vals, dim3(nblocks(n_loc)), dim3(kBS), 0, s, n_loc, rowptr, colidx, nzmap, l2g,
                           lambda, x, dvals);
}

void launch_set_values(hipStream_t s, int64_t nnz, const int32_t *nzmap, const double *val_glob, double *val64,
                       float *val32)
{
    if (nnz > 0)
        hipLaunchKernelGGL(k_set_values, dim3(nblocks(nnz)), dim3(kBS), 0, s, nnz, nzmap, val_glob, val64, val32);
}

// explicit instantiations
template void launch_gather<double>(hipStream_t, int32_t, const int32_t *, const double *, double *);
template void launch_gather<float>(hipStream_t, int32_t, const int32_t *, const double *, float *);
template void launch_scatter<double>(hipStream_t, int32_t, const int32_t *, const double *, double *, const DevState *);
template void launch_scatter<float>(hipStream_t, int32_t, const int32_t *, const float *, double *, const DevState *);
template void launch_spmv<double, double>(hipStream_t, const Csr &, const double *, double *);
template void launch_spmv<float, float>(hipStream_t, const Csr &, const float *, float *);
template void launch_spmv_cg<double, double>(hipStream_t, const Csr &, const double *, const double *, double *,
                                             double *, double *, DevState *, bool);
template void launch_spmv_cg<float, float>(hipStream_t, const Csr &, const float *, const float *, float *, float *,
                                           double *, DevState *, bool);
template void launch_iface_sum<double>(hipStream_t, const Iface &, double *);
template void launch_iface_sum<float>(hipStream_t, const Iface &, float *);
template void launch_update<double>(hipStream_t, const Iface &, double *, const double *, double *, const double *,
                                    double *, DevState *, bool);
template void launch_update<float>(hipStream_t, const Iface &, float *, const float *, float *, const float *,
                                   double *, DevState *, bool);
template void launch_residual<double>(hipStream_t, const Iface &, const double *, const double *, double *, double *,
                                      double *, DevState *, bool, bool);
template void launch_residual<float>(hipStream_t, const Iface &, const float *, const float *, float *, float *,
                                     double *, DevState *, bool, bool);

}  // namespace ss
