// The whole CG solve of a small system in one launch of one workgroup.
//
// For a few thousand unknowns (the 64 x 64 Poisson system of the paper's
// smallest class) an iteration moves well under a megabyte, and the two
// launches per iteration of the streaming kernels cost more than their work.
// Here one workgroup of 768 threads (three waves per SIMD, up to 168
// registers a thread; 512 threads with more rows each measured 1.22 against
// 0.98 ms on the 64 x 64 system) runs Algorithm 3 (M = I) from the first
// residual to the converged, recomputed one:
//   - every thread owns up to R rows of the block-diagonal matrix of all
//     sub-domains (rows t, t + 768, ...), whose values and column positions
//     stay in its registers for the whole solve;
//   - x and p live in LDS (up to 160 KB a workgroup on gfx950; the local
//     products gather p there), r in the registers of the thread whose rows
//     they are (only that thread reads or writes them: 0.97 -> 0.91 ms on
//     the 64 x 64 system);
//   - the interface positions publish their unassembled product in LDS too
//     (their copy lists are copied there at the start), and every copy
//     of an interface node adds all copies in ascending sub-domain order
//     (Algorithms 4 and 5 on one address space);
//   - (p, A p) is the unassembled sum over all local rows, (r, r) the sum
//     over the owned positions (the 0/1 weights of Section 4.4.2), each a
//     fixed-order workgroup sum;
//   - the stopping rule, the residual recomputation at convergence with the
//     restart it may trigger, the iteration limit and the breakdown tests are
//     those of the streaming path; the scalars go to the run's DevState.
// Row sums are formed in stored column order with separately rounded
// products and sums, so the products are bitwise those of the other kernels.
#include "small.h"

#include "device_common.h"

#include <cmath>
#include <cstdint>

namespace ss {
namespace {

constexpr int kSW = kSmallThreads / 64;  // waves of the workgroup
constexpr int kHistRing = 256;           // residual history entries staged in LDS

// A lane's value from another lane by a DPP move (CTRL, rows ROW_MASK); lanes
// without a source, or outside the rows, get +0.  Both halves of the double
// move the same way.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 64 lanes of a wave in a fixed order, the total in lane 63:
// lanes pair up (quad_perm 1,0,3,2), then pairs (2,3,0,1), then each 16-lane
// row shifts by 4 and by 8, lane 15 of each row feeds the next row and lane 31
// the upper half (row_bcast 15 and 31, gfx9 DPP).  Register moves instead of
// LDS permutes.
__device__ __forceinline__ double wave_sum_last(double v)
{
    v = v + dpp_f64<0xb1, 0xf>(v);   // quad_perm: 1, 0, 3, 2
    v = v + dpp_f64<0x4e, 0xf>(v);   // quad_perm: 2, 3, 0, 1
    v = v + dpp_f64<0x114, 0xf>(v);  // row_shr: 4
    v = v + dpp_f64<0x118, 0xf>(v);  // row_shr: 8
    v = v + dpp_f64<0x142, 0xa>(v);  // row_bcast: 15 into rows 1 and 3
    v = v + dpp_f64<0x143, 0xc>(v);  // row_bcast: 31 into rows 2 and 3
    return v;
}

// Fixed-order workgroup sum, every thread gets the total.  Two alternating
// slot sets: a set is rewritten two sums later, after a barrier that every
// reader of its previous values has passed.
__device__ __forceinline__ double small_sum(double v, double *ws, int &set)
{
    v = wave_sum_last(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double *slot = ws + set * kSW;
    if (lane == 63) slot[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kSW; ++i) t = t + slot[i];
    set ^= 1;
    return t;
}

template <int R, int U>
__global__ __launch_bounds__(kSmallThreads) void k_cg_small(int32_t n_loc, int32_t n_own, int32_t n_if,
                                                            int32_t ngamma, int32_t n_copies,
                                                            const double *__restrict__ sval,
                                                            const uint32_t *__restrict__ scol,
                                                            const int32_t *__restrict__ pos_grp,
                                                            const int32_t *__restrict__ copy_ptr,
                                                            const int32_t *__restrict__ copy_pos,
                                                            const double *__restrict__ b, double *__restrict__ x,
                                                            DevState *__restrict__ st)
{
    constexpr int UW = (U + 1) / 2;  // column words per row: two 16-bit positions each
    extern __shared__ double smem[];
    double *pl = smem;              // p (or x while a residual is formed), n_loc
    double *xl = pl + n_loc;        // x, n_loc
    double *qif = xl + n_loc;       // unassembled products of the interface positions, n_if
    double *ws = qif + n_if;        // 2 * kSW sum slots
    double *hring = ws + 2 * kSW;   // kHistRing residual history entries
    // the interface copy lists, read from LDS inside the iterations
    int32_t *grp_l = reinterpret_cast<int32_t *>(hring + kHistRing);  // pos_grp, n_if
    int32_t *cptr_l = grp_l + n_if;                                // copy_ptr, ngamma + 1
    int32_t *cpos_l = cptr_l + ngamma + 1;                         // copy_pos, n_copies
    const int t = threadIdx.x;
    int set = 0;
    for (int i = t; i < n_if; i += kSmallThreads) grp_l[i] = pos_grp[i];
    for (int i = t; i <= ngamma; i += kSmallThreads) cptr_l[i] = copy_ptr[i];
    for (int i = t; i < n_copies; i += kSmallThreads) cpos_l[i] = copy_pos[i];

    double val[R][U];
    uint32_t cw[R][UW];
    double rr_[R];  // r of the thread's own rows (row t + k kSmallThreads)
#pragma unroll
    for (int k = 0; k < R; ++k) rr_[k] = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = t + k * kSmallThreads;
        const bool in = i < n_loc;
#pragma unroll
        for (int u = 0; u < U; ++u) val[k][u] = in ? sval[(size_t)u * n_loc + i] : 0.0;
#pragma unroll
        for (int w = 0; w < UW; ++w) cw[k][w] = in ? scol[(size_t)w * n_loc + i] : 0u;
        if (in) xl[i] = x[i];
    }

    // q = A_bd v for own row k (v in pl); the row length rides in the free
    // upper half of the last column word (U odd)
    auto rowsum = [&](int k) -> double {
        const int len = (int)(cw[k][UW - 1] >> 16);
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = (int)((cw[k][u >> 1] >> (16 * (u & 1))) & 0xffffu);
            if (u < len) s = s + val[k][u] * pl[c];
        }
        return s;
    };
    auto assembled = [&](int i) -> double {
        const int g = grp_l[i];
        double s = 0.0;
        for (int e = cptr_l[g]; e < cptr_l[g + 1]; ++e) s = s + qif[cpos_l[e]];
        return s;
    };

    const double tol = st->tol;
    const int kmax = st->kmax;
    double *hist = st->hist;
    const int hcap = st->hist_cap;
    // The residual history goes to a ring in LDS and reaches memory in blocks
    // written by wave 0: a global store inside the loop would make every
    // barrier wait for it.  Entries [flushed, k] are in the ring (k - flushed
    // < kHistRing); every thread tracks `flushed` the same way.
    int flushed = 0, last = -1;  // last: the highest entry recorded
    auto flush = [&](int upto) {  // entries [flushed, upto) to memory
        if (hist && (threadIdx.x >> 6) == 0)
            for (int j = flushed + (int)(threadIdx.x & 63); j < upto && j < hcap; j += 64)
                hist[j] = hring[j & (kHistRing - 1)];
        flushed = upto;
    };
    auto record = [&](int k, double v) {
        if (k - flushed >= kHistRing) flush(k);
        if (threadIdx.x == 0) hring[k & (kHistRing - 1)] = v;
        last = k;
    };
    int k_it = 0, restarts = -1, status = ST_RUNNING;
    double bb = 0.0, stop = 0.0, rr = 0.0;

    for (bool first = true; status == ST_RUNNING; first = false) {
        // ---- r = b - A x, p = r (the first residual, and every recomputation)
        ++restarts;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = t + k * kSmallThreads;
            if (i < n_loc) pl[i] = xl[i];
        }
        __syncthreads();
        double q[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = t + k * kSmallThreads;
            q[k] = i < n_loc ? rowsum(k) : 0.0;
            if (i < n_if) qif[i] = q[k];
        }
        double arr = 0.0, abb = 0.0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = t + k * kSmallThreads;
            if (i < n_loc) {
                const double qa = i < n_if ? assembled(i) : q[k];
                const double bi = b[i];
                const double ri = bi - qa;
                rr_[k] = ri;
                if (i < n_own || i >= n_if) {
                    arr = arr + ri * ri;
                    abb = abb + bi * bi;
                }
            }
        }
        rr = small_sum(arr, ws, set);
        if (first) {
            bb = small_sum(abb, ws, set);
            if (!isfinite(bb)) {
                status = ST_BREAKDOWN;
                break;
            }
            if (bb == 0.0) {
                record(0, 0.0);
                status = ST_ZERO_RHS;
                break;
            }
            stop = tol * sqrt(bb);
        }
        if (!isfinite(rr)) {
            status = ST_BREAKDOWN;
            break;
        }
        record(k_it, sqrt(rr / bb));
        if (sqrt(rr) <= stop) {
            status = ST_CONVERGED;
            break;
        }
        if (k_it >= kmax) {
            status = ST_MAXIT;
            break;
        }
        // every read of pl (x) happened before the sums' barriers
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int i = t + k * kSmallThreads;
            if (i < n_loc) pl[i] = rr_[k];
        }
        __syncthreads();

        // ---- CG iterations until the recurrence meets the tolerance
        for (;;) {
            double apq = 0.0;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int i = t + k * kSmallThreads;
                q[k] = i < n_loc ? rowsum(k) : 0.0;
                if (i < n_if) qif[i] = q[k];
                if (i < n_loc) apq = apq + pl[i] * q[k];
            }
            const double pAp = small_sum(apq, ws, set);  // its barrier also publishes qif
            if (!(pAp > 0.0) || !isfinite(pAp)) {
                status = ST_BREAKDOWN;
                break;
            }
            const double alpha = rr / pAp;
            double arn = 0.0;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int i = t + k * kSmallThreads;
                if (i < n_loc) {
                    const double qa = i < n_if ? assembled(i) : q[k];
                    xl[i] = xl[i] + alpha * pl[i];
                    const double ri = rr_[k] - alpha * qa;
                    rr_[k] = ri;
                    if (i < n_own || i >= n_if) arn = arn + ri * ri;
                }
            }
            const double rr_new = small_sum(arn, ws, set);
            if (!isfinite(rr_new)) {  // as the streaming path: the step is not counted
                status = ST_BREAKDOWN;
                break;
            }
            ++k_it;
            record(k_it, sqrt(rr_new / bb));
            const double beta = rr_new / rr;
            rr = rr_new;
            if (sqrt(rr_new) <= stop) break;  // recompute the residual, restart if needed
            if (k_it >= kmax) {
                status = ST_MAXIT;
                break;
            }
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int i = t + k * kSmallThreads;
                if (i < n_loc) pl[i] = rr_[k] + beta * pl[i];
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int i = t + k * kSmallThreads;
        if (i < n_loc) x[i] = xl[i];
    }
    flush(last + 1);  // the recorded entries not yet in memory
    if (t == 0) {
        st->bb = bb;
        st->stop = stop;
        st->rr_last = rr;
        st->iter_last = k_it;
        st->restarts = restarts;
        dev::flag_store(&st->status, status);
    }
}

template <int R, int U>
void launch_r(hipStream_t s, const SmallMat &M, const Iface &I, const double *b, double *x, DevState *st)
{
    const size_t lds = small_lds_bytes(M.n_loc, I.n_if, I.ngamma, M.n_copies);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_cg_small<R, U>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k_cg_small<R, U>), dim3(1), dim3(kSmallThreads), lds, s, M.n_loc, I.n_own, I.n_if,
                       I.ngamma, M.n_copies, M.val, M.colw, I.pos_grp, I.copy_ptr, I.copy_pos, b, x, st);
}

}  // namespace

int32_t small_rows(int32_t rows_needed, int32_t width)
{
    const int32_t cap = width == 5 ? 6 : width == 7 ? 5 : 0;
    return rows_needed >= 1 && rows_needed <= cap ? rows_needed : 0;
}

void launch_cg_small(hipStream_t s, const SmallMat &M, const Iface &I, const double *b, double *x, DevState *st)
{
    if (M.width == 5) {
        switch (M.rows) {
        case 1: launch_r<1, 5>(s, M, I, b, x, st); break;
        case 2: launch_r<2, 5>(s, M, I, b, x, st); break;
        case 3: launch_r<3, 5>(s, M, I, b, x, st); break;
        case 4: launch_r<4, 5>(s, M, I, b, x, st); break;
        case 5: launch_r<5, 5>(s, M, I, b, x, st); break;
        case 6: launch_r<6, 5>(s, M, I, b, x, st); break;
        default: break;
        }
    } else if (M.width == 7) {
        switch (M.rows) {
        case 1: launch_r<1, 7>(s, M, I, b, x, st); break;
        case 2: launch_r<2, 7>(s, M, I, b, x, st); break;
        case 3: launch_r<3, 7>(s, M, I, b, x, st); break;
        case 4: launch_r<4, 7>(s, M, I, b, x, st); break;
        case 5: launch_r<5, 7>(s, M, I, b, x, st); break;
        default: break;
        }
    }
}

}  // namespace ss
