// HIP kernels of the sub-structured CG for gfx950 (MI355X).
//
// One CG iteration (Algorithm 3, M = I) with every sub-domain resident on the
// device is two launches (the SpMV on a persistent, fixed-size grid):
//   k_update: finishes (p, A p) -> alpha, assembles the interface values of
//             q = A_bd p (Algorithms 4 and 5: every copy of an interface node
//             reads all copies and adds them in ascending sub-domain order),
//             r -= alpha q, and writes partials of the weighted local (r, r)
//             (Section 4.4.2);
//   k_spmv_*: finishes (r, r) -> beta and the stopping test, applies the
//             previous update's x += alpha p to its own rows, forms
//             p = r + beta p on the fly, runs the local SpMV of every
//             sub-domain on the block-diagonal matrix (Section 4.4.1, first
//             step) and writes partials of (p, A_s p).
// The SELL kernel also computes the band-column product of the band
// splitting (Section 4.3.1) when instantiated with BAND.
// "Finishes" means: every workgroup adds up the previous kernel's
// per-workgroup partials itself, in one fixed order, so all workgroups obtain
// bitwise the same scalar without a grid-wide barrier or a separate launch;
// those loads go out with the workgroup's first operand loads, the status
// word and the state's scalars, behind one wait.  Workgroup 0 records the
// scalars.  All sums are fixed-order,
// hence bitwise reproducible run to run.  Compiled with -ffp-contract=off:
// products and sums are rounded separately, as the expressions are written.
#include "kernels.h"

#include "device_common.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <type_traits>

namespace ss {
namespace {

using dev::block_sum_all;
using dev::wave_sum;
using dev::xcd_remap;

__device__ __forceinline__ int32_t load_status(const DevState *st) { return dev::flag_load(&st->status); }

__device__ __forceinline__ void store_status(DevState *st, int32_t v) { dev::flag_store(&st->status, v); }

// Status read once per workgroup and shared, so the whole workgroup takes the
// same branch.
__device__ __forceinline__ bool running(const DevState *st, int *s_flag)
{
    if (threadIdx.x == 0) *s_flag = load_status(st);
    __syncthreads();
    return *s_flag == ST_RUNNING;
}

// Sum of n partials in a fixed order (thread t adds partials t, t+kBS, ...
// left to right, then the workgroup tree), returned to every thread.  Loads
// go out 8 at a time before the adds.
__device__ __forceinline__ double sum_partials_all(const double *__restrict__ partial, int n, double *ws)
{
    double v = 0.0;
    for (int base = 0; base < n; base += 8 * kBS) {
        double t[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int idx = base + i * kBS + (int)threadIdx.x;
            t[i] = idx < n ? partial[idx] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) v = v + t[i];
    }
    return block_sum_all(v, ws);
}

// Sum of n partials at a 16-byte aligned address, 16 values per thread in
// flight per round: thread t adds the pairs t, t + kBS, ... (each pair's two
// values in order), thread 0 the odd last value, then the workgroup tree.
// A fixed order, so every workgroup obtains the same bits.
__device__ __forceinline__ double sum_partials_vec(const double *__restrict__ partial, int n)
{
    const double2 *p2 = reinterpret_cast<const double2 *>(partial);
    const int npair = n >> 1;
    double v = 0.0;
    for (int base = 0; base < npair; base += 8 * kBS) {
        double2 t[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int idx = base + i * kBS + (int)threadIdx.x;
            t[i] = idx < npair ? p2[idx] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            v = v + t[i].x;
            v = v + t[i].y;
        }
    }
    if ((n & 1) && threadIdx.x == 0) v = v + partial[n - 1];
    return v;
}

// The first round of sum_partials_vec loaded ahead, so that these loads go
// out with a kernel's first operand loads and share their wait: pairs t,
// t + kBS, ..., t + (R-1) kBS of thread t.  The loads are unconditional (past
// the end they repeat the last pair; with a single partial there is no pair
// to load) and the pairs past the end are dropped where they are added, so
// that no use sits next to a load.
template <int R>
__device__ __forceinline__ void pre_pairs(double2 (&t)[R], const double *__restrict__ partial, int n)
{
    const double2 *p2 = reinterpret_cast<const double2 *>(partial);
    const int npair = n >> 1;
    if (npair == 0) {
#pragma unroll
        for (int i = 0; i < R; ++i) t[i] = make_double2(0.0, 0.0);
        return;
    }
#pragma unroll
    for (int i = 0; i < R; ++i) t[i] = p2[min(i * kBS + (int)threadIdx.x, npair - 1)];
}

// sum_partials_vec from a preloaded first round: thread t still adds its
// pairs t, t + kBS, ... in turn (+0 past the end changes nothing), so the
// bits are the same.
template <int R>
__device__ __forceinline__ double sum_pre(const double2 (&t)[R], const double *__restrict__ partial, int n)
{
    const double2 *p2 = reinterpret_cast<const double2 *>(partial);
    const int npair = n >> 1;
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const bool in = i * kBS + (int)threadIdx.x < npair;
        v = v + (in ? t[i].x : 0.0);
        v = v + (in ? t[i].y : 0.0);
    }
    for (int base = R * kBS; base < npair; base += 8 * kBS) {
        double2 u[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int idx = base + i * kBS + (int)threadIdx.x;
            u[i] = idx < npair ? p2[idx] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            v = v + u[i].x;
            v = v + u[i].y;
        }
    }
    if ((n & 1) && threadIdx.x == 0) v = v + partial[n - 1];
    return v;
}

// Two fixed-order workgroup sums in one pass (each with exactly the order of
// block_sum_all).  ws: 2 * (kBS/64) + 2 slots.
__device__ __forceinline__ void block_sum2_all(double &a, double &b, double *ws)
{
    constexpr int W = kBS / 64;
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        ws[w] = a;
        ws[W + w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            ta = ta + ws[i];
            tb = tb + ws[W + i];
        }
        ws[2 * W] = ta;
        ws[2 * W + 1] = tb;
    }
    __syncthreads();
    a = ws[2 * W];
    b = ws[2 * W + 1];
    __syncthreads();
}

// p_k = r_k + beta p_{k-1}, evaluated in FP64 and rounded to the vector type.
template <typename XT>
__device__ __forceinline__ XT pupd(XT r, XT p, double beta)
{
    return (XT)((double)r + beta * (double)p);
}

// Element i of an array whose base is wave-uniform, through a 32-bit byte
// offset: the base stays in scalar registers and a lane needs one VGPR for
// the offset (arrays of at most 4 GiB: SELL storage is built for fewer than
// 2^29 positions).
template <typename T>
__device__ __forceinline__ T ld32(const T *__restrict__ base, uint32_t i)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + i * (uint32_t)sizeof(T));
}

template <typename T>
__device__ __forceinline__ void st32(T *__restrict__ base, uint32_t i, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + i * (uint32_t)sizeof(T)) = v;
}

// PLAIN: q = A x.  FIRST / STEP: p = r + beta p formed on the fly at every
// gathered column (beta = 0 for FIRST), q = A p, (p, A p) partials; STEP also
// finishes (r, r) and applies the previous x update.  PQ: q = A p for a p
// already formed (k_pstep), (p, A p) partials.
enum { SPMV_PLAIN = 0, SPMV_FIRST = 1, SPMV_STEP = 2, SPMV_PQ = 3 };

// Pairs of partials per thread loaded ahead: of the update partials by the
// CG-step SpMV (one per kUI * kBS positions: one round up to ~3M positions)
// and by k_pstep (a streaming kernel that keeps its registers for occupancy,
// 8 waves per SIMD: ~1M positions, and (r, z) not ahead), of the SpMV
// partials by the update (one per SpMV workgroup: up to 2048).
constexpr int kPreRound = 12;
constexpr int kPreRoundS = 4;
constexpr int kPreRoundA = 4;

// The state a CG step reads before its stopping test, loaded with the
// step's first operands (no kernel of the step writes these fields).
struct StepIn {
    double rz;    // (r, z) of the slot
    double stop;  // threshold on ||r||
    int32_t iter, kmax;
};

__device__ __forceinline__ StepIn load_step_in(const DevState *st, int slot)
{
    return StepIn{st->rz[slot], st->stop, st->iter[slot], st->kmax};
}

// The CG-step prologue: from the finished (r, r) [and (r, z)] of the
// previous update, record iteration k+1 (workgroup 0) and take the stopping
// test on ||r||.  Returns beta = (r, z)_new / (r, z), or sets *stop.
__device__ __forceinline__ double step_test(double rr_new, double rz_new, StepIn in, int slot, DevState *st,
                                            bool *stop_out)
{
    const double rz_cur = in.rz;
    const int k_new = in.iter + 1;
    int stop = ST_RUNNING;
    if (!isfinite(rr_new) || !isfinite(rz_new))
        stop = ST_BREAKDOWN;
    else if (sqrt(rr_new) <= in.stop)
        stop = ST_CONVERGED;
    else if (k_new >= in.kmax)
        stop = ST_MAXIT;
    const double beta = rz_new / rz_cur;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (stop != ST_BREAKDOWN) {
            st->rr[slot ^ 1] = rr_new;
            st->rz[slot ^ 1] = rz_new;
            st->iter[slot ^ 1] = k_new;
            st->rr_last = rr_new;
            st->iter_last = k_new;
            st->beta = beta;
            if (st->hist && k_new < st->hist_cap) st->hist[k_new] = sqrt(rr_new / st->bb);
        }
        if (stop != ST_RUNNING) store_status(st, stop);
    }
    *stop_out = stop != ST_RUNNING;
    return beta;
}

// finish (r, r) [and (r, z)] from the update partials, then step_test.
// part_b2 = nullptr: no preconditioner, (r, z) = (r, r).
__device__ __forceinline__ double finish_rr(const double *__restrict__ part_b, const double *__restrict__ part_b2,
                                            int nb, int slot, DevState *st, double *ws, bool *stop_out)
{
    double rr_new, rz_new;
    if (part_b2) {
        rr_new = sum_partials_vec(part_b, nb);
        rz_new = sum_partials_vec(part_b2, nb);
        block_sum2_all(rr_new, rz_new, ws);
    } else {
        rr_new = block_sum_all(sum_partials_vec(part_b, nb), ws);
        rz_new = rr_new;
    }
    return step_test(rr_new, rz_new, load_step_in(st, slot), slot, st, stop_out);
}

// The same from preloaded first rounds of the partials and state.
template <int R>
__device__ __forceinline__ double finish_rr_pre(const double2 (&tb)[R], const double2 (&tb2)[R],
                                                const double *__restrict__ part_b,
                                                const double *__restrict__ part_b2, int nb, StepIn in, int slot,
                                                DevState *st, double *ws, bool *stop_out)
{
    double rr_new, rz_new;
    if (part_b2) {
        rr_new = sum_pre<R>(tb, part_b, nb);
        rz_new = sum_pre<R>(tb2, part_b2, nb);
        block_sum2_all(rr_new, rz_new, ws);
    } else {
        rr_new = block_sum_all(sum_pre<R>(tb, part_b, nb), ws);
        rz_new = rr_new;
    }
    return step_test(rr_new, rz_new, in, slot, st, stop_out);
}

// ---- local SpMV, SELL-64 -----------------------------------------------------
//
// A wave owns chunks of 64 rows, one row per lane.  Entry j of the 64 rows is
// stored contiguously, so the value / column loads are coalesced and, for
// matrices whose rows of a chunk have similar column offsets (grid
// numberings), so are the x gathers.  Each lane adds its row's products left
// to right in stored (column) order -- the order of a sequential CSR row sum.
// Workgroup w (after the XCD remap) owns the stored chunks [w*cpb, (w+1)*cpb)
// (cpos maps them to row positions); its 4 waves take every 4th chunk.

// Column position of a 16-bit entry: bit 15 selects the window base.
__device__ __forceinline__ int narrow_col(uint32_t v, int2 base) { return ((v & 0x8000u) ? base.y : base.x) + (int)(v & 0x7fffu); }

// Length of chunk c (wave-uniform), read as the 32-bit word holding its
// byte so that it comes through the scalar path (the length array is padded
// to whole words).
__device__ __forceinline__ int chunk_len(const uint8_t *__restrict__ clen, int c)
{
    const uint32_t wd = reinterpret_cast<const uint32_t *>(clen)[c >> 2];
    return (int)((wd >> (8 * (c & 3))) & 0xffu);
}

// The loads of a chunk's batch (see k_spmv_sell), addressed from the
// chunk's wave-uniform bases: its values cv, its first row pos.
//
// The column words of slots j0..j0+U-1, the last slot repeated past L; decoded
// at use (decode_cols), so that the loads can stay in flight across other
// work.  One 32-bit load per entry for either kind of chunk: a wide chunk's
// int32 position, or the aligned word holding the 16-bit offsets of lanes 2l
// and 2l+1 of a narrow chunk (every chunk's offsets start at an even index,
// chunks being 64 entries a slot).
template <int U>
__device__ __forceinline__ void load_cwords(uint32_t (&cw)[U], int cb, int j0, int L, int lane,
                                            const int32_t *__restrict__ col, const uint16_t *__restrict__ col16)
{
    const bool narrow = cb >= 0;
    const uint32_t *w32 = narrow ? reinterpret_cast<const uint32_t *>(col16 + cb)
                                 : reinterpret_cast<const uint32_t *>(col + ~cb);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int off = max(min(j0 + u, L - 1), 0) * 64 + lane;
        cw[u] = ld32(w32, (uint32_t)(narrow ? off >> 1 : off));
    }
}

// The values of slots 0..U-1, the last slot repeated past L.
template <typename VT, int U>
__device__ __forceinline__ void load_vals(VT (&vv)[U], const VT *__restrict__ cv, int L, int lane)
{
#pragma unroll
    for (int u = 0; u < U; ++u) vv[u] = ld32(cv, (uint32_t)(max(min(u, L - 1), 0) * 64 + lane));
}

// A row's own length and operands (r, p_{k-1}, x), at a clamped position
// for the lanes past the last row.
template <typename XT, int MODE>
__device__ __forceinline__ void load_row(int &len, XT &rv, XT &pv, XT &xv, int pos, int lane, int nrows,
                                         const uint8_t *__restrict__ rlen, const XT *__restrict__ r,
                                         const XT *__restrict__ p, const XT *__restrict__ x)
{
    const uint32_t t = (uint32_t)min(lane, nrows - 1 - pos);
    const int l = ld32(rlen + pos, t);
    len = pos + lane < nrows ? l : 0;
    rv = pv = xv = XT(0);
    if (MODE == SPMV_FIRST || MODE == SPMV_STEP) rv = ld32(r + pos, t);
    if (MODE != SPMV_PLAIN) pv = ld32(p + pos, t);
    if (MODE == SPMV_STEP) xv = ld32(x + pos, t);
}

// load_row for a dictionary chunk of at most 7 slots: the length comes with
// the lane's index word (and every row of the chunk exists).
template <typename XT, int MODE>
__device__ __forceinline__ void load_row_nolen(XT &rv, XT &pv, XT &xv, int pos, int lane, const XT *__restrict__ r,
                                               const XT *__restrict__ p, const XT *__restrict__ x)
{
    rv = pv = xv = XT(0);
    if (MODE == SPMV_FIRST || MODE == SPMV_STEP) rv = ld32(r + pos, (uint32_t)lane);
    if (MODE != SPMV_PLAIN) pv = ld32(p + pos, (uint32_t)lane);
    if (MODE == SPMV_STEP) xv = ld32(x + pos, (uint32_t)lane);
}

template <int U>
__device__ __forceinline__ void decode_cols(int (&cc)[U], const uint32_t (&cw)[U], int cb, int2 base, int lane)
{
    // select by mask rather than by a branch of the wave
    const uint32_t m = cb >= 0 ? 0xffffffffu : 0u;
    const int sh = (lane & 1) * 16;
#pragma unroll
    for (int u = 0; u < U; ++u)
        cc[u] = (int)(((uint32_t)narrow_col((cw[u] >> sh) & 0xffffu, base) & m) | (cw[u] & ~m));
}

// A dictionary chunk's lane word of offset indices and the lane's entry
// (lane & 15) of the chunk's 16 offsets.
__device__ __forceinline__ void load_dict(uint32_t &dw, int &tab, int blk, int lane,
                                          const int32_t *__restrict__ dtab, const uint32_t *__restrict__ dword)
{
    dw = ld32(dword + blk * 64, (uint32_t)lane);
    tab = ld32(dtab + blk * 16, (uint32_t)(lane & 15));
}

// Columns of a dictionary chunk's slots 0..U-1: the row plus the offset its
// 4-bit index names, fetched from the lane holding it.
template <int U>
__device__ __forceinline__ void decode_dict(int (&cc)[U], uint32_t dw, int tab, int row)
{
#pragma unroll
    for (int u = 0; u < U; ++u) cc[u] = row + __shfl(tab, (int)((dw >> (4 * u)) & 15u), 64);
}

// Rows of several batches: the lane's two words of 6-bit indices for batch j
// of wide dictionary block blk (dict_batches batches a block).
__device__ __forceinline__ uint64_t wide_word(const uint32_t *__restrict__ dword, int blk, int nbatch, int j, int lane)
{
    const uint2 w = reinterpret_cast<const uint2 *>(dword)[((size_t)blk * nbatch + j) * 64 + lane];
    return ((uint64_t)w.y << 32) | w.x;
}

// Columns of a batch's slots 0..U-1: the row plus the offset (one of the
// block's 64, one per lane) its 6-bit index names.
template <int U>
__device__ __forceinline__ void decode_wide(int (&cc)[U], uint64_t bits, int tab, int row)
{
#pragma unroll
    for (int u = 0; u < U; ++u) cc[u] = row + __shfl(tab, (int)((bits >> (6 * u)) & 63u), 64);
}

// Band-column product (one device): the row sum is split where the column
// crosses into the next band of bm columns (the last band takes the rest);
// the band partial sums are added in band order.  First column of the band
// after the one holding column col (INT_MAX for the last band).
__device__ __forceinline__ int band_next(int col, int bm, int nbands)
{
    const int b = col / bm;
    return b >= nbands - 1 ? INT_MAX : (b + 1) * bm;
}

// ONE: every chunk has at most U entries per row, so a chunk is one batch.
// Then the wave software-pipelines its chunks: a chunk's columns are loaded
// with the chunk before, and its gathers, values and own operands go out
// together with the next chunk's columns, behind one wait.  Otherwise (rows
// longer than U) the batches of each chunk are walked in turn, the same way
// batch to batch.  Every vector is addressed from its base through 32-bit
// offsets (fewer than 2^29 positions).
// BAND: the band-column product (positions are global ids, bands of bm).
// DICT_ON (ONE, U <= 8, no BAND): the chunks with an offset dictionary
// (cdict, dtab, dword) come first in the workgroup's range and take their
// columns from it.
template <typename VT, typename XT, int MODE, int U, bool ONE, bool BAND, bool DICT_ON>
__global__ __launch_bounds__(kBS) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_spmv_sell(
    int32_t nrows, int32_t nchunks, const int32_t *__restrict__ cptr, const int32_t *__restrict__ cpos,
    const uint8_t *__restrict__ clen, const uint8_t *__restrict__ rlen, const int32_t *__restrict__ ccol,
    const int32_t *__restrict__ col, const uint16_t *__restrict__ col16, const int2 *__restrict__ cbase,
    const VT *__restrict__ val, const XT *__restrict__ pin, const XT *__restrict__ r, XT *__restrict__ pout,
    XT *__restrict__ q, XT *__restrict__ x, double *__restrict__ part_a, const double *__restrict__ part_b,
    const double *__restrict__ part_b2, int32_t nb, int32_t slot, DevState *__restrict__ st,
    const int32_t *__restrict__ gate, int32_t bm, int32_t nbands, const int32_t *__restrict__ cdict,
    const int32_t *__restrict__ dtab, const uint32_t *__restrict__ dword, int32_t dict_batches)
{
    constexpr bool CG = MODE != SPMV_PLAIN;                        // status, (p, A p)
    constexpr bool PUPD = MODE == SPMV_FIRST || MODE == SPMV_STEP;  // p formed here
    // rows of several batches with the wide offset dictionaries
    constexpr bool WIDE = !ONE && DICT_ON && !BAND && U <= 10;
    // one-batch rows of at most 8 entries with the offset dictionaries
    constexpr bool USE_DICT = ONE && DICT_ON && U <= 8 && !BAND;
    constexpr int W = kBS / 64;
    __shared__ double ws[2 * (kBS / 64) + 2];
    __shared__ int s_flag;
    if (gate && dev::flag_load(gate) == 0) return;
    // the status word, the first chunk's columns and (STEP) the first round
    // of the update partials and the state go out together, behind one wait
    int flag0 = ST_RUNNING;
    if (CG && threadIdx.x == 0) flag0 = load_status(st);
    // the wave index is uniform: chunk headers come through the scalar path
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int rb = xcd_remap(blockIdx.x, gridDim.x);
    const int cpb = (nchunks + (int)gridDim.x - 1) / (int)gridDim.x;
    const int cend = min(rb * cpb + cpb, nchunks);
    int c = rb * cpb + w;

    // the columns of the first chunk's first batch, loaded before beta is
    // known
    int cc[U];
    uint32_t cw[U];      // column words of the next batch to run, decoded at use
    uint64_t wbits = 0;  // several batches, wide dictionary: that batch's index word
    int base = 0, L = 0, cb = 0, pos = 0, row = 0, len = 0, blk = -1;
    int2 wb = make_int2(0, 0);
    uint32_t dw = 0;  // ONE, dictionary chunk: the lane's 4-bit offset indices
    int tab = 0;      // and offset (lane & 15) of the chunk's table (wide: entry lane of 64)
    if (c < cend) {
        base = cptr[c];
        L = chunk_len(clen, c);
        cb = ccol[c];
        if (cb >= 0) wb = cbase[c];
        pos = cpos[c];
        row = pos + lane;
        if constexpr (ONE) {
            // the chunk's columns in its own encoding
            if (USE_DICT) blk = cdict[c];
            if (USE_DICT && blk >= 0)
                load_dict(dw, tab, blk, lane, dtab, dword);
            else
                load_cwords<U>(cw, cb, 0, L, lane, col, col16);
        } else {
            // the first batch's columns
            if (WIDE) {
                blk = cdict[c];
                if (blk >= 0) tab = ld32(dtab + blk * 64, (uint32_t)lane);
            }
            if (WIDE && blk >= 0)
                wbits = wide_word(dword, blk, dict_batches, 0, lane);
            else
                load_cwords<U>(cw, cb, 0, L, lane, col, col16);
        }
    }
    double2 tb[kPreRound], tb2[kPreRound];
    StepIn in{};
    if constexpr (MODE == SPMV_STEP) {
        pre_pairs<kPreRound>(tb, part_b, nb);
        if (part_b2) pre_pairs<kPreRound>(tb2, part_b2, nb);
        in = load_step_in(st, slot);
    }
    // x_k = x_{k-1} + alpha p_{k-1} is deferred to here.  It is owed whenever
    // the update of this slot ran (alpha != 0), whatever the status shows by
    // now: workgroup 0 may already have recorded this step's stop.
    const double alpha = MODE == SPMV_STEP ? st->alpha[slot] : 0.0;
    bool stop = false;
    if (CG) {
        if (threadIdx.x == 0) s_flag = flag0;
        __syncthreads();
        stop = s_flag != ST_RUNNING;
    }
    double beta = 0.0;
    if (MODE == SPMV_STEP && !stop)
        beta = finish_rr_pre<kPreRound>(tb, tb2, part_b, part_b2, nb, in, slot, st, ws, &stop);
    if (stop) {
        if (MODE == SPMV_STEP && alpha != 0.0)
            for (int c2 = rb * cpb + w; c2 < cend; c2 += W) {
                const int rr = cpos[c2] + lane;
                if (rr < nrows) x[rr] = (XT)((double)x[rr] + alpha * (double)pin[rr]);
            }
        return;
    }

    double acc = 0.0;
    if constexpr (ONE) {
        // Every chunk is one batch, and the wave software-pipelines its chunks:
        // for chunk c it issues the gathers (their columns were loaded with the
        // previous chunk), then chunk c's values and its rows' own r, p, x,
        // then the columns of its next chunk c+W (the header through the
        // scalar path, then the column or index words -- always the same loads,
        // at chunk c again when there is no next chunk of the kind), waits once
        // for all of them and for chunk c-W's stores, computes chunk c and
        // issues its stores.  So each chunk waits for one round trip of memory,
        // on loads and stores issued together, and only the next chunk's
        // columns are held across it.  Inside the workgroup's range the
        // dictionary chunks come first: the wave runs them in one loop, which
        // takes the columns from the index words, and then the rest of its
        // chunks in a second loop, which takes them from the column words
        // (every chunk has those).
        bool have = true;  // the next chunk is of the running loop's kind
        auto run_chunk = [&](auto kind) {
            constexpr bool DICT = decltype(kind)::value && USE_DICT;
            // a dictionary chunk's rows all exist; with at most 7 slots their
            // lengths come with the index words (top 4 bits)
            constexpr bool LEN_IN_WORD = DICT && U < 8;
            if constexpr (LEN_IN_WORD) len = (int)(dw >> 28);
            XT rx[U], px[U];
            if constexpr (DICT)
                decode_dict<U>(cc, dw, tab, row);
            else
                decode_cols<U>(cc, cw, cb, wb, lane);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (PUPD) rx[u] = ld32(r, (uint32_t)cc[u]);
                px[u] = ld32(pin, (uint32_t)cc[u]);
            }
            // keep the issue order: the gathers first
            __builtin_amdgcn_sched_barrier(0);
            // chunk c's values and its rows' own operands
            VT cv[U];
            load_vals<VT, U>(cv, val + base, L, lane);
            XT ro, po, xo;
            if constexpr (LEN_IN_WORD)
                load_row_nolen<XT, MODE>(ro, po, xo, pos, lane, r, pin, x);
            else
                load_row<XT, MODE>(len, ro, po, xo, pos, lane, nrows, rlen, r, pin, x);
            // the columns of the wave's next chunk when it is of this kind, else
            // of chunk c again (unused)
            const int nc = c + W;
            const bool nxt = nc < cend && (!DICT || cdict[nc] >= 0);
            const int lc = nxt ? nc : c;
            const int nbase = cptr[lc], nL = chunk_len(clen, lc), npos = cpos[lc];
            int ncb = 0;
            int2 nwb = make_int2(0, 0);
            uint32_t ncw[U], ndw = 0;
            int ntab = 0;
            if constexpr (DICT) {
                load_dict(ndw, ntab, cdict[lc], lane, dtab, dword);
            } else {
                ncb = ccol[lc];
                nwb = cbase[lc];
                load_cwords<U>(ncw, ncb, 0, nL, lane, col, col16);
            }
            __builtin_amdgcn_sched_barrier(0);
            // one wait for all that is in flight (with stores outstanding a
            // wait for the gathers alone is not possible)
            __builtin_amdgcn_s_waitcnt(dev::kWaitVmcnt0);
            XT prod[U];
#pragma unroll
            for (int u = 0; u < U; ++u) prod[u] = (XT)cv[u] * (PUPD ? pupd(rx[u], px[u], beta) : px[u]);
            XT sacc = XT(0);
            if constexpr (BAND) {
                // the products exist before the band bookkeeping branches
#pragma unroll
                for (int u = 0; u < U; ++u) asm volatile("" : "+v"(prod[u]));
                XT btot = XT(0);
                int bnext = -1;  // the first entry opens the row's first band
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (u < len) {
                        if (cc[u] >= bnext) {
                            btot = btot + sacc;
                            sacc = XT(0);
                            bnext = band_next(cc[u], bm, nbands);
                        }
                        sacc = sacc + prod[u];
                    }
                sacc = btot + sacc;
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (u < len) sacc = sacc + prod[u];
            }
            // computed here, on every lane: otherwise the compiler sinks the
            // products -- and the gathers with them -- into the store branch
            asm volatile("" : "+v"(sacc));
            if (row < nrows) {
                st32(q + pos, (uint32_t)lane, sacc);
                if (CG) {
                    const XT pr = PUPD ? pupd(ro, po, beta) : po;
                    if (PUPD) st32(pout + pos, (uint32_t)lane, pr);
                    if (MODE == SPMV_STEP) st32(x + pos, (uint32_t)lane, (XT)((double)xo + alpha * (double)po));
                    acc = acc + (double)pr * (double)sacc;
                }
            }
            c = nc;
            have = nxt;
            base = nbase;
            L = nL;
            pos = npos;
            row = npos + lane;
            if constexpr (DICT) {
                dw = ndw;
                tab = ntab;
            } else {
                cb = ncb;
                wb = nwb;
#pragma unroll
                for (int u = 0; u < U; ++u) cw[u] = ncw[u];
            }
        };
        if constexpr (USE_DICT) {
            if (c < cend && blk >= 0) {
                do
                    run_chunk(std::true_type{});
                while (have);
                // the rest of the wave's chunks: column words
                if (c < cend) {
                    base = cptr[c];
                    L = chunk_len(clen, c);
                    cb = ccol[c];
                    wb = cbase[c];
                    pos = cpos[c];
                    row = pos + lane;
                    load_cwords<U>(cw, cb, 0, L, lane, col, col16);
                }
            }
        }
        while (c < cend) run_chunk(std::false_type{});
    } else {
        // Rows of several batches.  The wave walks its chunks batch by batch.
        // For each batch it issues the gathers (their columns were loaded with
        // the batch before), the batch's values and the columns of the next
        // batch -- of this chunk, or the first of the wave's next chunk --, and
        // waits once for all of them; the rows' lengths and own operands come
        // with a chunk's first batch.
        for (; c < cend; c += W) {
            // the wave's next chunk (chunk c again past the end: its first
            // batch's columns are loaded and not used)
            const int nc = c + W;
            const int lc = nc < cend ? nc : c;
            const int nbase = cptr[lc], nL = chunk_len(clen, lc), ncb = ccol[lc], npos = cpos[lc];
            const int2 nwb = cbase[lc];
            const int nblk = WIDE ? cdict[lc] : -1;
            const uint32_t t = (uint32_t)min(lane, nrows - 1 - pos);
            const int l = ld32(rlen + pos, t);
            len = pos + lane < nrows ? l : 0;
            XT ro = XT(0), po = XT(0), xo = XT(0);
            if (CG) po = ld32(pin + pos, t);
            if (PUPD) ro = ld32(r + pos, t);
            if (MODE == SPMV_STEP) xo = ld32(x + pos, t);
            XT sacc = XT(0);
            XT btot = XT(0);
            int bnext = -1;
            for (int j0 = 0; j0 < L; j0 += U) {
                if (WIDE && blk >= 0)
                    decode_wide<U>(cc, wbits, tab, row);
                else
                    decode_cols<U>(cc, cw, cb, wb, lane);
                XT xr[U], xp[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (PUPD) xr[u] = ld32(r, (uint32_t)cc[u]);
                    xp[u] = ld32(pin, (uint32_t)cc[u]);
                }
                __builtin_amdgcn_sched_barrier(0);
                VT bv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) bv[u] = ld32(val + base, (uint32_t)(min(j0 + u, L - 1) * 64 + lane));
                if (j0 + U < L) {
                    if (WIDE && blk >= 0)
                        wbits = wide_word(dword, blk, dict_batches, j0 / U + 1, lane);
                    else
                        load_cwords<U>(cw, cb, j0 + U, L, lane, col, col16);
                } else {
                    if (WIDE && nblk >= 0) {
                        tab = ld32(dtab + nblk * 64, (uint32_t)lane);
                        wbits = wide_word(dword, nblk, dict_batches, 0, lane);
                    } else {
                        load_cwords<U>(cw, ncb, 0, nL, lane, col, col16);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                // one wait for all that is in flight (see the one-batch loop)
                __builtin_amdgcn_s_waitcnt(dev::kWaitVmcnt0);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const XT xx = PUPD ? pupd(xr[u], xp[u], beta) : xp[u];
                    if (j0 + u < len) {
                        if (BAND && cc[u] >= bnext) {
                            btot = btot + sacc;
                            sacc = XT(0);
                            bnext = band_next(cc[u], bm, nbands);
                        }
                        sacc = sacc + (XT)bv[u] * xx;
                    }
                }
            }
            if (BAND) sacc = btot + sacc;
            if (row < nrows) {
                st32(q + pos, (uint32_t)lane, sacc);
                if (CG) {
                    const XT pr = PUPD ? pupd(ro, po, beta) : po;
                    if (PUPD) st32(pout + pos, (uint32_t)lane, pr);
                    if (MODE == SPMV_STEP) st32(x + pos, (uint32_t)lane, (XT)((double)xo + alpha * (double)po));
                    acc = acc + (double)pr * (double)sacc;
                }
            }
            base = nbase;
            L = nL;
            cb = ncb;
            wb = nwb;
            pos = npos;
            row = npos + lane;
            blk = nblk;
        }
    }
    if (CG) {
        const double part = block_sum_all(acc, ws);
        if (threadIdx.x == 0) part_a[blockIdx.x] = part;
    }
}

// ---- the p-update of the split CG step ------------------------------------
//
// For matrices whose rows take several batches (27-point stencils), forming
// p = r + beta p at every gathered column doubles the gathers of the SpMV;
// there the step is split: this kernel finishes (r, r) -> beta and the
// stopping test (as the fused step's prologue), writes p_k = r + beta p_(k-1)
// (the same expression, so the same bits) and applies the previous update's
// x += alpha p_(k-1); the SpMV (mode PQ) then gathers p_k alone.  Batches of
// kUI * kBS positions per workgroup.
template <typename XT>
__global__ __launch_bounds__(kBS) void k_pstep(int32_t n, const XT *__restrict__ r, const XT *__restrict__ pin,
                                               XT *__restrict__ pout, XT *__restrict__ x,
                                               const double *__restrict__ part_b,
                                               const double *__restrict__ part_b2, int32_t nb, int32_t slot,
                                               DevState *__restrict__ st)
{
    constexpr int B = kUI * kBS;
    __shared__ double ws[2 * (kBS / 64) + 2];
    __shared__ int s_flag;
    // the status word, the operands, the first round of the update partials
    // and the state go out together (as in k_spmv_sell)
    int flag0 = ST_RUNNING;
    if (threadIdx.x == 0) flag0 = load_status(st);
    const int b0 = (int)blockIdx.x * B;
    XT rv[kUI], pv[kUI], xv[kUI];
#pragma unroll
    for (int i = 0; i < kUI; ++i) {
        const int c = min(b0 + (int)threadIdx.x + i * kBS, n - 1);
        rv[i] = r[c];
        pv[i] = pin[c];
        xv[i] = x[c];
    }
    double2 tb[kPreRoundS];
    pre_pairs<kPreRoundS>(tb, part_b, nb);
    const StepIn in = load_step_in(st, slot);
    // the x update is owed whenever this slot's update ran (see k_spmv_sell)
    const double alpha = st->alpha[slot];
    if (threadIdx.x == 0) s_flag = flag0;
    __syncthreads();
    bool stop = s_flag != ST_RUNNING;
    double beta = 0.0;
    if (!stop) {
        // (r, z) of a preconditioned run from the partials as they come
        double rr_new = sum_pre<kPreRoundS>(tb, part_b, nb), rz_new;
        if (part_b2) {
            rz_new = sum_partials_vec(part_b2, nb);
            block_sum2_all(rr_new, rz_new, ws);
        } else {
            rr_new = block_sum_all(rr_new, ws);
            rz_new = rr_new;
        }
        beta = step_test(rr_new, rz_new, in, slot, st, &stop);
    }
#pragma unroll
    for (int i = 0; i < kUI; ++i) {
        const int c = b0 + (int)threadIdx.x + i * kBS;
        if (c < n) {
            if (!stop) pout[c] = pupd(rv[i], pv[i], beta);
            if (alpha != 0.0) x[c] = (XT)((double)xv[i] + alpha * (double)pv[i]);
        }
    }
}

// ---- local SpMV, CSR row tiles (rows of very uneven length) -------------------
//
// Workgroup w owns tiles [w*tpb, (w+1)*tpb); a tile is consecutive rows with
// at most TN entries (or one longer row).  Values and columns are streamed
// with coalesced loads into LDS products; then each row's thread adds its
// products left to right.

template <typename VT, typename XT, int TN, int MODE>
__global__ __launch_bounds__(kBS) void k_spmv_csr(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                                  const VT *__restrict__ val, const int32_t *__restrict__ tile_row,
                                                  int32_t ntiles, const XT *__restrict__ pin,
                                                  const XT *__restrict__ r, XT *__restrict__ pout,
                                                  XT *__restrict__ q, XT *__restrict__ x,
                                                  double *__restrict__ part_a, const double *__restrict__ part_b,
                                                  const double *__restrict__ part_b2, int32_t nb, int32_t slot,
                                                  DevState *__restrict__ st, const int32_t *__restrict__ gate)
{
    constexpr bool CG = MODE != SPMV_PLAIN;
    constexpr int NI = TN / kBS;
    __shared__ XT prod[TN];
    __shared__ XT wsx[kBS / 64 + 1];
    __shared__ double ws[2 * (kBS / 64) + 2];
    __shared__ int s_flag;
    if (gate && dev::flag_load(gate) == 0) return;
    const int rb = xcd_remap(blockIdx.x, gridDim.x);
    const int tpb = (ntiles + (int)gridDim.x - 1) / (int)gridDim.x;
    const int tend = min(rb * tpb + tpb, ntiles);
    // the deferred x update is owed whenever this slot's update ran (see the
    // SELL kernel)
    const double alpha = MODE == SPMV_STEP ? st->alpha[slot] : 0.0;
    bool stop = CG && !running(st, &s_flag);
    double beta = 0.0;
    if (MODE == SPMV_STEP && !stop) beta = finish_rr(part_b, part_b2, nb, slot, st, ws, &stop);
    if (stop) {
        if (MODE == SPMV_STEP && alpha != 0.0 && rb * tpb < tend)
            for (int row = tile_row[rb * tpb] + (int)threadIdx.x; row < tile_row[tend]; row += kBS)
                x[row] = (XT)((double)x[row] + alpha * (double)pin[row]);
        return;
    }
    double acc = 0.0;
    for (int tile = rb * tpb; tile < tend; ++tile) {
        const int r0 = tile_row[tile], r1 = tile_row[tile + 1];
        const int k0 = rowptr[r0], k1 = rowptr[r1];
        if (k1 - k0 <= TN) {
            if (k1 > k0) {
                int jj[NI];
                VT vv[NI];
                XT xx[NI];
#pragma unroll
                for (int i = 0; i < NI; ++i) jj[i] = col[min(k0 + (int)threadIdx.x + i * kBS, k1 - 1)];
#pragma unroll
                for (int i = 0; i < NI; ++i) vv[i] = val[min(k0 + (int)threadIdx.x + i * kBS, k1 - 1)];
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
                    const XT pold = pin[row];
                    const XT pr = pupd(r[row], pold, beta);
                    pout[row] = pr;
                    if (MODE == SPMV_STEP) x[row] = (XT)((double)x[row] + alpha * (double)pold);
                    acc = acc + (double)pr * (double)s;
                }
            }
            __syncthreads();
        } else {
            // one row longer than a tile: strided partial sums, fixed-order tree
            XT s = XT(0);
            for (int k = k0 + (int)threadIdx.x; k < k1; k += kBS) {
                const int j = col[k];
                const XT xj = CG ? pupd(r[j], pin[j], beta) : pin[j];
                s = s + (XT)val[k] * xj;
            }
            s = block_sum_all(s, wsx);
            if (threadIdx.x == 0) {
                q[r0] = s;
                if (CG) {
                    const XT pold = pin[r0];
                    const XT pr = pupd(r[r0], pold, beta);
                    pout[r0] = pr;
                    if (MODE == SPMV_STEP) x[r0] = (XT)((double)x[r0] + alpha * (double)pold);
                    acc = acc + (double)pr * (double)s;
                }
            }
        }
    }
    if (CG) {
        const double part = block_sum_all(acc, ws);
        if (threadIdx.x == 0) part_a[blockIdx.x] = part;
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

// ---- alpha + assembly + r update + (r, r) partials ----------------------------
//
// Workgroup b (in dispatch order, so the slower interface batches start
// first) takes positions [b*B, b*B + B), B = kUI * kBS.  x += alpha p is left
// to the next SpMV step, which reads p anyway.

template <typename XT>
__global__ __launch_bounds__(kBS) void k_update(int32_t n_loc, int32_t n_own, int32_t n_if,
                                                const int32_t *__restrict__ pos_grp,
                                                const int32_t *__restrict__ copy_ptr,
                                                const int32_t *__restrict__ copy_pos, const double *__restrict__ dinv,
                                                XT *__restrict__ r, XT *__restrict__ z, const XT *__restrict__ q,
                                                double *__restrict__ part_b, double *__restrict__ part_b2,
                                                const double *__restrict__ part_a, int32_t na, int32_t slot,
                                                DevState *__restrict__ st)
{
    constexpr int B = kUI * kBS;
    __shared__ double ws[2 * (kBS / 64) + 2];
    __shared__ int s_flag;
    // the status word, the operands of a full interior batch, the first round
    // of the SpMV partials and (r, z) go out together, behind one wait
    int flag0 = ST_RUNNING;
    if (threadIdx.x == 0) flag0 = load_status(st);
    const bool pc = dinv != nullptr;
    const int b0 = (int)blockIdx.x * B;
    // a full batch of interior positions: operands loaded before alpha is known
    const bool plain = b0 >= n_if && b0 + B <= n_loc;
    XT rv[kUI], qv[kUI];
    double dv[kUI];
    if (plain) {
#pragma unroll
        for (int i = 0; i < kUI; ++i) {
            const int c = b0 + (int)threadIdx.x + i * kBS;
            rv[i] = r[c];
            qv[i] = q[c];
            dv[i] = pc ? dinv[c] : 1.0;
        }
    }
    double2 ta[kPreRoundA];
    pre_pairs<kPreRoundA>(ta, part_a, na);
    const double rz_cur = st->rz[slot];
    if (threadIdx.x == 0) s_flag = flag0;
    __syncthreads();
    if (s_flag != ST_RUNNING) {
        // no update this slot: the next step owes no x update
        if (blockIdx.x == 0 && threadIdx.x == 0) st->alpha[slot] = 0.0;
        return;
    }

    // finish (p, A p): alpha, or a breakdown when it is not positive
    const double pAp = block_sum_all(sum_pre<kPreRoundA>(ta, part_a, na), ws);
    const bool bad = !(pAp > 0.0) || !isfinite(pAp);
    const double alpha = rz_cur / pAp;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->pAp = pAp;
        st->alpha[slot] = bad ? 0.0 : alpha;
        if (bad) store_status(st, ST_BREAKDOWN);
    }
    if (bad) return;

    double acc = 0.0, acc2 = 0.0;
    if (plain) {
#pragma unroll
        for (int i = 0; i < kUI; ++i) {
            const int c = b0 + (int)threadIdx.x + i * kBS;
            const XT rc = (XT)((double)rv[i] - alpha * (double)qv[i]);
            r[c] = rc;
            acc = acc + (double)rc * (double)rc;
            if (pc) {
                const XT zc = (XT)(dv[i] * (double)rc);
                z[c] = zc;
                acc2 = acc2 + (double)rc * (double)zc;
            }
        }
    } else {
        for (int i = 0; i < kUI; ++i) {
            const int c = b0 + (int)threadIdx.x + i * kBS;
            if (c < n_loc) {
                const XT qc = c >= n_if ? q[c] : assembled(q, pos_grp[c], copy_ptr, copy_pos);
                const XT rc = (XT)((double)r[c] - alpha * (double)qc);
                r[c] = rc;
                const bool own = c < n_own || c >= n_if;
                if (own) acc = acc + (double)rc * (double)rc;
                if (pc) {
                    const XT zc = (XT)(dinv[c] * (double)rc);
                    z[c] = zc;
                    if (own) acc2 = acc2 + (double)rc * (double)zc;
                }
            }
        }
    }
    if (pc) {
        block_sum2_all(acc, acc2, ws);
        if (threadIdx.x == 0) {
            part_b[blockIdx.x] = acc;
            part_b2[blockIdx.x] = acc2;
        }
    } else {
        const double part = block_sum_all(acc, ws);
        if (threadIdx.x == 0) part_b[blockIdx.x] = part;
    }
}

// ---- fresh residual r = b - A x (assembly of q = A_bd x included) -----------

template <typename XT, bool FIRST>
__global__ __launch_bounds__(kBS) void k_residual(int32_t n_loc, int32_t n_own, int32_t n_if,
                                                  const int32_t *__restrict__ pos_grp,
                                                  const int32_t *__restrict__ copy_ptr,
                                                  const int32_t *__restrict__ copy_pos,
                                                  const double *__restrict__ dinv, const XT *__restrict__ b,
                                                  const XT *__restrict__ q, XT *__restrict__ r, XT *__restrict__ z,
                                                  XT *__restrict__ p0, double *__restrict__ partial)
{
    constexpr int B = kUI * kBS;
    __shared__ double ws[2 * (kBS / 64) + 2];
    const bool pc = dinv != nullptr;
    const int b0 = (int)blockIdx.x * B;
    double arr = 0.0, abb = 0.0, arz = 0.0;
    for (int i = 0; i < kUI; ++i) {
        const int c = b0 + (int)threadIdx.x + i * kBS;
        if (c < n_loc) {
            const XT qc = c >= n_if ? q[c] : assembled(q, pos_grp[c], copy_ptr, copy_pos);
            const XT bc = b[c];
            const XT rc = bc - qc;
            r[c] = rc;
            XT zc = rc;
            if (pc) {
                zc = (XT)(dinv[c] * (double)rc);
                z[c] = zc;
            }
            p0[c] = zc;
            if (c < n_own || c >= n_if) {
                arr = arr + (double)rc * (double)rc;
                if (pc) arz = arz + (double)rc * (double)zc;
                if (FIRST) abb = abb + (double)bc * (double)bc;
            }
        }
    }
    const double prr = block_sum_all(arr, ws);
    const double pbb = FIRST ? block_sum_all(abb, ws) : 0.0;
    const double prz = pc ? block_sum_all(arz, ws) : 0.0;
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = prr;
        partial[gridDim.x + blockIdx.x] = pbb;
        partial[2 * gridDim.x + blockIdx.x] = prz;
    }
}

// One workgroup: (r, r), (r, z) [and (b, b)], the stopping test, slot 0 of
// the state.
__global__ __launch_bounds__(kBS) void k_finish_residual(DevState *st, const double *partial, int n, int first, int pc)
{
    __shared__ double ws[2 * (kBS / 64) + 2];
    const double rr = sum_partials_all(partial, n, ws);
    const double bb = first ? sum_partials_all(partial + n, n, ws) : 0.0;
    const double rz = pc ? sum_partials_all(partial + 2 * n, n, ws) : rr;
    if (threadIdx.x != 0) return;
    if (first) {
        st->bb = bb;
        if (!isfinite(bb)) {
            store_status(st, ST_BREAKDOWN);
            return;
        }
        if (bb == 0.0) {
            if (st->hist && st->hist_cap > 0) st->hist[0] = 0.0;
            store_status(st, ST_ZERO_RHS);
            return;
        }
        st->stop = st->tol * sqrt(bb);
    }
    if (!isfinite(rr) || !isfinite(rz)) {
        store_status(st, ST_BREAKDOWN);
        return;
    }
    const int k = st->iter_last;
    st->rr[0] = rr;
    st->rz[0] = rz;
    st->iter[0] = k;
    st->rr_last = rr;
    if (st->hist && k < st->hist_cap) st->hist[k] = sqrt(rr / st->bb);
    if (sqrt(rr) <= st->stop)
        store_status(st, ST_CONVERGED);
    else if (k >= st->kmax)
        store_status(st, ST_MAXIT);
    else
        store_status(st, ST_RUNNING);
}

// ---- FP32-value iterative refinement ---------------------------------------

template <typename XT>
__global__ __launch_bounds__(kBS) void k_ir_prepare(int32_t n_loc, int32_t n_own, int32_t n_if,
                                                    const double *__restrict__ r64, XT *__restrict__ rin,
                                                    XT *__restrict__ p0, XT *__restrict__ d,
                                                    double *__restrict__ partial, const DevState *__restrict__ outer)
{
    constexpr int B = kUI * kBS;
    __shared__ double ws[2 * (kBS / 64) + 2];
    const double sc = sqrt(outer->rr_last);
    const int b0 = (int)blockIdx.x * B;
    double acc = 0.0;
    for (int i = 0; i < kUI; ++i) {
        const int c = b0 + (int)threadIdx.x + i * kBS;
        if (c < n_loc) {
            const XT v = (XT)(r64[c] / sc);
            rin[c] = v;
            p0[c] = v;
            d[c] = XT(0);
            if (c < n_own || c >= n_if) acc = acc + (double)v * (double)v;
        }
    }
    const double part = block_sum_all(acc, ws);
    if (threadIdx.x == 0) partial[blockIdx.x] = part;
}

__global__ __launch_bounds__(kBS) void k_ir_start(DevState *in, const DevState *outer, const double *partial, int n,
                                                  double inner_tol, int32_t inner_maxit, int32_t maxit)
{
    __shared__ double ws[2 * (kBS / 64) + 2];
    const double rr = sum_partials_all(partial, n, ws);
    if (threadIdx.x != 0) return;
    const int k = outer->iter_last;
    in->rr[0] = rr;
    in->rz[0] = rr;
    in->iter[0] = k;
    in->rr_last = rr;
    in->iter_last = k;
    in->bb = outer->bb / outer->rr_last;  // inner history: sqrt(rr / bb_in) = ||r|| / ||b|| estimate
    in->tol = inner_tol;
    in->stop = inner_tol * sqrt(rr);
    in->kmax = inner_maxit > 0 ? (int32_t)min((long long)k + inner_maxit, (long long)maxit) : maxit;
    in->hist = outer->hist;
    in->hist_cap = outer->hist_cap;
    if (!isfinite(rr))
        store_status(in, ST_BREAKDOWN);
    else if (sqrt(rr) <= in->stop)
        store_status(in, ST_CONVERGED);
    else if (k >= in->kmax)
        store_status(in, ST_MAXIT);
    else
        store_status(in, ST_RUNNING);
}

template <typename XT>
__global__ __launch_bounds__(kBS) void k_ir_accumulate(int32_t n_loc, double *__restrict__ x64,
                                                       const XT *__restrict__ d, const DevState *__restrict__ in,
                                                       DevState *__restrict__ outer)
{
    const int c = blockIdx.x * kBS + threadIdx.x;
    const bool broke = in->status == ST_BREAKDOWN;
    if (c == 0) {
        outer->iter_last = in->iter_last;
        if (broke) store_status(outer, ST_BREAKDOWN);
    }
    if (broke || c >= n_loc) return;
    const double sc = sqrt(outer->rr_last);
    x64[c] = x64[c] + sc * (double)d[c];
}

// ---- FP32 CG with FP64 residual replacement ----------------------------------

template <typename XT>
__global__ __launch_bounds__(kBS) void k_ru_start(int32_t n_loc, int32_t n_own, int32_t n_if,
                                                  const double *__restrict__ r64, XT *__restrict__ rin,
                                                  XT *__restrict__ d, double *__restrict__ partial)
{
    constexpr int B = kUI * kBS;
    __shared__ double ws[2 * (kBS / 64) + 2];
    const int b0 = (int)blockIdx.x * B;
    double acc = 0.0;
    for (int i = 0; i < kUI; ++i) {
        const int c = b0 + (int)threadIdx.x + i * kBS;
        if (c < n_loc) {
            const XT v = (XT)r64[c];
            rin[c] = v;
            d[c] = XT(0);
            if (c < n_own || c >= n_if) acc = acc + (double)v * (double)v;
        }
    }
    const double part = block_sum_all(acc, ws);
    if (threadIdx.x == 0) partial[blockIdx.x] = part;
}

__global__ __launch_bounds__(kBS) void k_ru_start_finish(DevState *in, const DevState *outer, const double *partial,
                                                         int n, double delta)
{
    __shared__ double ws[2 * (kBS / 64) + 2];
    const double rr = sum_partials_all(partial, n, ws);
    if (threadIdx.x != 0) return;
    const int k = outer->iter_last;
    in->rr[0] = rr;
    in->rz[0] = rr;
    in->iter[0] = k;
    in->rr_last = rr;
    in->iter_last = k;
    in->bb = outer->bb;
    in->tol = outer->tol;
    in->stop = outer->stop;
    in->kmax = outer->kmax;
    in->hist = outer->hist;
    in->hist_cap = outer->hist_cap;
    in->rref = sqrt(outer->rr_last);
    in->delta = delta;
    in->refresh = 0;
    store_status(in, isfinite(rr) ? ST_RUNNING : ST_BREAKDOWN);
}

// Chunk end: replace now?  (After an even number of steps the current
// (r, r) and iteration count are in slot 0.)
__global__ void k_ru_check(DevState *in)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const bool now = load_status(in) == ST_RUNNING && sqrt(in->rr[0]) <= in->delta * in->rref;
    dev::flag_store(&in->refresh, now ? 1 : 0);
}

template <typename XT>
__global__ __launch_bounds__(kBS) void k_ru_fold_gated(int32_t n_loc, double *__restrict__ x64, XT *__restrict__ d,
                                                       const DevState *__restrict__ in)
{
    if (dev::flag_load(&in->refresh) == 0) return;
    const int c = blockIdx.x * kBS + threadIdx.x;
    if (c >= n_loc) return;
    x64[c] = x64[c] + (double)d[c];
    d[c] = XT(0);
}

template <typename XT>
__global__ __launch_bounds__(kBS) void k_ru_residual(int32_t n_loc, int32_t n_own, int32_t n_if,
                                                     const int32_t *__restrict__ pos_grp,
                                                     const int32_t *__restrict__ copy_ptr,
                                                     const int32_t *__restrict__ copy_pos,
                                                     const double *__restrict__ b, const double *__restrict__ q,
                                                     double *__restrict__ r64, XT *__restrict__ rin,
                                                     double *__restrict__ partial, const DevState *__restrict__ in)
{
    constexpr int B = kUI * kBS;
    __shared__ double ws[2 * (kBS / 64) + 2];
    if (dev::flag_load(&in->refresh) == 0) return;
    const int b0 = (int)blockIdx.x * B;
    double a64 = 0.0, a32 = 0.0;
    for (int i = 0; i < kUI; ++i) {
        const int c = b0 + (int)threadIdx.x + i * kBS;
        if (c < n_loc) {
            const double qc = c >= n_if ? q[c] : assembled(q, pos_grp[c], copy_ptr, copy_pos);
            const double rc = b[c] - qc;
            r64[c] = rc;
            const XT v = (XT)rc;
            rin[c] = v;
            if (c < n_own || c >= n_if) {
                a64 = a64 + rc * rc;
                a32 = a32 + (double)v * (double)v;
            }
        }
    }
    const double p64 = block_sum_all(a64, ws);
    const double p32 = block_sum_all(a32, ws);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = p64;
        partial[gridDim.x + blockIdx.x] = p32;
    }
}

// The true residual decides: converged, or CG goes on from the new r with
// the same search direction.
__global__ __launch_bounds__(kBS) void k_ru_refresh_finish(DevState *in, DevState *outer, const double *partial, int n)
{
    __shared__ double ws[2 * (kBS / 64) + 2];
    __shared__ int32_t go;
    if (threadIdx.x == 0) go = dev::flag_load(&in->refresh);
    __syncthreads();
    if (go == 0) return;
    const double rr64 = sum_partials_all(partial, n, ws);
    const double rr32 = sum_partials_all(partial + n, n, ws);
    if (threadIdx.x != 0) return;
    const int k = in->iter[0];
    outer->rr_last = rr64;
    in->nrefresh = in->nrefresh + 1;
    if (in->hist && k < in->hist_cap) in->hist[k] = sqrt(rr64 / in->bb);
    if (!isfinite(rr64) || !isfinite(rr32)) {
        store_status(in, ST_BREAKDOWN);
    } else if (sqrt(rr64) <= in->stop) {
        store_status(in, ST_CONVERGED);
    } else {
        in->rr[0] = rr32;
        in->rz[0] = rr32;
        in->rr_last = rr32;
        in->rref = sqrt(rr64);
    }
}

template <typename XT>
__global__ __launch_bounds__(kBS) void k_ru_fold(int32_t n_loc, double *__restrict__ x64, XT *__restrict__ d,
                                                 const DevState *__restrict__ in, DevState *__restrict__ outer)
{
    const int c = blockIdx.x * kBS + threadIdx.x;
    const bool broke = in->status == ST_BREAKDOWN;
    if (c == 0) {
        outer->iter_last = in->iter_last;
        if (broke) store_status(outer, ST_BREAKDOWN);
    }
    if (broke || c >= n_loc) return;
    x64[c] = x64[c] + (double)d[c];
    d[c] = XT(0);
}

// ---- gathers, scatters, gradient -------------------------------------------

template <typename ST, typename XT>
__global__ __launch_bounds__(kBS) void k_gather(int32_t n_loc, const int32_t *__restrict__ l2g,
                                                const ST *__restrict__ src, XT *__restrict__ dst)
{
    const int c = blockIdx.x * kBS + threadIdx.x;
    if (c < n_loc) dst[c] = (XT)src[l2g[c]];
}

template <typename XT, typename DT>
__global__ __launch_bounds__(kBS) void k_scatter(int32_t n, const int32_t *__restrict__ g2own,
                                                 const XT *__restrict__ src, DT *__restrict__ dst,
                                                 const DevState *__restrict__ st)
{
    const int i = blockIdx.x * kBS + threadIdx.x;
    if (i >= n) return;
    const bool zero = st && st->status == ST_ZERO_RHS;
    dst[i] = zero ? DT(0) : (DT)src[g2own[i]];
}

// one thread per row: SELL threads walk the stored chunks (lane = row of the
// chunk), CSR threads the rows
__global__ __launch_bounds__(kBS) void k_grad_vals(Mat A, const int32_t *__restrict__ nzmap,
                                                   const int32_t *__restrict__ l2g, const double *__restrict__ lambda,
                                                   const double *__restrict__ x, double *__restrict__ dvals)
{
    const int t = blockIdx.x * kBS + threadIdx.x;
    if (A.fmt == FMT_SELL) {
        const int c = t >> 6, lane = t & 63;
        if (c >= A.nchunks) return;
        const int row = A.cpos[c] + lane;
        if (row >= A.nrows) return;
        const double li = lambda[l2g[row]];
        const int base = A.cptr[c], len = A.rlen[row], cb = A.ccol[c];
        for (int j = 0; j < len; ++j) {
            const int k = base + j * 64 + lane;
            const int cj = cb >= 0 ? narrow_col(A.col16[cb + j * 64 + lane], A.cbase[c]) : A.col[~cb + j * 64 + lane];
            dvals[nzmap[k]] = -(li * x[l2g[cj]]);
        }
    } else {
        if (t >= A.nrows) return;
        const double li = lambda[l2g[t]];
        for (int k = A.rowptr[t]; k < A.rowptr[t + 1]; ++k) dvals[nzmap[k]] = -(li * x[l2g[A.col[k]]]);
    }
}

__global__ __launch_bounds__(kBS) void k_set_values(int64_t len, const int32_t *__restrict__ nzmap,
                                                    const double *__restrict__ src, double *__restrict__ v64,
                                                    float *__restrict__ v32)
{
    const int64_t e = (int64_t)blockIdx.x * kBS + threadIdx.x;
    if (e >= len) return;
    const int m = nzmap[e];
    const double v = m >= 0 ? src[m] : 0.0;
    v64[e] = v;
    if (v32) v32[e] = (float)v;
}

// dinv[c] = 1 / a_ii of the node held at position c, a_ii = val_glob[dnz[c]]
__global__ __launch_bounds__(kBS) void k_set_dinv(int32_t n_loc, const int32_t *__restrict__ dnz,
                                                  const double *__restrict__ val_glob, double *__restrict__ dinv)
{
    const int c = blockIdx.x * kBS + threadIdx.x;
    if (c < n_loc) dinv[c] = 1.0 / val_glob[dnz[c]];
}

inline int nblocks(int64_t n) { return (int)((n + kBS - 1) / kBS); }
inline int nblocks(int64_t n, int per) { return (int)((n + per - 1) / per); }

template <typename VT, typename XT, int MODE>
void spmv_dispatch(hipStream_t s, const Mat &A, const XT *pin, const XT *r, XT *pout, XT *q, XT *x, Partials P,
                   DevState *st, int slot, const int32_t *gate = nullptr)
{
    if (A.nrows == 0) return;
    const dim3 grid(A.grid), block(kBS);
    if (A.fmt == FMT_SELL) {
#define SS_SELL(U, ONE, BAND)                                                                                    \
    hipLaunchKernelGGL((k_spmv_sell<VT, XT, MODE, U, ONE, BAND, false>), grid, block, 0, s, A.nrows, A.nchunks,   \
                       A.cptr, A.cpos, A.clen, A.rlen, A.ccol, A.col, A.col16, A.cbase, (const VT *)A.val, pin, r,  \
                       pout, q, x, P.a, (const double *)P.b, (const double *)P.b2, P.nb, slot, st, gate, A.band_m,  \
                       A.nbands, nullptr, nullptr, nullptr, 0)
#define SS_SELL_W(U)                                                                                             \
    hipLaunchKernelGGL((k_spmv_sell<VT, XT, MODE, U, false, false, true>), grid, block, 0, s, A.nrows, A.nchunks,  \
                       A.cptr, A.cpos, A.clen, A.rlen, A.ccol, A.col, A.col16, A.cbase, (const VT *)A.val, pin, r,  \
                       pout, q, x, P.a, (const double *)P.b, (const double *)P.b2, P.nb, slot, st, gate, A.band_m,  \
                       A.nbands, A.cdict, A.dtab, A.dword, A.dict_batches)
#define SS_SELL_D(U)                                                                                             \
    hipLaunchKernelGGL((k_spmv_sell<VT, XT, MODE, U, true, false, true>), grid, block, 0, s, A.nrows, A.nchunks, A.cptr,  \
                       A.cpos, A.clen, A.rlen, A.ccol, A.col, A.col16, A.cbase, (const VT *)A.val, pin, r, pout, q, x, \
                       P.a, (const double *)P.b, (const double *)P.b2, P.nb, slot, st, gate, A.band_m, A.nbands, A.cdict,  \
                       A.dtab, A.dword, 0)
#define SS_SELL_U(ONE, BAND)                    \
    switch (A.unroll) {                         \
    case 5: SS_SELL(5, ONE, BAND); break;       \
    case 7: SS_SELL(7, ONE, BAND); break;       \
    case 9: SS_SELL(9, ONE, BAND); break;       \
    default: SS_SELL(8, ONE, BAND); break;      \
    }
        // the band-column product exists in FP64 only (the setup refuses others)
        if constexpr (std::is_same<VT, double>::value && std::is_same<XT, double>::value) {
            if (A.nbands > 1) {
                if (A.one_batch) {
                    SS_SELL_U(true, true)
                } else {
                    SS_SELL_U(false, true)
                }
                return;
            }
        }
        if (A.one_batch && A.cdict && A.unroll <= 8) {
            // offset dictionaries (rows of at most 8 entries)
            switch (A.unroll) {
            case 5: SS_SELL_D(5); break;
            case 7: SS_SELL_D(7); break;
            default: SS_SELL_D(8); break;
            }
        } else if (A.one_batch) {
            SS_SELL_U(true, false)
        } else if (A.cdict && A.dict_batches > 0 && A.unroll <= 10) {
            // wide offset dictionaries (rows of several batches)
            switch (A.unroll) {
            case 5: SS_SELL_W(5); break;
            case 7: SS_SELL_W(7); break;
            case 9: SS_SELL_W(9); break;
            default: SS_SELL_W(8); break;
            }
        } else {
            SS_SELL_U(false, false)
        }
#undef SS_SELL_U
#undef SS_SELL_W
#undef SS_SELL_D
#undef SS_SELL
        return;
    }
#define SS_SPMV(TN)                                                                                              \
    hipLaunchKernelGGL((k_spmv_csr<VT, XT, TN, MODE>), grid, block, 0, s, A.rowptr, A.col, (const VT *)A.val,    \
                       A.tile_row, A.ntiles, pin, r, pout, q, x, P.a, (const double *)P.b, (const double *)P.b2,  \
                       P.nb, slot, st, gate)
    switch (A.tile_nnz) {
    case 1024: SS_SPMV(1024); break;
    case 4096: SS_SPMV(4096); break;
    default: SS_SPMV(2048); break;
    }
#undef SS_SPMV
}

// q = A p and the (p, A p) partials for a p already formed (split step).
template <typename VT, typename XT>
void spmv_pq_dispatch(hipStream_t s, const Mat &A, const XT *p, XT *q, Partials P, DevState *st)
{
    const dim3 grid(A.grid), block(kBS);
#define SS_PQ(U, BAND, WD)                                                                                          \
    hipLaunchKernelGGL((k_spmv_sell<VT, XT, SPMV_PQ, U, false, BAND, WD>), grid, block, 0, s, A.nrows, A.nchunks,    \
                       A.cptr, A.cpos, A.clen, A.rlen, A.ccol, A.col, A.col16, A.cbase, (const VT *)A.val, p,       \
                       (const XT *)nullptr, (XT *)nullptr, q, (XT *)nullptr, P.a, (const double *)nullptr,          \
                       (const double *)nullptr, 0, 0, st, (const int32_t *)nullptr, A.band_m, A.nbands,             \
                       WD ? A.cdict : nullptr, WD ? A.dtab : nullptr, WD ? A.dword : nullptr, WD ? A.dict_batches : 0)
#define SS_PQ_U(BAND, WD)                  \
    switch (A.unroll) {                    \
    case 5: SS_PQ(5, BAND, WD); break;     \
    case 7: SS_PQ(7, BAND, WD); break;     \
    case 9: SS_PQ(9, BAND, WD); break;     \
    default: SS_PQ(8, BAND, WD); break;    \
    }
    if constexpr (std::is_same<VT, double>::value && std::is_same<XT, double>::value) {
        if (A.nbands > 1) {
            SS_PQ_U(true, false)
            return;
        }
    }
    if (A.cdict && A.dict_batches > 0 && A.unroll <= 10) {
        SS_PQ_U(false, true)
    } else {
        SS_PQ_U(false, false)
    }
#undef SS_PQ_U
#undef SS_PQ
}

}  // namespace

// ---- launchers -----------------------------------------------------------------

template <typename ST, typename XT>
void launch_gather(hipStream_t s, int32_t n_loc, const int32_t *l2g, const ST *src, XT *dst)
{
    if (n_loc > 0)
        hipLaunchKernelGGL((k_gather<ST, XT>), dim3(nblocks(n_loc)), dim3(kBS), 0, s, n_loc, l2g, src, dst);
}

template <typename XT, typename DT>
void launch_scatter(hipStream_t s, int32_t n, const int32_t *g2own, const XT *src, DT *dst, const DevState *st)
{
    if (n > 0) hipLaunchKernelGGL((k_scatter<XT, DT>), dim3(nblocks(n)), dim3(kBS), 0, s, n, g2own, src, dst, st);
}

template <typename VT, typename XT>
void launch_spmv(hipStream_t s, const Mat &A, const XT *x, XT *q)
{
    spmv_dispatch<VT, XT, SPMV_PLAIN>(s, A, x, nullptr, nullptr, q, nullptr, Partials{nullptr, nullptr, 0, 0}, nullptr,
                                      0);
}

template <typename VT, typename XT>
void launch_spmv_first(hipStream_t s, const Mat &A, const XT *pin, const XT *r, XT *pout, XT *q, Partials P,
                       DevState *st)
{
    spmv_dispatch<VT, XT, SPMV_FIRST>(s, A, pin, r, pout, q, nullptr, P, st, 0);
}

template <typename VT, typename XT>
void launch_spmv_step(hipStream_t s, const Mat &A, const XT *pin, const XT *r, XT *pout, XT *q, XT *x, Partials P,
                      DevState *st, int slot)
{
    if (A.nrows == 0) return;
    if (!split_step(A)) {
        spmv_dispatch<VT, XT, SPMV_STEP>(s, A, pin, r, pout, q, x, P, st, slot);
        return;
    }
    // rows of several batches: p formed once per position, then the SpMV on it
    hipLaunchKernelGGL(k_pstep<XT>, dim3(nblocks(A.nrows, kUI * kBS)), dim3(kBS), 0, s, A.nrows, r, pin, pout, x,
                       (const double *)P.b, (const double *)P.b2, P.nb, slot, st);
    spmv_pq_dispatch<VT, XT>(s, A, pout, q, P, st);
}

template <typename XT>
void launch_iface_sum(hipStream_t s, const Iface &I, XT *q)
{
    if (I.ngamma > 0)
        hipLaunchKernelGGL(k_iface_sum<XT>, dim3(nblocks(I.ngamma)), dim3(kBS), 0, s, I.ngamma, I.copy_ptr,
                           I.copy_pos, q);
}

template <typename XT>
void launch_update(hipStream_t s, const Iface &I, XT *r, XT *z, const XT *q, Partials P, DevState *st, int slot)
{
    hipLaunchKernelGGL(k_update<XT>, dim3(I.grid), dim3(kBS), 0, s, I.n_loc, I.n_own, I.n_if, I.pos_grp,
                       I.copy_ptr, I.copy_pos, I.dinv, r, z, q, P.b, P.b2, (const double *)P.a, P.na, slot, st);
}

template <typename XT>
void launch_residual(hipStream_t s, const Iface &I, const XT *b, const XT *q, XT *r, XT *z, XT *p0, double *partial,
                     DevState *st, bool first)
{
    if (first)
        hipLaunchKernelGGL((k_residual<XT, true>), dim3(I.grid), dim3(kBS), 0, s, I.n_loc, I.n_own, I.n_if,
                           I.pos_grp, I.copy_ptr, I.copy_pos, I.dinv, b, q, r, z, p0, partial);
    else
        hipLaunchKernelGGL((k_residual<XT, false>), dim3(I.grid), dim3(kBS), 0, s, I.n_loc, I.n_own, I.n_if,
                           I.pos_grp, I.copy_ptr, I.copy_pos, I.dinv, b, q, r, z, p0, partial);
    hipLaunchKernelGGL(k_finish_residual, dim3(1), dim3(kBS), 0, s, st, partial, I.grid, first ? 1 : 0,
                       I.dinv ? 1 : 0);
}

void launch_grad_vals(hipStream_t s, const Mat &A, const int32_t *nzmap, const int32_t *l2g, const double *lambda,
                      const double *x, double *dvals)
{
    const int64_t threads = A.fmt == FMT_SELL ? (int64_t)A.nchunks * 64 : A.nrows;
    if (threads > 0)
        hipLaunchKernelGGL(k_grad_vals, dim3(nblocks(threads)), dim3(kBS), 0, s, A, nzmap, l2g, lambda, x, dvals);
}

void launch_set_dinv(hipStream_t s, int32_t n_loc, const int32_t *dnz, const double *val_glob, double *dinv)
{
    if (n_loc > 0) hipLaunchKernelGGL(k_set_dinv, dim3(nblocks(n_loc)), dim3(kBS), 0, s, n_loc, dnz, val_glob, dinv);
}

void launch_set_values(hipStream_t s, int64_t len, const int32_t *nzmap, const double *val_glob, double *val64,
                       float *val32)
{
    if (len > 0)
        hipLaunchKernelGGL(k_set_values, dim3(nblocks(len)), dim3(kBS), 0, s, len, nzmap, val_glob, val64, val32);
}

template <typename XT>
void launch_ir_prepare(hipStream_t s, const Iface &I, const double *r64, XT *rin, XT *p0, XT *d, double *partial,
                       const DevState *outer, DevState *inner, double inner_tol, int32_t inner_maxit, int32_t maxit)
{
    hipLaunchKernelGGL(k_ir_prepare<XT>, dim3(I.grid), dim3(kBS), 0, s, I.n_loc, I.n_own, I.n_if, r64, rin, p0, d,
                       partial, outer);
    hipLaunchKernelGGL(k_ir_start, dim3(1), dim3(kBS), 0, s, inner, outer, partial, I.grid, inner_tol, inner_maxit,
                       maxit);
}

template <typename XT>
void launch_ir_accumulate(hipStream_t s, int32_t n_loc, double *x64, const XT *d, const DevState *inner,
                          DevState *outer)
{
    hipLaunchKernelGGL(k_ir_accumulate<XT>, dim3(nblocks(std::max(n_loc, 1))), dim3(kBS), 0, s, n_loc, x64, d, inner,
                       outer);
}

template <typename XT>
void launch_ru_start(hipStream_t s, const Iface &I, const double *r64, XT *rin, XT *d, double *partial,
                     const DevState *outer, DevState *inner, double delta)
{
    hipLaunchKernelGGL(k_ru_start<XT>, dim3(I.grid), dim3(kBS), 0, s, I.n_loc, I.n_own, I.n_if, r64, rin, d, partial);
    hipLaunchKernelGGL(k_ru_start_finish, dim3(1), dim3(kBS), 0, s, inner, outer, partial, I.grid, delta);
}

template <typename XT>
void launch_ru_refresh(hipStream_t s, const Iface &I, const Mat &A64, double *x64, XT *d, const double *b64,
                       double *q64, double *r64, XT *rin, double *partial, DevState *inner, DevState *outer)
{
    hipLaunchKernelGGL(k_ru_check, dim3(1), dim3(64), 0, s, inner);
    hipLaunchKernelGGL(k_ru_fold_gated<XT>, dim3(nblocks(std::max(I.n_loc, 1))), dim3(kBS), 0, s, I.n_loc, x64, d,
                       inner);
    spmv_dispatch<double, double, SPMV_PLAIN>(s, A64, x64, nullptr, nullptr, q64, nullptr,
                                              Partials{nullptr, nullptr, 0, 0}, nullptr, 0, &inner->refresh);
    hipLaunchKernelGGL(k_ru_residual<XT>, dim3(I.grid), dim3(kBS), 0, s, I.n_loc, I.n_own, I.n_if, I.pos_grp,
                       I.copy_ptr, I.copy_pos, b64, q64, r64, rin, partial, inner);
    hipLaunchKernelGGL(k_ru_refresh_finish, dim3(1), dim3(kBS), 0, s, inner, outer, partial, I.grid);
}

template <typename XT>
void launch_ru_fold(hipStream_t s, int32_t n_loc, double *x64, XT *d, const DevState *inner, DevState *outer)
{
    hipLaunchKernelGGL(k_ru_fold<XT>, dim3(nblocks(std::max(n_loc, 1))), dim3(kBS), 0, s, n_loc, x64, d, inner,
                       outer);
}

// explicit instantiations
#define SS_INST(XT)                                                                                                  \
    template void launch_gather<double, XT>(hipStream_t, int32_t, const int32_t *, const double *, XT *);            \
    template void launch_scatter<XT, double>(hipStream_t, int32_t, const int32_t *, const XT *, double *,           \
                                             const DevState *);                                                      \
    template void launch_spmv<XT, XT>(hipStream_t, const Mat &, const XT *, XT *);                                   \
    template void launch_spmv_first<XT, XT>(hipStream_t, const Mat &, const XT *, const XT *, XT *, XT *, Partials,  \
                                            DevState *);                                                             \
    template void launch_spmv_step<XT, XT>(hipStream_t, const Mat &, const XT *, const XT *, XT *, XT *, XT *,       \
                                           Partials, DevState *, int);                                               \
    template void launch_iface_sum<XT>(hipStream_t, const Iface &, XT *);                                            \
    template void launch_update<XT>(hipStream_t, const Iface &, XT *, XT *, const XT *, Partials, DevState *, int); \
    template void launch_residual<XT>(hipStream_t, const Iface &, const XT *, const XT *, XT *, XT *, XT *,          \
                                      double *, DevState *, bool);                                                   \
    template void launch_ir_prepare<XT>(hipStream_t, const Iface &, const double *, XT *, XT *, XT *, double *,      \
                                        const DevState *, DevState *, double, int32_t, int32_t);                     \
    template void launch_ir_accumulate<XT>(hipStream_t, int32_t, double *, const XT *, const DevState *, DevState *); \
    template void launch_ru_start<XT>(hipStream_t, const Iface &, const double *, XT *, XT *, double *,             \
                                      const DevState *, DevState *, double);                                         \
    template void launch_ru_refresh<XT>(hipStream_t, const Iface &, const Mat &, double *, XT *, const double *,     \
                                        double *, double *, XT *, double *, DevState *, DevState *);                 \
    template void launch_ru_fold<XT>(hipStream_t, int32_t, double *, XT *, const DevState *, DevState *);
SS_INST(double)
SS_INST(float)
#undef SS_INST
// FP32 in and out (the FP32 product of ss_cg_apply_f32)
template void launch_gather<float, float>(hipStream_t, int32_t, const int32_t *, const float *, float *);
template void launch_scatter<float, float>(hipStream_t, int32_t, const int32_t *, const float *, float *,
                                           const DevState *);

}  // namespace ss
