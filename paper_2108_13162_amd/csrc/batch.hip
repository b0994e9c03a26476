// Batched CG: many independent SPD systems, each with NR right-hand sides,
// every (system, right-hand side) pair an independent CG (Algorithm 3, M = I,
// one sub-domain), all pairs advanced by the same launches.
//
// Device layout.  The systems' rows are concatenated; vectors hold the NR
// values of a row next to each other ([row][NR], FP64), so one read of a
// matrix entry serves all right-hand sides and a row's values are one
// 8*NR-byte access.  The matrix is SELL-64 per system (chunks of 64 rows of
// one system, one row per lane, entries column-major inside the chunk,
// columns as concatenated row indices).  Eight chunks form a 512-row granule,
// the unit of every partial sum: the dot products of a system are fixed-order
// sums of its granule partials, so results do not depend on how granules are
// grouped into workgroup tiles or on the grid size -- the launch shape the
// autotuner picks changes timing only.
//
// One CG iteration is two launches over the tiles of the systems that still
// have a running pair (a device-side list, rebuilt at the end of every polled
// chunk of iterations):
//   k_bupdate: (p, A p) of the system from its granule partials -> alpha per
//              pair, r -= alpha q, granule partials of (r, r);
//   k_bspmv:   (r, r) -> stopping test and beta per pair, x += alpha p of the
//              previous update for the tile's own rows (it reads p anyway),
//              p = r + beta p on the fly, q = A p, granule partials of (p, A p).
// Every workgroup of a system computes the system's scalars itself from the
// same partials in the same order (bitwise equal everywhere); the workgroup
// of the system's first tile records them.  A pair that stops freezes its x
// and r; a system with no running pair leaves the list.
//
// The same per-tile code also runs under a persistent schedule (k_bflow):
// one launch for all iterations, each system moving through its own update
// and SpMV phases (see "all iterations in one launch" below).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "device_common.h"
#include "host_common.h"
#include "ss_internal.h"

using namespace ss;

namespace {

constexpr int kWG = dev::kWG;
constexpr int kWaves = kWG / 64;
constexpr int kChunk = 64;                       // rows per SELL chunk
constexpr int kGranRows = 512;                   // rows per granule
constexpr int kMaxRowLen = 255;
constexpr int kRingBytes = 32768;                // LDS window of the staged SpMV
constexpr int kGridLimit = 65536;

enum : int32_t { BS_RUNNING = 0, BS_CONVERGED = 1, BS_MAXIT = 2, BS_BREAKDOWN = 3, BS_ZERO_RHS = 4 };
enum { M_PLAIN = 0, M_FIRST = 1, M_STEP = 2 };

struct BMat {
    const int32_t *col;   // [stored] chunk-major, lane-minor
    const double *val;    // [stored]
    const int32_t *cptr;  // [nchunks] first stored entry of each chunk
    const int32_t *crow;  // [nchunks+1] first row of each chunk (rows of chunk c: crow[c] .. crow[c+1])
    const uint8_t *clen;  // [nchunks] stored entries per lane
    const uint8_t *rlen;  // [nrows] entries of each row
};

struct BTiles {
    const int32_t *list;      // tiles to process
    const int32_t *nlist;     // their number (device)
    const int32_t *tile_sys;  // [ntiles] system of each tile
    const int32_t *tile_g0;   // [ntiles+1] granules of tile t: tile_g0[t] .. tile_g0[t+1]
    const int32_t *gran_c0;   // [ngran+1] chunks of granule g
    const int32_t *sys_g0;    // [nsys+1] granules of system s
    const int32_t *sys_h;     // [nsys] largest |column - row| of system s
};

// Per-pair CG state, pair (s, j) at index s * NR + j.  (r, r) and the
// iteration count are kept in two slots: the step kernel reads slot c and
// writes slot 1 - c.
struct BState {
    double *rr0, *rr1;
    int32_t *it0, *it1;
    double *bb, *stop, *rr_last;
    int32_t *it_last, *status, *restarts;
    int32_t *nrun;        // pairs still running (device)
    const int32_t *kmax;  // iteration limit (device)
    double *alpha;        // alpha of the last update per pair (0 for a stopped pair)
};

__device__ __forceinline__ double *rr_slot(const BState &S, int slot) { return slot ? S.rr1 : S.rr0; }
__device__ __forceinline__ int32_t *it_slot(const BState &S, int slot) { return slot ? S.it1 : S.it0; }

template <int NR>
__device__ __forceinline__ void ld_row(const double *__restrict__ v, int row, double (&o)[NR])
{
    if constexpr (NR == 1) {
        o[0] = v[row];
    } else if constexpr (NR == 2) {
        const double2 a = *reinterpret_cast<const double2 *>(v + 2 * row);
        o[0] = a.x;
        o[1] = a.y;
    } else {
        const double2 *p = reinterpret_cast<const double2 *>(v + 4 * row);
        const double2 a = p[0], b = p[1];
        o[0] = a.x;
        o[1] = a.y;
        o[2] = b.x;
        o[3] = b.y;
    }
}

template <int NR>
__device__ __forceinline__ void st_row(double *__restrict__ v, int row, const double (&o)[NR])
{
    if constexpr (NR == 1) {
        v[row] = o[0];
    } else if constexpr (NR == 2) {
        *reinterpret_cast<double2 *>(v + 2 * row) = make_double2(o[0], o[1]);
    } else {
        double2 *p = reinterpret_cast<double2 *>(v + 4 * row);
        p[0] = make_double2(o[0], o[1]);
        p[1] = make_double2(o[2], o[3]);
    }
}

// The pair statuses of system s, in two parts, so that their loads go out
// with a tile's other first loads and share their wait: pre_status issues
// them (thread j < NR gets pair j's), publish_status shares them through LDS
// and returns true if any pair is running.
template <int NR>
__device__ __forceinline__ int32_t pre_status(const BState &S, int s)
{
    return threadIdx.x < NR ? dev::flag_load(&S.status[s * NR + threadIdx.x]) : BS_RUNNING;
}

template <int NR>
__device__ __forceinline__ bool publish_status(int32_t f, int32_t *sh)
{
    __syncthreads();  // sh may still be read from the previous tile
    if (threadIdx.x < NR) sh[threadIdx.x] = f;
    __syncthreads();
    bool any = false;
#pragma unroll
    for (int j = 0; j < NR; ++j) any = any || sh[j] == BS_RUNNING;
    return any;
}

// Per right-hand side, the sum of part[g * NR + j] over granules g0 .. g1, in
// a fixed order: thread t adds flat elements t, t + kWG, ... (all of the same
// j = t % NR), then the lanes of equal residue, then the waves in order.
// Every thread receives the NR sums.  ws: kWaves * NR.
template <int NR>
__device__ __forceinline__ void sys_sum_tail(double v, double *ws, double (&out)[NR])
{
    v = dev::wave_sum_strided<NR>(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane < NR) ws[w * NR + lane] = v;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        double t = ws[j];
#pragma unroll
        for (int i = 1; i < kWaves; ++i) t = t + ws[i * NR + j];
        out[j] = t;
    }
    __syncthreads();
}

template <int NR>
__device__ __forceinline__ void sys_sum(const double *__restrict__ part, int g0, int g1, double *ws, double (&out)[NR])
{
    const int lo = g0 * NR, hi = g1 * NR;
    double v = 0.0;
    for (int e = lo + (int)threadIdx.x; e < hi; e += kWG) v = v + part[e];
    sys_sum_tail<NR>(v, ws, out);
}

// sys_sum with its first kPreSys elements per thread loaded ahead (with a
// tile's first loads, at the last element past the end) and dropped where
// they are added when past the end: the same order, so the same bits.
constexpr int kPreSys = 2;  // one round for systems of up to 128 granules with 4 right-hand sides

template <int NR>
__device__ __forceinline__ void pre_sys(double (&t)[kPreSys], const double *__restrict__ part, int g0, int g1)
{
    const int lo = g0 * NR, hi = g1 * NR;
#pragma unroll
    for (int i = 0; i < kPreSys; ++i) t[i] = part[min(lo + (int)threadIdx.x + i * kWG, hi - 1)];
}

template <int NR>
__device__ __forceinline__ void sys_sum_pre(const double (&t)[kPreSys], const double *__restrict__ part, int g0,
                                            int g1, double *ws, double (&out)[NR])
{
    const int lo = g0 * NR, hi = g1 * NR;
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < kPreSys; ++i) v = v + (lo + (int)threadIdx.x + i * kWG < hi ? t[i] : 0.0);
    for (int e = lo + (int)threadIdx.x + kPreSys * kWG; e < hi; e += kWG) v = v + part[e];
    sys_sum_tail<NR>(v, ws, out);
}

// Granule partial of per-thread values of right-hand side t % NR (flat
// element layout): written to part[g * NR + j].
template <int NR>
__device__ __forceinline__ void granule_store_strided(double v, double *__restrict__ part, int g, double *ws)
{
    v = dev::wave_sum_strided<NR>(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane < NR) ws[w * NR + lane] = v;
    __syncthreads();
    if (threadIdx.x < NR) {
        double t = ws[threadIdx.x];
#pragma unroll
        for (int i = 1; i < kWaves; ++i) t = t + ws[i * NR + threadIdx.x];
        part[g * NR + threadIdx.x] = t;
    }
    __syncthreads();
}

// Granule partial of per-thread values of every right-hand side (row
// layout: each thread holds NR accumulators).
template <int NR>
__device__ __forceinline__ void granule_store_rows(const double (&acc)[NR], double *__restrict__ part, int g, double *ws)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
        const double v = dev::wave_sum(acc[j]);
        if (lane == 0) ws[w * NR + j] = v;
    }
    __syncthreads();
    if (threadIdx.x < NR) {
        double t = ws[threadIdx.x];
#pragma unroll
        for (int i = 1; i < kWaves; ++i) t = t + ws[i * NR + threadIdx.x];
        part[g * NR + threadIdx.x] = t;
    }
    __syncthreads();
}

// This workgroup's share of the tile list: the list is cut into 8 contiguous
// XCD ranges (so a system's tiles share an L2), strided inside the XCD.
struct Share {
    int i, end, step;
};
__device__ __forceinline__ Share list_share(int nact)
{
    const int x = blockIdx.x % dev::kNumXcd, loc = blockIdx.x / dev::kNumXcd, gx = gridDim.x / dev::kNumXcd;
    const int lo = (int)((int64_t)nact * x / dev::kNumXcd), hi = (int)((int64_t)nact * (x + 1) / dev::kNumXcd);
    return Share{lo + loc, hi, gx};
}

// ---- SpMV over the listed tiles ------------------------------------------------
//  M_PLAIN: q = A pin.
//  M_FIRST: p = r (pairs running), q = A p, partials (p, q) -> part_a.
//  M_STEP : (r, r) from part_b -> stopping test, beta; p = r + beta pin;
//           q = A p, partials (p, q) -> part_a.
//
// Staged path (systems whose entries all lie within h <= HMAX rows of the
// diagonal): the workgroup keeps the vector it multiplies (p = r + beta p,
// r or pin) for the rows [first row of the granule - h, last row + h) in an
// LDS ring of W rows, sliding granule by granule through its tile, so every
// vector row is read from memory once per tile (plus the 2h halo rows) and
// the column gathers are LDS reads.  Other systems gather from memory.
// x += alpha p of the previous update (per right-hand side) for rows
// [r0, r1), in row layout.
template <int NR>
__device__ __forceinline__ void x_update_rows(double *__restrict__ x, const double *__restrict__ p, int r0, int r1,
                                              const double (&al)[NR])
{
    for (int row = r0 + (int)threadIdx.x; row < r1; row += kWG) {
        double xv[NR], pv[NR];
        ld_row<NR>(x, row, xv);
        ld_row<NR>(p, row, pv);
#pragma unroll
        for (int j = 0; j < NR; ++j)
            if (al[j] != 0.0) xv[j] = xv[j] + al[j] * pv[j];
        st_row<NR>(x, row, xv);
    }
}

template <int NR>
constexpr int ring_rows()
{
    return kRingBytes / (8 * NR);  // a power of two
}

// One tile t of the SpMV (whole workgroup).  ws: kWaves * NR, sh_st: NR,
// ring: ring_rows<NR>() * NR doubles of LDS.
template <int NR, int U, int MODE, bool ALL_STAGED>
__device__ __forceinline__ void spmv_tile(const BMat &M, const BTiles &T, const BState &S, int t,
                                          const double *__restrict__ pin, const double *__restrict__ r,
                                          double *__restrict__ pout, double *__restrict__ q, double *__restrict__ x,
                                          double *__restrict__ part_a, const double *__restrict__ part_b, int slot,
                                          double *ws, int32_t *sh_st, double *ring)
{
    constexpr bool CG = MODE != M_PLAIN;
    constexpr int W = ring_rows<NR>();
    constexpr int HMAX = (W - kGranRows) / 2;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    {
        const int s = T.tile_sys[t];
        double beta[NR];
#pragma unroll
        for (int j = 0; j < NR; ++j) beta[j] = 0.0;
        // alpha of the previous update (0 for a pair that did not run in it):
        // the x += alpha p that update left to this step
        double al[NR];
        bool xupd = false;
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            al[j] = MODE == M_STEP ? S.alpha[s * NR + j] : 0.0;
            xupd = xupd || al[j] != 0.0;
        }
        const int own0 = M.crow[T.gran_c0[T.tile_g0[t]]], own1 = M.crow[T.gran_c0[T.tile_g0[t + 1]]];
        // the statuses, the system's (r, r) partials and the pairs' state go
        // out together, behind one wait
        const int32_t f = CG ? pre_status<NR>(S, s) : BS_RUNNING;
        double tp[kPreSys];
        double rrv[NR], stv[NR];
        int32_t itv[NR];
        int kmax = 0;
        if (MODE == M_STEP) {
            pre_sys<NR>(tp, part_b, T.sys_g0[s], T.sys_g0[s + 1]);
            const double *rrc = rr_slot(S, slot);
            const int32_t *itc = it_slot(S, slot);
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                rrv[j] = rrc[s * NR + j];
                itv[j] = itc[s * NR + j];
                stv[j] = S.stop[s * NR + j];
            }
            kmax = *S.kmax;
        }
        if (CG) {
            // (the statuses may already show this step's stops, recorded by
            // the system's first tile: the x update is owed all the same)
            if (!publish_status<NR>(f, sh_st)) {
                if (MODE == M_STEP && xupd) x_update_rows<NR>(x, pin, own0, own1, al);
                return;
            }
            bool any = false;
            if (MODE == M_STEP) {
                double rrn[NR];
                sys_sum_pre<NR>(tp, part_b, T.sys_g0[s], T.sys_g0[s + 1], ws, rrn);
                const bool lead = T.tile_g0[t] == T.sys_g0[s] && threadIdx.x == 0;
#pragma unroll
                for (int j = 0; j < NR; ++j) {
                    if (sh_st[j] != BS_RUNNING) continue;
                    const int pr = s * NR + j;
                    const int kn = itv[j] + 1;
                    int32_t stop = BS_RUNNING;
                    if (!isfinite(rrn[j]))
                        stop = BS_BREAKDOWN;
                    else if (sqrt(rrn[j]) <= stv[j])
                        stop = BS_CONVERGED;
                    else if (kn >= kmax)
                        stop = BS_MAXIT;
                    if (lead) {
                        if (stop != BS_BREAKDOWN) {
                            rr_slot(S, slot ^ 1)[pr] = rrn[j];
                            it_slot(S, slot ^ 1)[pr] = kn;
                            S.rr_last[pr] = rrn[j];
                            S.it_last[pr] = kn;
                        }
                        if (stop != BS_RUNNING) {
                            dev::flag_store(&S.status[pr], stop);
                            atomicSub(S.nrun, 1);
                        }
                    }
                    if (stop == BS_RUNNING) {
                        beta[j] = rrn[j] / rrv[j];
                        any = true;
                    }
                }
            } else {
                any = true;
            }
            if (!any) {
                // every pair stops here: the previous update's x still lands
                if (MODE == M_STEP && xupd) x_update_rows<NR>(x, pin, own0, own1, al);
                return;
            }
        }
        const int g0 = T.tile_g0[t], g1 = T.tile_g0[t + 1];
        const int h = T.sys_h[s];
        const bool staged = ALL_STAGED || h <= HMAX;  // ALL_STAGED: every system qualifies
        const int S0 = M.crow[T.gran_c0[T.sys_g0[s]]], S1 = M.crow[T.gran_c0[T.sys_g0[s + 1]]];
        int hi = -1;  // ring holds rows [.., hi)
        for (int g = g0; g < g1; ++g) {
            const int c0 = T.gran_c0[g], c1 = T.gran_c0[g + 1];
            // first batch of the wave's first chunk, issued before the staging
            int cc[U];
            double vv[U];
            bool have = false;
            if (c0 + w < c1) {
                const int L0 = M.clen[c0 + w], base0 = M.cptr[c0 + w];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (u < L0) {
                        const int k = base0 + u * kChunk + lane;
                        cc[u] = M.col[k];
                        vv[u] = M.val[k];
                    }
                }
                have = true;
            }
            if (staged) {
                const int a = M.crow[c0], e = M.crow[c1];
                const int need = min(S1, e + h);
                const int from = hi < 0 ? max(S0, a - h) : hi;
                for (int row = from + (int)threadIdx.x; row < need; row += kWG) {
                    double v[NR];
                    if (MODE == M_PLAIN) {
                        ld_row<NR>(pin, row, v);
                    } else if (MODE == M_FIRST) {
                        ld_row<NR>(r, row, v);
                    } else {
                        double rv[NR], pv[NR];
                        ld_row<NR>(r, row, rv);
                        ld_row<NR>(pin, row, pv);
#pragma unroll
                        for (int j = 0; j < NR; ++j) v[j] = rv[j] + beta[j] * pv[j];
                        if (row >= own0 && row < own1) {
                            double xv[NR];
                            ld_row<NR>(x, row, xv);
#pragma unroll
                            for (int j = 0; j < NR; ++j)
                                if (al[j] != 0.0) xv[j] = xv[j] + al[j] * pv[j];
                            st_row<NR>(x, row, xv);
                        }
                    }
                    st_row<NR>(ring, row & (W - 1), v);
                }
                hi = need;
                __syncthreads();
            }
            double acc[NR];
#pragma unroll
            for (int j = 0; j < NR; ++j) acc[j] = 0.0;
            for (int c = c0 + w; c < c1; c += kWaves) {
                const int row = M.crow[c] + lane;
                const bool valid = row < M.crow[c + 1];
                const int len = valid ? (int)M.rlen[row] : 0;
                const int L = M.clen[c];
                const int base = M.cptr[c];
                double sum[NR];
#pragma unroll
                for (int j = 0; j < NR; ++j) sum[j] = 0.0;
                for (int j0 = 0; j0 < L; j0 += U) {
                    if (!have) {
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            if (j0 + u < L) {
                                const int k = base + (j0 + u) * kChunk + lane;
                                cc[u] = M.col[k];
                                vv[u] = M.val[k];
                            }
                        }
                    }
                    have = false;
                    if (staged) {
                        // LDS gathers are short: use each entry at once
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            if (j0 + u < len) {
                                double xr[NR];
                                ld_row<NR>(ring, cc[u] & (W - 1), xr);
#pragma unroll
                                for (int j = 0; j < NR; ++j) sum[j] = sum[j] + vv[u] * xr[j];
                            }
                        }
                    } else {
                        double xx[U][NR];
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            if (j0 + u < L) {
                                if (MODE == M_PLAIN) {
                                    ld_row<NR>(pin, cc[u], xx[u]);
                                } else if (MODE == M_FIRST) {
                                    ld_row<NR>(r, cc[u], xx[u]);
                                } else {
                                    double rv[NR], pv[NR];
                                    ld_row<NR>(r, cc[u], rv);
                                    ld_row<NR>(pin, cc[u], pv);
#pragma unroll
                                    for (int j = 0; j < NR; ++j) xx[u][j] = rv[j] + beta[j] * pv[j];
                                }
                            }
                        }
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            if (j0 + u < len) {
#pragma unroll
                                for (int j = 0; j < NR; ++j) sum[j] = sum[j] + vv[u] * xx[u][j];
                            }
                    }
                }
                have = false;
                if (valid) {
                    st_row<NR>(q, row, sum);
                    if (CG) {
                        double pr[NR];
                        if (staged) {
                            ld_row<NR>(ring, row & (W - 1), pr);
                        } else if (MODE == M_FIRST) {
                            ld_row<NR>(r, row, pr);
                        } else {
                            double rv[NR], pv[NR];
                            ld_row<NR>(r, row, rv);
                            ld_row<NR>(pin, row, pv);
#pragma unroll
                            for (int j = 0; j < NR; ++j) pr[j] = rv[j] + beta[j] * pv[j];
                            if (MODE == M_STEP) {
                                double xv[NR];
                                ld_row<NR>(x, row, xv);
#pragma unroll
                                for (int j = 0; j < NR; ++j)
                                if (al[j] != 0.0) xv[j] = xv[j] + al[j] * pv[j];
                                st_row<NR>(x, row, xv);
                            }
                        }
                        st_row<NR>(pout, row, pr);
#pragma unroll
                        for (int j = 0; j < NR; ++j) acc[j] = acc[j] + pr[j] * sum[j];
                    }
                }
            }
            if (CG)
                granule_store_rows<NR>(acc, part_a, g, ws);  // ends with a barrier
            else if (staged)
                __syncthreads();  // ring reads done before the next granule is staged
        }
    }
}

template <int NR, int U, int MODE, bool ALL_STAGED>
__global__ __launch_bounds__(kWG) void k_bspmv(BMat M, BTiles T, BState S, const double *__restrict__ pin,
                                               const double *__restrict__ r, double *__restrict__ pout,
                                               double *__restrict__ q, double *__restrict__ x,
                                               double *__restrict__ part_a, const double *__restrict__ part_b,
                                               int slot, const int32_t *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    __shared__ double ws[kWaves * NR];
    __shared__ int32_t sh_st[NR];
    __shared__ __align__(16) double ring[ring_rows<NR>() * NR];
    const Share sh = list_share(*T.nlist);
    for (int i = sh.i; i < sh.end; i += sh.step)
        spmv_tile<NR, U, MODE, ALL_STAGED>(M, T, S, T.list[i], pin, r, pout, q, x, part_a, part_b, slot, ws, sh_st,
                                           ring);
}

// ---- alpha + x / r update + (r, r) partials ----------------------------------

// One tile t of the update (whole workgroup).  ws: kWaves * NR, sh_st: NR.
template <int NR>
__device__ __forceinline__ void update_tile(const BMat &M, const BTiles &T, const BState &S, int t,
                                            double *__restrict__ r, const double *__restrict__ q,
                                            double *__restrict__ part_b, const double *__restrict__ part_a, int slot,
                                            double *ws, int32_t *sh_st)
{
    constexpr int NI = kGranRows * NR / kWG;  // elements per thread of a full granule
    const int jt = threadIdx.x % NR;
    {
        const int s = T.tile_sys[t];
        // the statuses, the operands of the first granule, the system's
        // (p, A p) partials and the pairs' (r, r) go out together, behind one
        // wait
        const int32_t f = pre_status<NR>(S, s);
        const int g0 = T.tile_g0[t], g1 = T.tile_g0[t + 1];
        double rv[NI], qv[NI];
        int e0 = M.crow[T.gran_c0[g0]] * NR, e1 = M.crow[T.gran_c0[g0 + 1]] * NR;
        bool full = e1 - e0 == kGranRows * NR;
        if (full) {
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const int e = e0 + (int)threadIdx.x + k * kWG;
                rv[k] = r[e];
                qv[k] = q[e];
            }
        }
        double tp[kPreSys];
        pre_sys<NR>(tp, part_a, T.sys_g0[s], T.sys_g0[s + 1]);
        double rrv[NR];
        const double *rrc = rr_slot(S, slot);
#pragma unroll
        for (int j = 0; j < NR; ++j) rrv[j] = rrc[s * NR + j];
        if (!publish_status<NR>(f, sh_st)) {
            // nothing ran: the next step owes no x update for this system
            if (T.tile_g0[t] == T.sys_g0[s] && threadIdx.x < NR) S.alpha[s * NR + threadIdx.x] = 0.0;
            return;
        }
        double pAp[NR];
        sys_sum_pre<NR>(tp, part_a, T.sys_g0[s], T.sys_g0[s + 1], ws, pAp);
        const bool lead = T.tile_g0[t] == T.sys_g0[s] && threadIdx.x == 0;
        bool any = false, run = false;
        double a = 0.0;  // alpha of this thread's right-hand side jt
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            double al = 0.0;
            if (sh_st[j] == BS_RUNNING) {
                const int pr = s * NR + j;
                if (!(pAp[j] > 0.0) || !isfinite(pAp[j])) {
                    if (lead) {
                        dev::flag_store(&S.status[pr], BS_BREAKDOWN);
                        atomicSub(S.nrun, 1);
                    }
                } else {
                    al = rrv[j] / pAp[j];
                    any = true;
                    if (j == jt) run = true;
                }
            }
            if (j == jt) a = al;
            // the next CG step applies x += alpha p with these (0: no change)
            if (lead) S.alpha[s * NR + j] = al;
        }
        if (!any) return;
        for (int g = g0; g < g1; ++g) {
            if (g != g0) {
                e0 = M.crow[T.gran_c0[g]] * NR;
                e1 = M.crow[T.gran_c0[g + 1]] * NR;
                full = e1 - e0 == kGranRows * NR;
                if (full) {
#pragma unroll
                    for (int k = 0; k < NI; ++k) {
                        const int e = e0 + (int)threadIdx.x + k * kWG;
                        rv[k] = r[e];
                        qv[k] = q[e];
                    }
                }
            }
            double accv = 0.0;
            if (full) {
                if (run) {
#pragma unroll
                    for (int k = 0; k < NI; ++k) {
                        const int e = e0 + (int)threadIdx.x + k * kWG;
                        const double rn = rv[k] - a * qv[k];
                        r[e] = rn;
                        accv = accv + rn * rn;
                    }
                }
            } else {
                for (int e = e0 + (int)threadIdx.x; e < e1; e += kWG) {
                    if (run) {
                        const double rn = r[e] - a * q[e];
                        r[e] = rn;
                        accv = accv + rn * rn;
                    }
                }
            }
            granule_store_strided<NR>(accv, part_b, g, ws);
        }
    }
}

template <int NR>
__global__ __launch_bounds__(kWG) void k_bupdate(BMat M, BTiles T, BState S, double *__restrict__ r,
                                                 const double *__restrict__ q, double *__restrict__ part_b,
                                                 const double *__restrict__ part_a, int slot)
{
    __shared__ double ws[kWaves * NR];
    __shared__ int32_t sh_st[NR];
    const Share sh = list_share(*T.nlist);
    for (int i = sh.i; i < sh.end; i += sh.step) update_tile<NR>(M, T, S, T.list[i], r, q, part_b, part_a, slot, ws, sh_st);
}

// ---- all iterations in one launch ----------------------------------------------
//
// The iterations of every system run inside one persistent launch, each
// system at its own pace: phase seq of system s is the update of its step
// seq / 2 when seq is even, the SpMV step after that update when odd (slot
// and p ping-pong from seq / 2 as in the chunked launches).  A phase is the
// system's tiles, claimed one at a time by whichever workgroup is free: the
// claim word of s holds (seq << 32) | next unclaimed tile, and an atomic add
// on it hands out the tile.  The workgroup that finishes the last tile of a
// phase publishes the next one (after an update: the SpMV step; after a step:
// the next update while a pair of s runs, else s retires).  Phases of one
// system never overlap, so the kernels' per-tile code runs unchanged and the
// results are bitwise those of the chunked launches; systems do not wait for
// each other, and no workgroup waits for a particular other one: a free
// workgroup takes a tile of one of the first systems in priority order
// (largest first) that have one, else polls.  Every workgroup leaves when all systems
// have retired, or when no phase has finished for a long time (an error
// flag the host reports; it never happens in a correct run).

constexpr uint32_t kRetired = 0xffffffffu;
constexpr uint32_t kStallPolls = 1u << 22;  // polls without a finished phase before giving up
constexpr int kSpread = 8;                  // claimable systems a free workgroup chooses among

struct BFlow {
    unsigned long long *claim;  // [nsys] (seq << 32) | next tile
    int32_t *done;              // [nsys] finished tiles of the current phase
    const int32_t *prio;        // [nsys] systems in claiming order
    const int32_t *sys_t0;      // [nsys+1] tiles of system s: sys_t0[s] .. sys_t0[s+1]
    int32_t *ctl;               // [0] systems not retired, [1] finished phases, [2] stall flag
    int32_t nsys;
};

__device__ __forceinline__ unsigned long long claim_load(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Claims a tile (whole workgroup).  False when every system has retired or
// the stall limit was reached.  sh: 5 + kSpread ints of LDS.
//
// A workgroup that finds nothing to claim waits for the count of finished
// phases to move (every publication of a phase, and every retirement, is
// counted after it is made), then looks again; while it waits it polls that
// one counter, sleeping between polls.
__device__ bool flow_claim(const BFlow &F, int &s_out, uint32_t &seq_out, int &tile_out, int32_t *sh)
{
    uint32_t polls = 0;  // thread 0: polls without a finished phase
    int32_t seen = -1;   // thread 0: finished-phase count of the last look
    for (;;) {
        __syncthreads();  // sh is free
        if (threadIdx.x < kSpread) sh[5 + threadIdx.x] = INT_MAX;
        __syncthreads();
        // candidates: for each residue k of the priority index modulo
        // kSpread, the first system of that residue with a tile left (so the
        // candidates are among the first such systems in priority order); a
        // workgroup takes the one its index selects, so claims spread over
        // several counters
        for (int i = (int)threadIdx.x; i < F.nsys; i += kWG) {
            const int s = F.prio[i];
            const unsigned long long c = claim_load(&F.claim[s]);
            if ((uint32_t)(c >> 32) != kRetired && (uint32_t)c < (uint32_t)(F.sys_t0[s + 1] - F.sys_t0[s])) {
                atomicMin(&sh[5 + (i & (kSpread - 1))], i);
                break;  // this thread's later entries come after i
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t res = 0;  // 0: look again, 1: claimed, 2: leave
            int nc = 0;
#pragma unroll
            for (int k = 0; k < kSpread; ++k) nc += sh[5 + k] != INT_MAX;
            int i = INT_MAX;
            if (nc) {
                int want = (int)(blockIdx.x % (unsigned)nc);
#pragma unroll
                for (int k = 0; k < kSpread; ++k)
                    if (sh[5 + k] != INT_MAX) {
                        if (want == 0) i = sh[5 + k];
                        --want;
                    }
            }
            if (i != INT_MAX) {
                const int s = F.prio[i];
                const unsigned long long old = __hip_atomic_fetch_add(&F.claim[s], 1ull, __ATOMIC_RELAXED,
                                                                      __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t seq = (uint32_t)(old >> 32), tile = (uint32_t)old;
                if (seq != kRetired && tile < (uint32_t)(F.sys_t0[s + 1] - F.sys_t0[s])) {
                    sh[1] = s;
                    sh[2] = (int32_t)seq;
                    sh[3] = (int32_t)tile;
                    res = 1;
                    // the previous phase's vectors, partials and scalars,
                    // written by other workgroups, are visible from here on
                    // (one invalidation of this CU's L1 and the L2 serves the
                    // workgroup's waves, which read after the barrier below)
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
            }
            // nothing claimed: look again at once if a tile was seen (another
            // workgroup was faster) or phases finished since the last look,
            // else wait until they do
            while (res == 0) {
                const int32_t fin = __hip_atomic_load(&F.ctl[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                if (fin != seen) {
                    seen = fin;
                    polls = 0;
                    if (dev::flag_load(&F.ctl[0]) == 0 || dev::flag_load(&F.ctl[2]) != 0) res = 2;
                    break;
                }
                if (i != INT_MAX) break;
                if (++polls > kStallPolls) {
                    dev::flag_store(&F.ctl[2], 1);
                    res = 2;
                } else if ((polls & 255u) == 0 && dev::flag_load(&F.ctl[2]) != 0) {
                    res = 2;
                } else {
                    __builtin_amdgcn_s_sleep(16);
                }
            }
            sh[4] = res;
        }
        __syncthreads();
        const int32_t res = sh[4];
        if (res == 2) return false;
        if (res == 1) {
            s_out = sh[1];
            seq_out = (uint32_t)sh[2];
            tile_out = sh[3];
            return true;
        }
    }
}

// After a tile of phase seq of system s (whole workgroup): the finisher of
// the phase's last tile publishes the next phase or retires the system.
template <int NR>
__device__ void flow_finish(const BFlow &F, const BState &S, int s, uint32_t seq)
{
    // every wave's stores have reached the L2 before the barrier; one
    // device-scope release (an L2 write-back) by thread 0 then covers them all
    __builtin_amdgcn_s_waitcnt(dev::kWaitVmcnt0);
    __syncthreads();
    if (threadIdx.x != 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const int nt = F.sys_t0[s + 1] - F.sys_t0[s];
    const int32_t old = __hip_atomic_fetch_add(&F.done[s], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old != nt - 1) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    bool next = true;
    if (seq & 1u) {  // after a step: the statuses its first tile recorded
        next = false;
        for (int j = 0; j < NR; ++j) next = next || dev::flag_load(&S.status[s * NR + j]) == BS_RUNNING;
    }
    __hip_atomic_store(&F.done[s], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long word = (unsigned long long)(next ? seq + 1u : kRetired) << 32;
    __hip_atomic_store(&F.claim[s], word, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (!next) __hip_atomic_fetch_add(&F.ctl[0], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // counted after the publication (and retirement) it announces
    __hip_atomic_fetch_add(&F.ctl[1], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NR, int U, bool ALL_STAGED>
__global__ __launch_bounds__(kWG) void k_bflow(BMat M, BTiles T, BState S, BFlow F, double *__restrict__ r,
                                               double *__restrict__ q, double *__restrict__ x,
                                               double *__restrict__ p0, double *__restrict__ p1,
                                               double *__restrict__ part_a, double *__restrict__ part_b)
{
    __shared__ double ws[kWaves * NR];
    __shared__ int32_t sh_st[NR];
    __shared__ int32_t sh[5 + kSpread];
    __shared__ __align__(16) double ring[ring_rows<NR>() * NR];
    int s, tile;
    uint32_t seq;
    while (flow_claim(F, s, seq, tile, sh)) {
        const int t = F.sys_t0[s] + tile;
        const int slot = (int)((seq >> 1) & 1u);
        if ((seq & 1u) == 0)
            update_tile<NR>(M, T, S, t, r, q, part_b, part_a, slot, ws, sh_st);
        else
            spmv_tile<NR, U, M_STEP, ALL_STAGED>(M, T, S, t, slot ? p0 : p1, r, slot ? p1 : p0, q, x, part_a,
                                                 part_b, slot, ws, sh_st, ring);
        flow_finish<NR>(F, S, s, seq);
    }
}

// Phase 0 for every system with a running pair, retired otherwise; counters.
template <int NR>
__global__ __launch_bounds__(kWG) void k_bflow_init(BState S, BFlow F)
{
    const int s = blockIdx.x * kWG + threadIdx.x;
    if (s >= F.nsys) return;
    bool run = false;
    for (int j = 0; j < NR; ++j) run = run || dev::flag_load(&S.status[s * NR + j]) == BS_RUNNING;
    F.claim[s] = run ? 0ull : (unsigned long long)kRetired << 32;
    F.done[s] = 0;
    if (run) atomicAdd(&F.ctl[0], 1);
}

__global__ __launch_bounds__(64) void k_bflow_reset(int32_t *ctl)
{
    if (threadIdx.x < 3) ctl[threadIdx.x] = 0;
}

// ---- fresh residual r = b - q (q = A x), partials (r, r) [and (b, b)] ------------

template <int NR, bool FIRST>
__global__ __launch_bounds__(kWG) void k_bresid(BMat M, BTiles T, const double *__restrict__ b,
                                                const double *__restrict__ q, double *__restrict__ r,
                                                double *__restrict__ part_r, double *__restrict__ part_bb,
                                                const int32_t *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    __shared__ double ws[kWaves * NR];
    const Share sh = list_share(*T.nlist);
    for (int i = sh.i; i < sh.end; i += sh.step) {
        const int t = T.list[i];
        const int g0 = T.tile_g0[t], g1 = T.tile_g0[t + 1];
        for (int g = g0; g < g1; ++g) {
            const int e0 = M.crow[T.gran_c0[g]] * NR, e1 = M.crow[T.gran_c0[g + 1]] * NR;
            double arr = 0.0, abb = 0.0;
            for (int e = e0 + (int)threadIdx.x; e < e1; e += kWG) {
                const double be = b[e];
                const double re = be - q[e];
                r[e] = re;
                arr = arr + re * re;
                if (FIRST) abb = abb + be * be;
            }
            granule_store_strided<NR>(arr, part_r, g, ws);
            if (FIRST) granule_store_strided<NR>(abb, part_bb, g, ws);
        }
    }
}

// One workgroup per system: (r, r) [and (b, b)] of each pair, stopping test,
// slot 0 of the state, running count.  Pairs that broke down or have b = 0
// stay stopped; the others are re-tested on the fresh residual (restarting CG
// from it when still above the tolerance and below the iteration limit).
template <int NR>
__global__ __launch_bounds__(kWG) void k_bfinish(BTiles T, BState S, const double *__restrict__ part_r,
                                                 const double *__restrict__ part_bb, double tol, int first,
                                                 const int32_t *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    __shared__ double ws[kWaves * NR];
    const int s = blockIdx.x;
    const int g0 = T.sys_g0[s], g1 = T.sys_g0[s + 1];
    double rr[NR], bb[NR];
    sys_sum<NR>(part_r, g0, g1, ws, rr);
    if (first) sys_sum<NR>(part_bb, g0, g1, ws, bb);
    if (threadIdx.x != 0) return;
    const int kmax = *S.kmax;
    for (int j = 0; j < NR; ++j) {
        const int pr = s * NR + j;
        if (first) {
            S.bb[pr] = bb[j];
            if (!isfinite(bb[j])) {
                dev::flag_store(&S.status[pr], BS_BREAKDOWN);
                continue;
            }
            if (bb[j] == 0.0) {
                S.rr_last[pr] = 0.0;
                dev::flag_store(&S.status[pr], BS_ZERO_RHS);
                continue;
            }
            S.stop[pr] = tol * sqrt(bb[j]);
        }
        const int32_t st = dev::flag_load(&S.status[pr]);
        if (st == BS_BREAKDOWN || st == BS_ZERO_RHS) continue;
        if (!isfinite(rr[j])) {
            dev::flag_store(&S.status[pr], BS_BREAKDOWN);
            continue;
        }
        const int k = S.it_last[pr];
        S.rr0[pr] = rr[j];
        S.it0[pr] = k;
        S.rr_last[pr] = rr[j];
        int32_t nst;
        if (sqrt(rr[j]) <= S.stop[pr])
            nst = BS_CONVERGED;
        else if (k >= kmax)
            nst = BS_MAXIT;
        else
            nst = BS_RUNNING;
        if (nst == BS_RUNNING) {
            atomicAdd(S.nrun, 1);
            if (!first) S.restarts[pr] = S.restarts[pr] + 1;
        }
        dev::flag_store(&S.status[pr], nst);
    }
}

// Tile list of the systems with a running pair (system order), one workgroup.
template <int NR>
__global__ __launch_bounds__(kWG) void k_bcompact(int32_t nsys, const int32_t *__restrict__ sys_t0,
                                                  const int32_t *__restrict__ status, int32_t *__restrict__ list,
                                                  int32_t *__restrict__ nlist)
{
    __shared__ int32_t scan[kWG];
    __shared__ int32_t base;
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (int s0 = 0; s0 < nsys; s0 += kWG) {
        const int s = s0 + (int)threadIdx.x;
        int nt = 0;
        if (s < nsys) {
            bool any = false;
            for (int j = 0; j < NR; ++j) any = any || dev::flag_load(&status[s * NR + j]) == BS_RUNNING;
            if (any) nt = sys_t0[s + 1] - sys_t0[s];
        }
        scan[threadIdx.x] = nt;
        __syncthreads();
        for (int o = 1; o < kWG; o <<= 1) {
            const int v = threadIdx.x >= (unsigned)o ? scan[threadIdx.x - o] : 0;
            __syncthreads();
            scan[threadIdx.x] += v;
            __syncthreads();
        }
        const int off = base + scan[threadIdx.x] - nt;
        for (int k = 0; k < nt; ++k) list[off + k] = sys_t0[s] + k;
        __syncthreads();
        if (threadIdx.x == kWG - 1) base = base + scan[kWG - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *nlist = base;
}

__global__ __launch_bounds__(kWG) void k_binit(BState S, int32_t npairs, int32_t *kmax_dev, int32_t kmax)
{
    const int i = blockIdx.x * kWG + threadIdx.x;
    if (i == 0) {
        *kmax_dev = kmax;
        *S.nrun = 0;
    }
    if (i >= npairs) return;
    S.it_last[i] = 0;
    S.restarts[i] = 0;
    S.rr_last[i] = 0.0;
    S.bb[i] = 0.0;
    S.stop[i] = 0.0;
    dev::flag_store(&S.status[i], BS_RUNNING);
}

__global__ __launch_bounds__(kWG) void k_bzero_count(int32_t *nrun, const int32_t *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    if (threadIdx.x == 0 && blockIdx.x == 0) *nrun = 0;
}

// The gate of a residual check inside the whole-solve graph: 1 when no pair
// runs any more (the check is due), else 0 (the kernels it gates return at
// once and the pairs go on iterating).
__global__ void k_bgate(const int32_t *__restrict__ nrun, int32_t *__restrict__ gate)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *gate = *nrun == 0 ? 1 : 0;
}

// x_out = x, zero for pairs with b = 0 (every tile of the full list).
template <int NR>
__global__ __launch_bounds__(kWG) void k_bstore(BMat M, BTiles T, const int32_t *__restrict__ status,
                                                const double *__restrict__ x, double *__restrict__ xo)
{
    __shared__ int32_t sh_st[NR];
    const int jt = threadIdx.x % NR;
    const Share sh = list_share(*T.nlist);
    for (int i = sh.i; i < sh.end; i += sh.step) {
        const int t = T.list[i];
        const int s = T.tile_sys[t];
        __syncthreads();
        if (threadIdx.x < NR) sh_st[threadIdx.x] = dev::flag_load(&status[s * NR + threadIdx.x]);
        __syncthreads();
        const bool zero = sh_st[jt] == BS_ZERO_RHS;
        const int e0 = M.crow[T.gran_c0[T.tile_g0[t]]] * NR, e1 = M.crow[T.gran_c0[T.tile_g0[t + 1]]] * NR;
        for (int e = e0 + (int)threadIdx.x; e < e1; e += kWG) xo[e] = zero ? 0.0 : x[e];
    }
}

// ---------------------------------------------------------------------------
// host side

struct Tiles {
    std::vector<int32_t> tile_sys, tile_g0, sys_t0;
};

// Granules per tile of a system whose entries lie within h rows of the
// diagonal, for the per-system choice (tile_granules 0): the staged SpMV
// reads the 2h rows around a tile twice, so the tile takes the fewest
// granules (1, 2, 4, 8) that keep those rows at most a quarter of its own.
int reach_granules(int32_t h)
{
    int k = 1;
    while (k < 8 && 2 * (int64_t)h * 4 > (int64_t)k * kGranRows) k *= 2;
    return k;
}

// Tiles of k granules (k = 0: reach_granules of each system's halo h),
// never crossing a system boundary.
Tiles make_tiles(const std::vector<int32_t> &sys_g0, int k0, const std::vector<int32_t> &h)
{
    Tiles T;
    const int nsys = (int)sys_g0.size() - 1;
    T.sys_t0.assign(nsys + 1, 0);
    T.tile_g0.push_back(0);
    for (int s = 0; s < nsys; ++s) {
        const int k = k0 > 0 ? k0 : reach_granules(h[s]);
        T.sys_t0[s] = (int32_t)T.tile_sys.size();
        for (int g = sys_g0[s]; g < sys_g0[s + 1]; g += k) {
            T.tile_sys.push_back(s);
            T.tile_g0.push_back(std::min(g + k, sys_g0[s + 1]));
        }
    }
    T.sys_t0[nsys] = (int32_t)T.tile_sys.size();
    return T;
}

bool tuning_valid(const ss_batch_tuning &t)
{
    const int k = t.tile_granules;
    if (k != 0 && k != 1 && k != 2 && k != 4 && k != 8) return false;
    if (t.grid != 0 && (t.grid < 8 || t.grid > kGridLimit || t.grid % 8 != 0)) return false;
    if (t.unroll != 4 && t.unroll != 5 && t.unroll != 8) return false;
    if (t.check_every < 2 || t.check_every > 1024 || t.check_every % 2 != 0) return false;
    if (t.schedule != SS_BATCH_CHUNKED && t.schedule != SS_BATCH_PERSISTENT && t.schedule != SS_BATCH_GRAPH)
        return false;
    return true;
}

std::mutex g_tune_mu;
std::map<std::string, ss_batch_tuning> g_tune_cache;

}  // namespace

struct ss_batch {
    int32_t nsys = 0, nrhs = 0, device = 0;
    int64_t nrows = 0, nnz = 0, stored = 0;
    int32_t nchunks = 0, ngran = 0, ntiles = 0;
    int32_t max_halo = 0;  // largest |column - row| over all systems
    std::string key;  // structure signature for the tuning cache
    hipStream_t stream = nullptr, cap = nullptr;
    DeviceMem mem;
    std::vector<int32_t> sys_g0_h;
    std::vector<int32_t> sys_h_h;  // largest |column - row| of each system (host)
    int32_t *sys_h = nullptr;
    // matrix and granules
    int32_t *col = nullptr, *cptr = nullptr, *crow = nullptr, *gran_c0 = nullptr, *sys_g0 = nullptr;
    double *val = nullptr;
    uint8_t *clen = nullptr, *rlen = nullptr;
    // tiles of the current tuning (allocated for the largest count)
    int32_t *tile_sys = nullptr, *tile_g0 = nullptr, *sys_t0 = nullptr;
    int32_t *list_full = nullptr, *list_act = nullptr, *n_full = nullptr, *n_act = nullptr;
    // vectors [nrows][nrhs]
    double *x = nullptr, *r = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
    double *part_a = nullptr, *part_b = nullptr, *part_c = nullptr;
    // pair state
    double *rr0 = nullptr, *rr1 = nullptr, *bb = nullptr, *stop = nullptr, *rr_last = nullptr;
    int32_t *it0 = nullptr, *it1 = nullptr, *it_last = nullptr, *status = nullptr, *restarts = nullptr;
    int32_t *nrun = nullptr, *kmax = nullptr;
    double *alpha = nullptr;
    // one-launch schedule
    unsigned long long *claim = nullptr;
    int32_t *done = nullptr, *prio = nullptr, *ctl = nullptr;
    int32_t *pinned = nullptr;  // host: polled running counts
    hipEvent_t ev[2] = {nullptr, nullptr};
    ss_batch_tuning tun{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t graph_pairs = 0;
    bool graph_ok = false;
    // SS_BATCH_GRAPH: the whole-solve graph (lchunks chunks of lpairs
    // pairs, a residual check, lchunks2 chunks, a residual check), the
    // chunks the longest solve so far took before its first residual check
    // and after it, the gate of the checks and the right-hand sides the
    // graph's checks read (copied in by every solve)
    hipGraph_t lgraph = nullptr;
    hipGraphExec_t lexec = nullptr;
    int32_t lchunks = 0, lchunks2 = 0, lpairs = 0, hint = 0, hint2 = 0;
    int32_t *gate = nullptr;
    double *bcopy = nullptr;
    const int32_t *cur_gate = nullptr;  // gate passed to the kernels being enqueued
    // host-side launches of the last solve (ss_batch_launches)
    int32_t n_graph = 0, n_chunk = 0, n_kernel = 0;

    BMat bmat() const { return BMat{col, val, cptr, crow, clen, rlen}; }
    BTiles tiles(bool full) const
    {
        return BTiles{full ? list_full : list_act, full ? n_full : n_act, tile_sys, tile_g0, gran_c0, sys_g0, sys_h};
    }
    BState state() const
    {
        return BState{rr0, rr1, it0, it1, bb, stop, rr_last, it_last, status, restarts, nrun, kmax, alpha};
    }
    int grid() const { return tun.grid ? tun.grid : std::max(8, (ntiles + 7) / 8 * 8); }
    BFlow flow() const { return BFlow{claim, done, prio, sys_t0, ctl, nsys}; }
};

namespace {

template <typename T>
int alloc_dev(ss_batch *b, T **dst, size_t count)
{
    *dst = (T *)b->mem.get(sizeof(T) * std::max<size_t>(count, 1));
    return *dst ? SS_OK : fail(SS_ENOMEM, "device allocation failed");
}

template <typename T>
int upload(ss_batch *b, T **dst, const std::vector<T> &src)
{
    int rc = alloc_dev(b, dst, src.size());
    if (rc != SS_OK) return rc;
    if (!src.empty()) SS_HIP(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return SS_OK;
}

void destroy_long_graph(ss_batch *b)
{
    if (b->lexec) (void)hipGraphExecDestroy(b->lexec);
    if (b->lgraph) (void)hipGraphDestroy(b->lgraph);
    b->lexec = nullptr;
    b->lgraph = nullptr;
    b->lchunks = 0;
}

// Both graphs (they hold the kernels' launch shape and tiles).
void destroy_graph(ss_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_ok = false;
    destroy_long_graph(b);
}

// Uploads the tiles of tuning t (the identity list is the full list).
int apply_tuning(ss_batch *b, const ss_batch_tuning &t)
{
    Tiles T = make_tiles(b->sys_g0_h, t.tile_granules, b->sys_h_h);
    const int nt = (int)T.tile_sys.size();
    std::vector<int32_t> ident(nt);
    for (int i = 0; i < nt; ++i) ident[i] = i;
    SS_HIP(hipStreamSynchronize(b->stream));
    SS_HIP(hipMemcpy(b->tile_sys, T.tile_sys.data(), sizeof(int32_t) * std::max(nt, 1), hipMemcpyHostToDevice));
    SS_HIP(hipMemcpy(b->tile_g0, T.tile_g0.data(), sizeof(int32_t) * (nt + 1), hipMemcpyHostToDevice));
    SS_HIP(hipMemcpy(b->sys_t0, T.sys_t0.data(), sizeof(int32_t) * (b->nsys + 1), hipMemcpyHostToDevice));
    SS_HIP(hipMemcpy(b->list_full, ident.data(), sizeof(int32_t) * std::max(nt, 1), hipMemcpyHostToDevice));
    SS_HIP(hipMemcpy(b->n_full, &nt, sizeof(int32_t), hipMemcpyHostToDevice));
    SS_HIP(hipMemcpy(b->n_act, &nt, sizeof(int32_t), hipMemcpyHostToDevice));
    b->ntiles = nt;
    b->tun = t;
    destroy_graph(b);
    return SS_OK;
}

// Largest |column - row| the staged SpMV handles for NR right-hand sides.
int staged_halo(int nr) { return (kRingBytes / (8 * nr) - kGranRows) / 2; }

template <int NR, int U, int MODE>
void spmv_t(ss_batch *b, hipStream_t st, bool full, const double *pin, const double *r, double *pout, double *q,
            int slot)
{
    if (b->max_halo <= staged_halo(NR))
        hipLaunchKernelGGL((k_bspmv<NR, U, MODE, true>), dim3(b->grid()), dim3(kWG), 0, st, b->bmat(),
                           b->tiles(full), b->state(), pin, r, pout, q, b->x, b->part_a, b->part_b, slot,
                           b->cur_gate);
    else
        hipLaunchKernelGGL((k_bspmv<NR, U, MODE, false>), dim3(b->grid()), dim3(kWG), 0, st, b->bmat(),
                           b->tiles(full), b->state(), pin, r, pout, q, b->x, b->part_a, b->part_b, slot,
                           b->cur_gate);
}

template <int NR, int MODE>
void spmv_u(ss_batch *b, hipStream_t st, bool full, const double *pin, const double *r, double *pout, double *q,
            int slot)
{
    if (b->tun.unroll == 4)
        spmv_t<NR, 4, MODE>(b, st, full, pin, r, pout, q, slot);
    else if (b->tun.unroll == 5)
        spmv_t<NR, 5, MODE>(b, st, full, pin, r, pout, q, slot);
    else
        spmv_t<NR, 8, MODE>(b, st, full, pin, r, pout, q, slot);
}

template <int MODE>
void spmv(ss_batch *b, hipStream_t st, bool full, const double *pin, const double *r, double *pout, double *q,
          int slot)
{
    switch (b->nrhs) {
    case 1: spmv_u<1, MODE>(b, st, full, pin, r, pout, q, slot); break;
    case 2: spmv_u<2, MODE>(b, st, full, pin, r, pout, q, slot); break;
    default: spmv_u<4, MODE>(b, st, full, pin, r, pout, q, slot); break;
    }
}

template <int NR>
void update_t(ss_batch *b, hipStream_t st, int slot)
{
    hipLaunchKernelGGL(k_bupdate<NR>, dim3(b->grid()), dim3(kWG), 0, st, b->bmat(), b->tiles(false), b->state(),
                       b->r, b->q, b->part_b, b->part_a, slot);
}

void update(ss_batch *b, hipStream_t st, int slot)
{
    switch (b->nrhs) {
    case 1: update_t<1>(b, st, slot); break;
    case 2: update_t<2>(b, st, slot); break;
    default: update_t<4>(b, st, slot); break;
    }
}

void compact(ss_batch *b, hipStream_t st)
{
    switch (b->nrhs) {
    case 1: hipLaunchKernelGGL(k_bcompact<1>, dim3(1), dim3(kWG), 0, st, b->nsys, b->sys_t0, b->status, b->list_act, b->n_act); break;
    case 2: hipLaunchKernelGGL(k_bcompact<2>, dim3(1), dim3(kWG), 0, st, b->nsys, b->sys_t0, b->status, b->list_act, b->n_act); break;
    default: hipLaunchKernelGGL(k_bcompact<4>, dim3(1), dim3(kWG), 0, st, b->nsys, b->sys_t0, b->status, b->list_act, b->n_act); break;
    }
}

template <int NR>
void residual_t(ss_batch *b, hipStream_t st, const double *b_dev, bool first)
{
    if (first)
        hipLaunchKernelGGL((k_bresid<NR, true>), dim3(b->grid()), dim3(kWG), 0, st, b->bmat(), b->tiles(true),
                           b_dev, b->q, b->r, b->part_b, b->part_c, b->cur_gate);
    else
        hipLaunchKernelGGL((k_bresid<NR, false>), dim3(b->grid()), dim3(kWG), 0, st, b->bmat(), b->tiles(true),
                           b_dev, b->q, b->r, b->part_b, b->part_c, b->cur_gate);
}

template <int NR>
void finish_t(ss_batch *b, hipStream_t st, double tol, bool first)
{
    hipLaunchKernelGGL(k_bfinish<NR>, dim3(b->nsys), dim3(kWG), 0, st, b->tiles(true), b->state(), b->part_b,
                       b->part_c, tol, first ? 1 : 0, b->cur_gate);
}

// r = b - A x for every pair, stopping tests; returns the running count.
// The residual check: q = A x, r = b - q, (r, r) [(b, b)], the stopping
// test of every pair, the running count; with b->cur_gate set, gated.
void enqueue_residual(ss_batch *b, hipStream_t st, const double *b_dev, double tol, bool first)
{
    spmv<M_PLAIN>(b, st, true, b->x, nullptr, nullptr, b->q, 0);
    hipLaunchKernelGGL(k_bzero_count, dim3(1), dim3(kWG), 0, st, b->nrun, b->cur_gate);
    switch (b->nrhs) {
    case 1: residual_t<1>(b, st, b_dev, first); finish_t<1>(b, st, tol, first); break;
    case 2: residual_t<2>(b, st, b_dev, first); finish_t<2>(b, st, tol, first); break;
    default: residual_t<4>(b, st, b_dev, first); finish_t<4>(b, st, tol, first); break;
    }
}

int residual_phase(ss_batch *b, const double *b_dev, double tol, bool first, int32_t *nrun)
{
    enqueue_residual(b, b->stream, b_dev, tol, first);
    SS_HIP(hipGetLastError());
    SS_HIP(hipMemcpyAsync(&b->pinned[0], b->nrun, sizeof(int32_t), hipMemcpyDeviceToHost, b->stream));
    SS_HIP(hipStreamSynchronize(b->stream));
    *nrun = b->pinned[0];
    return SS_OK;
}

// Pair j of a chunk: update of iteration k, step of iteration k+1; p ping-pong
// and scalar slot alternate, chunks are even so each starts with p in p1.
void enqueue_pair(ss_batch *b, hipStream_t st, int j)
{
    const int slot = j & 1;
    double *pcur = slot ? b->p0 : b->p1;
    double *pnext = slot ? b->p1 : b->p0;
    update(b, st, slot);
    spmv<M_STEP>(b, st, false, pcur, b->r, pnext, b->q, slot);
}

int ensure_graph(ss_batch *b, int32_t pairs)
{
    if (b->graph_ok && b->graph_pairs == pairs) return SS_OK;
    destroy_graph(b);
    b->hint = b->hint2 = 0;  // counted in chunks of another length
    SS_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    for (int32_t k = 0; k < pairs; ++k) enqueue_pair(b, b->cap, k);
    compact(b, b->cap);
    hipGraph_t g = nullptr;
    SS_HIP(hipStreamEndCapture(b->cap, &g));
    b->graph = g;
    SS_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    b->graph_pairs = pairs;
    b->graph_ok = true;
    return SS_OK;
}

// The residual check of the whole-solve graph, and the restart it may
// start, as the host runs them between chunk loops: gated on no pair running
// any more (else every kernel of it returns at once and the chunks that
// follow go on with the running pairs), reading the solve's right-hand
// sides from the copy every solve makes.
void enqueue_check(ss_batch *b, hipStream_t st)
{
    hipLaunchKernelGGL(k_bgate, dim3(1), dim3(64), 0, st, b->nrun, b->gate);
    b->cur_gate = b->gate;
    enqueue_residual(b, st, b->bcopy, 0.0, false);
    b->cur_gate = nullptr;
    compact(b, st);
    b->cur_gate = b->gate;
    spmv<M_FIRST>(b, st, false, b->r, b->r, b->p1, b->q, 0);
    b->cur_gate = nullptr;
}

// The whole-solve graph: `chunks` times a chunk of `pairs` pairs and the
// rebuild of the running list, as the chunk graph runs them one launch at a
// time, the residual check, then `chunks2` more chunks and a check when the
// longest solve so far restarted pairs.
int ensure_long_graph(ss_batch *b, int32_t pairs, int32_t chunks, int32_t chunks2)
{
    if (b->lexec && b->lchunks == chunks && b->lchunks2 == chunks2 && b->lpairs == pairs) return SS_OK;
    destroy_long_graph(b);
    int rc;
    if (!b->gate && (rc = alloc_dev(b, &b->gate, 1)) != SS_OK) return rc;
    if (!b->bcopy && (rc = alloc_dev(b, &b->bcopy, (size_t)b->nrows * b->nrhs)) != SS_OK) return rc;
    SS_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    for (int32_t seg = 0; seg < (chunks2 > 0 ? 2 : 1); ++seg) {
        for (int32_t c = 0; c < (seg == 0 ? chunks : chunks2); ++c) {
            for (int32_t k = 0; k < pairs; ++k) enqueue_pair(b, b->cap, k);
            compact(b, b->cap);
        }
        enqueue_check(b, b->cap);
    }
    hipGraph_t g = nullptr;
    SS_HIP(hipStreamEndCapture(b->cap, &g));
    b->lgraph = g;
    SS_HIP(hipGraphInstantiate(&b->lexec, g, nullptr, nullptr, 0));
    b->lchunks = chunks;
    b->lchunks2 = chunks2;
    b->lpairs = pairs;
    return SS_OK;
}

template <int NR, int U, bool ALL_STAGED>
int flow_launch(ss_batch *b)
{
    auto kern = k_bflow<NR, U, ALL_STAGED>;
    int grid = b->tun.grid;
    if (grid == 0) {
        // every workgroup resident at once (not needed for progress: a
        // workgroup never waits for another particular one)
        int per_cu = 0, cus = 0;
        SS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kWG, 0));
        SS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
        grid = std::max(8, std::min(kGridLimit, std::max(1, per_cu) * std::max(1, cus)) / 8 * 8);
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kWG), 0, b->stream, b->bmat(), b->tiles(true), b->state(), b->flow(),
                       b->r, b->q, b->x, b->p0, b->p1, b->part_a, b->part_b);
    return SS_OK;
}

template <int NR, int U>
int flow_launch_s(ss_batch *b)
{
    return b->max_halo <= staged_halo(NR) ? flow_launch<NR, U, true>(b) : flow_launch<NR, U, false>(b);
}

template <int NR>
int flow_t(ss_batch *b)
{
    hipLaunchKernelGGL(k_bflow_reset, dim3(1), dim3(64), 0, b->stream, b->ctl);
    hipLaunchKernelGGL(k_bflow_init<NR>, dim3((b->nsys + kWG - 1) / kWG), dim3(kWG), 0, b->stream, b->state(),
                       b->flow());
    switch (b->tun.unroll) {
    case 4: return flow_launch_s<NR, 4>(b);
    case 5: return flow_launch_s<NR, 5>(b);
    default: return flow_launch_s<NR, 8>(b);
    }
}

// Every iteration of every running pair in one launch (no host polling).
int iterate_flow(ss_batch *b)
{
    int rc;
    switch (b->nrhs) {
    case 1: rc = flow_t<1>(b); break;
    case 2: rc = flow_t<2>(b); break;
    default: rc = flow_t<4>(b); break;
    }
    if (rc != SS_OK) return rc;
    SS_HIP(hipGetLastError());
    SS_HIP(hipMemcpyAsync(&b->pinned[2], b->ctl + 2, sizeof(int32_t), hipMemcpyDeviceToHost, b->stream));
    SS_HIP(hipStreamSynchronize(b->stream));
    if (b->pinned[2] != 0) return fail(SS_EDEVICE, "batched solve: no phase finished within the stall limit");
    return SS_OK;
}

// Iterates until no pair is running; chunks are queued one ahead of the
// poll.  *chunks: the chunks it took.
int iterate(ss_batch *b, int32_t *chunks)
{
    *chunks = 0;
    if (b->tun.schedule == SS_BATCH_PERSISTENT) {
        ++b->n_kernel;
        return iterate_flow(b);
    }
    const int32_t chunk = b->tun.check_every;
    int rc = ensure_graph(b, chunk);
    if (rc != SS_OK) return rc;
    int32_t done = 0;  // chunks run
    int slot = 0;
    SS_HIP(hipGraphLaunch(b->exec, b->stream));
    ++b->n_chunk;
    SS_HIP(hipMemcpyAsync(&b->pinned[slot], b->nrun, sizeof(int32_t), hipMemcpyDeviceToHost, b->stream));
    SS_HIP(hipEventRecord(b->ev[slot], b->stream));
    for (;;) {
        const int nxt = slot ^ 1;
        SS_HIP(hipGraphLaunch(b->exec, b->stream));
        ++b->n_chunk;
        SS_HIP(hipMemcpyAsync(&b->pinned[nxt], b->nrun, sizeof(int32_t), hipMemcpyDeviceToHost, b->stream));
        SS_HIP(hipEventRecord(b->ev[nxt], b->stream));
        SS_HIP(hipEventSynchronize(b->ev[slot]));
        ++done;
        if (b->pinned[slot] == 0) {
            SS_HIP(hipEventSynchronize(b->ev[nxt]));
            *chunks = done;
            return SS_OK;
        }
        slot = nxt;
    }
}

// Fresh start of every pair from x (internal) for b_dev: init, residual,
// list of running systems, first step.  Returns the running count.
int start_pairs(ss_batch *b, const double *b_dev, double tol, int32_t maxit, int32_t *nrun)
{
    const int32_t np = b->nsys * b->nrhs;
    hipLaunchKernelGGL(k_binit, dim3((np + kWG - 1) / kWG), dim3(kWG), 0, b->stream, b->state(), np, b->kmax, maxit);
    int rc = residual_phase(b, b_dev, tol, true, nrun);
    if (rc != SS_OK || *nrun == 0) return rc;
    compact(b, b->stream);
    spmv<M_FIRST>(b, b->stream, false, b->r, b->r, b->p1, b->q, 0);
    SS_HIP(hipGetLastError());
    return SS_OK;
}

std::string structure_key(const std::vector<int32_t> &rows, const std::vector<int64_t> &nnz, int nrhs, int device)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    for (size_t s = 0; s < rows.size(); ++s) {
        mix((uint64_t)rows[s]);
        mix((uint64_t)nnz[s]);
    }
    return std::to_string(device) + ":" + std::to_string(nrhs) + ":" + std::to_string(rows.size()) + ":" +
           std::to_string(h);
}

}  // namespace

extern "C" {

void ss_batch_destroy(ss_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    destroy_graph(b);
    for (auto &e : b->ev)
        if (e) (void)hipEventDestroy(e);
    if (b->pinned) (void)hipHostFree(b->pinned);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    b->mem.clear();
    delete b;
}

int ss_batch_setup(int32_t nsys, const ss_csr *systems, int32_t nrhs, const ss_opts *o, void *hip_stream,
                   ss_batch **out)
{
    if (!out) return fail(SS_EINVAL, "out is NULL");
    *out = nullptr;
    if (nsys <= 0 || !systems) return fail(SS_EINVAL, "need nsys > 0 systems");
    if (nrhs != 1 && nrhs != 2 && nrhs != 4)
        return fail(SS_EUNSUPPORTED, "nrhs must be 1, 2 or 4 (pad with zero right-hand sides)");
    ss_opts opts;
    ss_opts_default(&opts);
    if (o) opts = *o;
    if ((opts.alloc == nullptr) != (opts.free == nullptr)) return fail(SS_EINVAL, "alloc and free go together");

    // host structure: SELL-64 chunks per system, granules of 8 chunks
    std::vector<int32_t> rows_h(nsys), halo(nsys, 0);
    std::vector<int64_t> nnz_h(nsys);
    int64_t nrows = 0, nnz = 0, stored = 0, nchunks = 0;
    for (int s = 0; s < nsys; ++s) {
        const ss_csr *A = &systems[s];
        int rc = validate_csr(A, true);
        if (rc != SS_OK) return fail(rc, "system " + std::to_string(s) + ": " + ss_last_error());
        for (int i = 0; i < A->n; ++i) {
            if (A->rowptr[i + 1] - A->rowptr[i] > kMaxRowLen)
                return fail(SS_EUNSUPPORTED, "system " + std::to_string(s) + ": a row holds more than 255 entries");
            for (int k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
                halo[s] = std::max(halo[s], std::abs(A->colidx[k] - i));
        }
        rows_h[s] = A->n;
        nnz_h[s] = A->nnz;
        nrows += A->n;
        nnz += A->nnz;
        nchunks += (A->n + kChunk - 1) / kChunk;
    }
    if (nrows * nrhs >= (int64_t)1 << 31) return fail(SS_EUNSUPPORTED, "batch too large (rows * nrhs >= 2^31)");

    std::vector<int32_t> cptr, crow, gran_c0, sys_g0, col;
    std::vector<uint8_t> clen, rlen;
    std::vector<double> val;
    try {
        cptr.reserve(nchunks);
        crow.reserve(nchunks + 1);
        clen.reserve(nchunks);
        rlen.reserve(nrows);
        sys_g0.push_back(0);
        int64_t row0 = 0;
        for (int s = 0; s < nsys; ++s) {
            const ss_csr *A = &systems[s];
            for (int c0 = 0; c0 < A->n; c0 += kChunk) {
                const int c1 = std::min(c0 + kChunk, A->n);
                int L = 0;
                for (int i = c0; i < c1; ++i) L = std::max(L, A->rowptr[i + 1] - A->rowptr[i]);
                if (c0 % kGranRows == 0) gran_c0.push_back((int32_t)crow.size());
                cptr.push_back((int32_t)stored);
                crow.push_back((int32_t)(row0 + c0));
                clen.push_back((uint8_t)L);
                const size_t at = col.size();
                col.resize(at + (size_t)L * kChunk);
                val.resize(at + (size_t)L * kChunk, 0.0);
                for (int l = 0; l < kChunk; ++l) {
                    const int i = c0 + l;
                    const int32_t pad = (int32_t)(row0 + c0);  // padding reads a valid row, value 0
                    const int a = i < c1 ? A->rowptr[i] : 0, e = i < c1 ? A->rowptr[i + 1] : 0;
                    for (int j = 0; j < L; ++j) {
                        const size_t k = at + (size_t)j * kChunk + l;
                        if (a + j < e) {
                            col[k] = (int32_t)(row0 + A->colidx[a + j]);
                            val[k] = A->val[a + j];
                        } else {
                            col[k] = pad;
                        }
                    }
                }
                for (int i = c0; i < c1; ++i) rlen.push_back((uint8_t)(A->rowptr[i + 1] - A->rowptr[i]));
                stored += (int64_t)L * kChunk;
                if (stored >= (int64_t)1 << 31) return fail(SS_EUNSUPPORTED, "batch too large (stored entries)");
            }
            sys_g0.push_back((int32_t)gran_c0.size());
            row0 += A->n;
        }
        crow.push_back((int32_t)nrows);
        gran_c0.push_back((int32_t)cptr.size());
    } catch (const std::bad_alloc &) {
        return fail(SS_ENOMEM, "host allocation failed");
    }

    ss_batch *b = new (std::nothrow) ss_batch;
    if (!b) return fail(SS_ENOMEM, "host allocation failed");
    auto bail = [&](int code) {
        ss_batch_destroy(b);
        return code;
    };
    b->mem.alloc = opts.alloc;
    b->mem.release = opts.free;
    b->mem.ctx = opts.alloc_ctx;
    b->stream = (hipStream_t)hip_stream;
    b->nsys = nsys;
    b->nrhs = nrhs;
    b->nrows = nrows;
    b->nnz = nnz;
    b->stored = stored;
    b->nchunks = (int32_t)cptr.size();
    b->ngran = (int32_t)gran_c0.size() - 1;
    b->sys_g0_h = sys_g0;
    b->sys_h_h = halo;
    b->max_halo = *std::max_element(halo.begin(), halo.end());
    if (hipGetDevice(&b->device) != hipSuccess) return bail(fail(SS_EDEVICE, "no HIP device"));
    b->key = structure_key(rows_h, nnz_h, nrhs, b->device);
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(SS_EDEVICE, "stream creation failed"));
    for (auto &e : b->ev)
        if (hipEventCreate(&e) != hipSuccess) return bail(fail(SS_EDEVICE, "event creation failed"));
    if (hipHostMalloc((void **)&b->pinned, 4 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess)
        return bail(fail(SS_ENOMEM, "pinned host allocation failed"));

    const size_t nv = (size_t)nrows * nrhs, np = (size_t)nsys * nrhs, ngp = (size_t)b->ngran * nrhs;
    int rc = SS_OK;
    if ((rc = upload(b, &b->col, col)) || (rc = upload(b, &b->val, val)) || (rc = upload(b, &b->cptr, cptr)) ||
        (rc = upload(b, &b->crow, crow)) || (rc = upload(b, &b->clen, clen)) || (rc = upload(b, &b->rlen, rlen)) ||
        (rc = upload(b, &b->gran_c0, gran_c0)) || (rc = upload(b, &b->sys_g0, sys_g0)) ||
        (rc = upload(b, &b->sys_h, halo)) ||
        (rc = alloc_dev(b, &b->tile_sys, (size_t)b->ngran)) || (rc = alloc_dev(b, &b->tile_g0, (size_t)b->ngran + 1)) ||
        (rc = alloc_dev(b, &b->sys_t0, (size_t)nsys + 1)) || (rc = alloc_dev(b, &b->list_full, (size_t)b->ngran)) ||
        (rc = alloc_dev(b, &b->list_act, (size_t)b->ngran)) || (rc = alloc_dev(b, &b->n_full, 1)) ||
        (rc = alloc_dev(b, &b->n_act, 1)) || (rc = alloc_dev(b, &b->x, nv)) || (rc = alloc_dev(b, &b->r, nv)) ||
        (rc = alloc_dev(b, &b->p0, nv)) || (rc = alloc_dev(b, &b->p1, nv)) || (rc = alloc_dev(b, &b->q, nv)) ||
        (rc = alloc_dev(b, &b->part_a, ngp)) || (rc = alloc_dev(b, &b->part_b, ngp)) ||
        (rc = alloc_dev(b, &b->part_c, ngp)) || (rc = alloc_dev(b, &b->rr0, np)) || (rc = alloc_dev(b, &b->rr1, np)) ||
        (rc = alloc_dev(b, &b->bb, np)) || (rc = alloc_dev(b, &b->stop, np)) || (rc = alloc_dev(b, &b->rr_last, np)) ||
        (rc = alloc_dev(b, &b->it0, np)) || (rc = alloc_dev(b, &b->it1, np)) || (rc = alloc_dev(b, &b->it_last, np)) ||
        (rc = alloc_dev(b, &b->status, np)) || (rc = alloc_dev(b, &b->restarts, np)) ||
        (rc = alloc_dev(b, &b->nrun, 1)) || (rc = alloc_dev(b, &b->kmax, 1)) || (rc = alloc_dev(b, &b->alpha, np)) ||
        (rc = alloc_dev(b, &b->claim, (size_t)nsys)) || (rc = alloc_dev(b, &b->done, (size_t)nsys)) ||
        (rc = alloc_dev(b, &b->ctl, 4)))
        return bail(rc);
    {
        // claiming order of the one-launch schedule: larger systems (more
        // rows, as a rule more iterations) first
        std::vector<int32_t> prio(nsys);
        for (int s = 0; s < nsys; ++s) prio[s] = s;
        std::stable_sort(prio.begin(), prio.end(), [&](int32_t a, int32_t c) { return rows_h[a] > rows_h[c]; });
        if ((rc = upload(b, &b->prio, prio)) != SS_OK) return bail(rc);
    }
    // p0 / p1 are read (times beta = 0) before first written for stopped pairs
    if (hipMemsetAsync(b->p0, 0, sizeof(double) * nv, b->stream) != hipSuccess ||
        hipMemsetAsync(b->p1, 0, sizeof(double) * nv, b->stream) != hipSuccess ||
        hipMemsetAsync(b->status, 0xff, sizeof(int32_t) * np, b->stream) != hipSuccess)
        return bail(fail(SS_EDEVICE, "initialisation failed"));
    ss_batch_tuning t{2, 0, 8, opts.check_every > 0 ? opts.check_every + (opts.check_every & 1) : 32,
                      SS_BATCH_CHUNKED};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(b->key);
        if (it != g_tune_cache.end()) t = it->second;
    }
    if (!tuning_valid(t)) t.check_every = 32;
    if ((rc = apply_tuning(b, t)) != SS_OK) return bail(rc);
    *out = b;
    return SS_OK;
}

int ss_batch_set_tuning(ss_batch *b, const ss_batch_tuning *t)
{
    if (!b || !t) return fail(SS_EINVAL, "NULL argument");
    if (!tuning_valid(*t)) return fail(SS_EINVAL, "tuning out of range");
    return apply_tuning(b, *t);
}

int ss_batch_get_tuning(const ss_batch *b, ss_batch_tuning *t)
{
    if (!b || !t) return fail(SS_EINVAL, "NULL argument");
    *t = b->tun;
    return SS_OK;
}

int ss_batch_launches(const ss_batch *b, int32_t *graphs, int32_t *chunks, int32_t *kernels)
{
    if (!b) return fail(SS_EINVAL, "batch is NULL");
    if (graphs) *graphs = b->n_graph;
    if (chunks) *chunks = b->n_chunk;
    if (kernels) *kernels = b->n_kernel;
    return SS_OK;
}

int ss_batch_info(const ss_batch *b, int32_t *nsys, int32_t *nrhs, int64_t *nrows, int64_t *nnz, int64_t *stored)
{
    if (!b) return fail(SS_EINVAL, "batch is NULL");
    if (nsys) *nsys = b->nsys;
    if (nrhs) *nrhs = b->nrhs;
    if (nrows) *nrows = b->nrows;
    if (nnz) *nnz = b->nnz;
    if (stored) *stored = b->stored;
    return SS_OK;
}

int ss_batch_solve(ss_batch *b, const double *b_dev, double *x_dev, double tol, int32_t maxit, ss_result *res,
                   ss_result *summary)
{
    if (!b) return fail(SS_EINVAL, "batch is NULL");
    if (!b_dev || !x_dev) return fail(SS_EINVAL, "b or x is NULL");
    if (!(tol >= 0.0) || maxit < 0) return fail(SS_EINVAL, "need tol >= 0 and maxit >= 0");
    const size_t nv = (size_t)b->nrows * b->nrhs;
    const char *bl = (const char *)b_dev, *xl = (const char *)x_dev;
    if (bl < xl + nv * sizeof(double) && xl < bl + nv * sizeof(double))
        return fail(SS_EINVAL, "b and x overlap");
    SS_HIP(hipMemcpyAsync(b->x, x_dev, sizeof(double) * nv, hipMemcpyDeviceToDevice, b->stream));
    int32_t nrun = 0;
    b->n_graph = b->n_chunk = b->n_kernel = 0;
    int rc = start_pairs(b, b_dev, tol, maxit, &nrun);
    if (rc != SS_OK) return rc;
    // SS_BATCH_GRAPH: once a solve has set the lengths, the whole solve (its
    // chunks, residual check, restart chunks, final check) is one graph
    // launch; a solve that outruns it goes on as below, and the next one
    // learns the lengths again
    const bool graph = b->tun.schedule == SS_BATCH_GRAPH;
    bool learn = graph;
    if (graph && (rc = ensure_graph(b, b->tun.check_every)) != SS_OK) return rc;
    if (graph && b->hint > 0 && nrun > 0) {
        if ((rc = ensure_long_graph(b, b->tun.check_every, b->hint, b->hint2)) != SS_OK) return rc;
        SS_HIP(hipMemcpyAsync(b->bcopy, b_dev, sizeof(double) * nv, hipMemcpyDeviceToDevice, b->stream));
        SS_HIP(hipGraphLaunch(b->lexec, b->stream));
        ++b->n_graph;
        SS_HIP(hipMemcpyAsync(&b->pinned[0], b->nrun, sizeof(int32_t), hipMemcpyDeviceToHost, b->stream));
        SS_HIP(hipStreamSynchronize(b->stream));
        nrun = b->pinned[0];
        learn = false;
        if (nrun > 0) b->hint = b->hint2 = 0;
    }
    for (int round = 0; nrun > 0; ++round) {
        int32_t chunks = 0;
        if ((rc = iterate(b, &chunks)) != SS_OK) return rc;
        if (learn && round == 0) b->hint = std::max(b->hint, chunks);
        if (learn && round == 1) b->hint2 = std::max(b->hint2, chunks);
        if ((rc = residual_phase(b, b_dev, tol, false, &nrun)) != SS_OK) return rc;
        if (nrun == 0) break;
        compact(b, b->stream);
        spmv<M_FIRST>(b, b->stream, false, b->r, b->r, b->p1, b->q, 0);
        SS_HIP(hipGetLastError());
    }
    switch (b->nrhs) {
    case 1: hipLaunchKernelGGL(k_bstore<1>, dim3(b->grid()), dim3(kWG), 0, b->stream, b->bmat(), b->tiles(true), b->status, b->x, x_dev); break;
    case 2: hipLaunchKernelGGL(k_bstore<2>, dim3(b->grid()), dim3(kWG), 0, b->stream, b->bmat(), b->tiles(true), b->status, b->x, x_dev); break;
    default: hipLaunchKernelGGL(k_bstore<4>, dim3(b->grid()), dim3(kWG), 0, b->stream, b->bmat(), b->tiles(true), b->status, b->x, x_dev); break;
    }
    SS_HIP(hipGetLastError());

    const size_t np = (size_t)b->nsys * b->nrhs;
    std::vector<int32_t> st(np), it(np), rs(np);
    std::vector<double> rr(np), bbv(np);
    SS_HIP(hipStreamSynchronize(b->stream));
    SS_HIP(hipMemcpy(st.data(), b->status, sizeof(int32_t) * np, hipMemcpyDeviceToHost));
    SS_HIP(hipMemcpy(it.data(), b->it_last, sizeof(int32_t) * np, hipMemcpyDeviceToHost));
    SS_HIP(hipMemcpy(rs.data(), b->restarts, sizeof(int32_t) * np, hipMemcpyDeviceToHost));
    SS_HIP(hipMemcpy(rr.data(), b->rr_last, sizeof(double) * np, hipMemcpyDeviceToHost));
    SS_HIP(hipMemcpy(bbv.data(), b->bb, sizeof(double) * np, hipMemcpyDeviceToHost));
    ss_result worst{SS_OK, 0, 0, 0, 0.0, 0.0};
    bool any_break = false, any_maxit = false;
    for (size_t i = 0; i < np; ++i) {
        ss_result r{};
        switch (st[i]) {
        case BS_CONVERGED:
        case BS_ZERO_RHS: r.status = SS_OK; break;
        case BS_MAXIT: r.status = SS_NOT_CONVERGED; any_maxit = true; break;
        default: r.status = SS_EBREAKDOWN; any_break = true; break;
        }
        r.iterations = it[i];
        r.restarts = rs[i];
        r.relres = st[i] == BS_ZERO_RHS ? 0.0 : std::sqrt(rr[i] / bbv[i]);
        r.true_relres = r.relres;
        if (res) res[i] = r;
        worst.iterations = std::max(worst.iterations, r.iterations);
        worst.restarts = std::max(worst.restarts, r.restarts);
        if (!(r.relres <= worst.relres)) worst.relres = r.relres;  // NaN propagates
    }
    worst.status = any_break ? SS_EBREAKDOWN : any_maxit ? SS_NOT_CONVERGED : SS_OK;
    worst.true_relres = worst.relres;
    if (summary) *summary = worst;
    if (worst.status == SS_EBREAKDOWN) fail(SS_EBREAKDOWN, "CG breakdown in at least one pair");
    return worst.status;
}

int ss_batch_tune(ss_batch *b, const double *b_dev, int32_t iters, int32_t force, ss_batch_tuning *chosen,
                  ss_batch_trial *trials, int32_t cap, int32_t *ntrials)
{
    if (!b || !b_dev) return fail(SS_EINVAL, "NULL argument");
    if (ntrials) *ntrials = 0;
    if (!force) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(b->key);
        if (it != g_tune_cache.end()) {
            int rc = apply_tuning(b, it->second);
            if (rc != SS_OK) return rc;
            if (chosen) *chosen = b->tun;
            return SS_OK;
        }
    }
    const int32_t pairs = std::max(2, (iters > 0 ? iters : 8) + ((iters > 0 ? iters : 8) & 1));
    const int32_t check = b->tun.check_every;
    const size_t nv = (size_t)b->nrows * b->nrhs;
    std::vector<ss_batch_tuning> cands;
    for (int k : {0, 1, 2, 4, 8}) {
        for (int g : {0, 2048, 1024})
            for (int u : {4, 5, 8}) cands.push_back(ss_batch_tuning{k, g, u, pairs, SS_BATCH_CHUNKED});
        for (int u : {4, 5, 8}) cands.push_back(ss_batch_tuning{k, 0, u, check, SS_BATCH_PERSISTENT});
    }
    ss_batch_tuning best = b->tun;
    double best_ms = 0.0;
    int32_t n = 0;
    for (const auto &c : cands) {
        const bool flow = c.schedule == SS_BATCH_PERSISTENT;
        int rc = apply_tuning(b, c);
        if (rc != SS_OK) return rc;
        if (!flow && (rc = ensure_graph(b, pairs)) != SS_OK) return rc;
        double ms = 0.0;
        for (int rep = 0; rep < 2; ++rep) {  // first repetition warms up
            SS_HIP(hipMemsetAsync(b->x, 0, sizeof(double) * nv, b->stream));
            int32_t nrun = 0;
            // the one launch runs until every pair reaches the iteration limit
            if ((rc = start_pairs(b, b_dev, 0.0, flow ? pairs : INT32_MAX, &nrun)) != SS_OK) return rc;
            SS_HIP(hipEventRecord(b->ev[0], b->stream));
            if (flow) {
                if (nrun > 0 && (rc = iterate_flow(b)) != SS_OK) return rc;
            } else {
                SS_HIP(hipGraphLaunch(b->exec, b->stream));
            }
            SS_HIP(hipEventRecord(b->ev[1], b->stream));
            SS_HIP(hipEventSynchronize(b->ev[1]));
            float f = 0.f;
            SS_HIP(hipEventElapsedTime(&f, b->ev[0], b->ev[1]));
            ms = (double)f / pairs;
        }
        const ss_batch_tuning used{c.tile_granules, c.grid, c.unroll, check, c.schedule};
        if (trials && n < cap) trials[n] = ss_batch_trial{used, ms};
        ++n;
        if (best_ms == 0.0 || ms < best_ms) {
            best_ms = ms;
            best = used;
        }
    }
    if (ntrials) *ntrials = std::min(n, cap > 0 ? cap : 0);
    int rc = apply_tuning(b, best);
    if (rc != SS_OK) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[b->key] = best;
    }
    if (chosen) *chosen = best;
    return SS_OK;
}

}  // extern "C"
