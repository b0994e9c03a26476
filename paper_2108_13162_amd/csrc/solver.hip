// Solver driver: device layout and setup, the CG loop of Algorithm 3 with
// device-resident scalars, HIP-graph replay of polled iteration chunks, and
// the solver entry points of ss.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "host_common.h"
#include "kernels.h"
#include "ss_internal.h"

using namespace ss;

namespace {

constexpr int kDefaultCheck = 32;
constexpr int32_t kHistMax = 1 << 22;  // residual history entries kept on the device
constexpr int kSpmvGridMax = 1024;      // persistent SpMV workgroups (4 per CU)
// Up to this many chunks the SpMV grid is 3 workgroups per CU: at 4 a wave
// gets one or two chunks and has little to pipeline (measured: 7% faster
// per iteration at 64^3, equal at 96^3; 4 per CU wins from ~1.4M rows on).
constexpr int kSpmvGridSmall = 768;
constexpr int kSmallChunks = 16384;
constexpr int kGridLimit = 65536;       // upper bound accepted for a requested grid

// Persistent SpMV grid: one workgroup per 4 chunks (or per CSR tile) at most.
int32_t spmv_grid(bool sell, int32_t units, int32_t opt)
{
    const int32_t work = sell ? (units + kBS / 64 - 1) / (kBS / 64) : units;
    const int32_t dflt = sell && units <= kSmallChunks ? kSpmvGridSmall : kSpmvGridMax;
    return xcd_grid(std::max(1, std::min(work, opt ? opt : dflt)));
}

// Offset dictionary of a chunk: at most kDictOffsets distinct column - row
// offsets, rows of at most kDictSlots entries (4-bit indices, 8 to a word).
constexpr int kDictOffsets = 16;
constexpr int kDictSlots = 8;
constexpr int kDictMinPerWg = 24;  // chunks per SpMV workgroup for the dictionaries to pay

// Host image of the device data of one partition.
struct Layout {
    // device position of every concatenated local position
    std::vector<int32_t> dev_pos;
    int32_t n_own = 0, n_if = 0;
    std::vector<int32_t> l2g, g2own, copy_pos, pos_grp;
    // matrix in device order
    int fmt = FMT_SELL;
    std::vector<int32_t> col, nzmap;  // storage order (SELL padded: nzmap = -1); SELL: wide chunks only
    std::vector<int32_t> ccol;        // SELL: per chunk, start in col16 (>= 0) or ~start in col
    std::vector<uint16_t> col16;      // SELL: window offsets of the narrow chunks
    std::vector<int32_t> cbase;       // SELL: two window bases per chunk
    int64_t col_bytes = 0;            // column data the SpMV reads: 2 or 4 B per stored (non-padding) entry,
                                      // a dictionary chunk's 4 B per row and 64 B table
    int64_t struct_bytes = 0;         // row structure the SpMV reads: SELL a chunk's start, first row, length,
                                      // column start, window bases (and dictionary block) and 1 B per row
                                      // unless a dictionary word holds it; CSR the row pointers
    bool encode_ok = true;            // column encoding verified
    std::vector<int32_t> cptr, cpos, rowptr, tile_row;
    std::vector<uint8_t> clen, rlen;
    std::vector<int32_t> cdict, dtab;  // SELL: dictionary block of each chunk (-1: none); 16 offsets a block
    std::vector<uint32_t> dword;       // SELL: per block and lane, the 4-bit offset indices of slots 0..7
    int32_t nchunks = 0, ntiles = 0, tile_nnz = 2048;
    int32_t unroll = 8;               // SELL: entries per lane loaded before use
    int32_t one_batch = 0;            // SELL: no chunk longer than unroll
    int64_t stored = 0;  // entries incl. padding
};

// Device order: all owned interface copies (sub-domain by sub-domain), then
// all other interface copies, then every sub-domain's interior positions, the
// local order kept inside each group.  Within one local row all columns
// belong to the same sub-domain and keep their relative order, so row sums
// are unchanged.  Interface positions come first so that their (slower,
// gathering) update batches are dispatched first.
void build_order(const ss_part *p, Layout &L)
{
    const int32_t P = p->P, nl = p->n_loc();
    L.dev_pos.assign(nl, -1);
    int32_t tot_int = 0, tot_own = 0;
    for (int32_t s = 0; s < P; ++s) {
        tot_int += p->n_int[s];
        tot_own += p->n_own[s];
    }
    const int32_t tot_if = nl - tot_int;
    int32_t a = tot_if, b = 0, c = tot_own;
    for (int32_t s = 0; s < P; ++s) {
        const int32_t o = p->sub_off[s], i1 = o + p->n_int[s], i2 = i1 + p->n_own[s], e = p->sub_off[s + 1];
        for (int32_t u = o; u < i1; ++u) L.dev_pos[u] = a++;
        for (int32_t u = i1; u < i2; ++u) L.dev_pos[u] = b++;
        for (int32_t u = i2; u < e; ++u) L.dev_pos[u] = c++;
    }
    L.n_own = tot_own;
    L.n_if = tot_if;
    L.l2g.assign(nl, 0);
    for (int32_t u = 0; u < nl; ++u) L.l2g[L.dev_pos[u]] = p->l2g[u];
    L.g2own.resize(p->n);
    for (int32_t i = 0; i < p->n; ++i) L.g2own[i] = L.dev_pos[p->g2own[i]];
    L.copy_pos.resize(p->copy_pos.size());
    for (size_t u = 0; u < p->copy_pos.size(); ++u) L.copy_pos[u] = L.dev_pos[p->copy_pos[u]];
    L.pos_grp.assign((size_t)tot_if, -1);
    for (size_t g = 0; g + 1 < p->copy_ptr.size(); ++g)
        for (int32_t u = p->copy_ptr[g]; u < p->copy_ptr[g + 1]; ++u) L.pos_grp[L.copy_pos[u]] = (int32_t)g;
}

// Matrix storage.  SELL-64 unless a row is longer than 255 entries or the
// chunk padding would add more than a quarter to the stored entries; then
// CSR row tiles.  `force` = SS_MAT_* selection from the options, `grid_opt`
// the SpMV grid option (the chunk order depends on the grid).
void build_matrix(const ss_part *p, Layout &L, int32_t tile_nnz, int32_t force, int32_t grid_opt)
{
    const int32_t nl = p->n_loc();
    // rows in device order
    std::vector<int32_t> src_row(nl);
    for (int32_t u = 0; u < nl; ++u) src_row[L.dev_pos[u]] = u;
    auto row_len = [&](int32_t t) { return p->bd_rowptr[src_row[t] + 1] - p->bd_rowptr[src_row[t]]; };
    int32_t maxlen = 0;
    for (int32_t t = 0; t < nl; ++t) maxlen = std::max(maxlen, row_len(t));
    const int32_t nch = (nl + 63) / 64;
    int64_t padded = 0;
    for (int32_t c = 0; c < nch; ++c) {
        int32_t m = 0;
        for (int32_t t = c * 64; t < std::min(nl, c * 64 + 64); ++t) m = std::max(m, row_len(t));
        padded += 64 * (int64_t)m;
    }
    const bool sell_ok = maxlen <= 255 && padded < INT32_MAX;
    bool sell = sell_ok && padded <= p->nnz + p->nnz / 4;
    if (force == SS_MAT_SELL && sell_ok) sell = true;
    if (force == SS_MAT_CSR) sell = false;
    L.tile_nnz = tile_nnz;
    if (sell) {
        L.fmt = FMT_SELL;
        L.nchunks = nch;
        L.rlen.assign(nl, 0);
        for (int32_t t = 0; t < nl; ++t) L.rlen[t] = (uint8_t)row_len(t);
        // processing order: the chunks holding interface rows (positions
        // [0, n_if)) are spread evenly among the interior chunks
        const int32_t nif_ch = (L.n_if + 63) / 64;
        std::vector<int32_t> order;
        order.reserve(nch);
        int64_t placed_if = 0;
        int32_t next_if = 0, next_in = nif_ch;
        for (int32_t i = 0; i < nch; ++i) {
            const bool take_if = next_if < nif_ch &&
                                 (next_in >= nch || (int64_t)(i + 1) * nif_ch > placed_if * nch);
            if (take_if) {
                order.push_back(next_if++);
                ++placed_if;
            } else {
                order.push_back(next_in++);
            }
        }
        // Offset dictionaries: with every chunk one batch of at most 8 entries
        // (the unroll is chosen below from the same lengths), a chunk whose
        // columns take at most 16 distinct offsets from their rows is stored
        // once more as 4-bit indices into a table of those offsets; the
        // pipelined SpMV then reads one word per lane instead of one per
        // entry.  Inside each SpMV workgroup's range these chunks come first.
        std::vector<char> dict_ok(nch, 0);
        {
            std::vector<int32_t> clen_id(nch, 0);
            for (int32_t id = 0; id < nch; ++id)
                for (int32_t t = id * 64; t < std::min(nl, id * 64 + 64); ++t)
                    clen_id[id] = std::max(clen_id[id], std::max(row_len(t), 1));
            int64_t best_u = INT64_MAX;
            int32_t u_sel = 8;
            for (int32_t u : {9, 8, 7, 5}) {
                int64_t slots = 0;
                for (int32_t id = 0; id < nch; ++id) slots += (int64_t)((clen_id[id] + u - 1) / u) * u;
                if (slots < best_u) {
                    best_u = slots;
                    u_sel = u;
                }
            }
            bool one = true;
            for (int32_t id = 0; id < nch; ++id) one = one && clen_id[id] <= u_sel;
            // only where a wave gets several chunks: the switch to the other
            // kind costs a reload outside the pipeline (per iteration: 64^3,
            // 1.3 chunks a wave, 4.5% slower; 96^3, 4.5 a wave, even; 128^3,
            // 8 a wave, 2.8% faster; 160^3, 4.3% faster)
            const int32_t g = spmv_grid(true, nch, grid_opt);
            if (one && u_sel <= kDictSlots && nch >= kDictMinPerWg * g) {
                for (int32_t id = 0; id < nch; ++id) {
                    const int32_t c0 = id * 64;
                    if (c0 + 64 > nl) continue;
                    int32_t tbl[kDictOffsets] = {0};  // padding entries point at the row itself
                    int nt = 1;
                    bool ok = true;
                    for (int32_t t = c0; t < c0 + 64 && ok; ++t) {
                        const int32_t u = src_row[t];
                        for (int32_t e = p->bd_rowptr[u]; e < p->bd_rowptr[u + 1] && ok; ++e) {
                            const int32_t d = L.dev_pos[p->bd_colidx[e]] - t;
                            int q = 0;
                            while (q < nt && tbl[q] != d) ++q;
                            if (q == nt) {
                                if (nt == kDictOffsets)
                                    ok = false;
                                else
                                    tbl[nt++] = d;
                            }
                        }
                    }
                    dict_ok[id] = ok;
                }
                const int32_t cpb = (nch + g - 1) / g;
                for (int32_t lo = 0; lo < nch; lo += cpb)
                    std::stable_partition(order.begin() + lo, order.begin() + std::min(nch, lo + cpb),
                                          [&](int32_t id) { return dict_ok[id] != 0; });
            }
        }
        L.cptr.assign(nch + 1, 0);
        L.cpos.assign(nch, 0);
        L.clen.assign(nch, 0);
        for (int32_t i = 0; i < nch; ++i) {
            const int32_t id = order[i];
            int32_t m = 0;
            for (int32_t t = id * 64; t < std::min(nl, id * 64 + 64); ++t) m = std::max(m, (int32_t)L.rlen[t]);
            // at least one stored entry per chunk (padding for a chunk of
            // empty rows), so every batch of a chunk has entries to gather
            m = std::max(m, (int32_t)1);
            L.cpos[i] = id * 64;
            L.clen[i] = (uint8_t)m;
            L.cptr[i + 1] = L.cptr[i] + 64 * m;
        }
        L.stored = L.cptr[nch];
        // the unroll that wastes the fewest loads on the chunk lengths (ties:
        // the larger); a 7-point stencil gets 7, a 27-point one 9
        int64_t best = INT64_MAX;
        for (int32_t u : {9, 8, 7, 5}) {
            int64_t slots = 0;
            for (int32_t i = 0; i < nch; ++i) slots += (int64_t)((L.clen[i] + u - 1) / u) * u;
            if (slots < best) {
                best = slots;
                L.unroll = u;
            }
        }
        // every chunk one batch: the SpMV pipelines chunk to chunk
        L.one_batch = 1;
        for (int32_t i = 0; i < nch; ++i)
            if (L.clen[i] > L.unroll) L.one_batch = 0;
        // padding points at a valid position (the row itself, or 0 past the
        // last row) and is masked out by the row length
        L.col.assign((size_t)L.stored, 0);
        L.nzmap.assign((size_t)L.stored, -1);
        for (int32_t i = 0; i < nch; ++i)
            for (int32_t lane = 0; lane < 64; ++lane) {
                const int32_t t = L.cpos[i] + lane;
                const int32_t len = t < nl ? L.rlen[t] : 0;
                for (int32_t j = 0; j < L.clen[i]; ++j) {
                    const int64_t k = L.cptr[i] + (int64_t)j * 64 + lane;
                    if (j < len) {
                        const int32_t e = p->bd_rowptr[src_row[t]] + j;
                        L.col[k] = L.dev_pos[p->bd_colidx[e]];
                        L.nzmap[k] = p->bd_nzmap[e];
                    } else {
                        L.col[k] = t < nl ? t : 0;
                    }
                }
            }
        // 16-bit columns for chunks whose entries all fall in two windows of
        // 32768 positions: one around the chunk's rows, one at the lowest
        // column outside it (the interface copies an interior chunk reads);
        // int32 positions otherwise, and for a chunk holding no row past the end
        std::vector<int32_t> wide;
        L.ccol.assign(nch, 0);
        L.cbase.assign(2 * (size_t)nch, 0);
        L.col_bytes = 0;
        for (int32_t i = 0; i < nch; ++i) {
            const int64_t k0 = L.cptr[i], k1 = L.cptr[i + 1];
            const int32_t b1 = std::max(0, L.cpos[i] - 16384);
            int32_t lo2 = INT32_MAX, hi2 = -1;
            for (int64_t k = k0; k < k1; ++k)
                if (L.col[k] < b1 || L.col[k] > b1 + 32767) {
                    lo2 = std::min(lo2, L.col[k]);
                    hi2 = std::max(hi2, L.col[k]);
                }
            const bool narrow = L.cpos[i] + 64 <= nl && (hi2 < 0 || hi2 - lo2 <= 32767);
            const int32_t b2 = hi2 < 0 ? 0 : lo2;
            int64_t real = 0;
            for (int32_t lane = 0; lane < 64; ++lane)
                if (L.cpos[i] + lane < nl) real += L.rlen[L.cpos[i] + lane];
            L.col_bytes += real * (narrow ? 2 : 4);
            if (narrow) {
                // the SpMV reads 16-bit offsets in aligned pairs: each chunk's
                // start is even (64 entries per slot)
                L.ccol[i] = (int32_t)L.col16.size();
                if (L.ccol[i] & 1) L.encode_ok = false;
                L.cbase[2 * (size_t)i] = b1;
                L.cbase[2 * (size_t)i + 1] = b2;
                for (int64_t k = k0; k < k1; ++k) {
                    const int32_t v = L.col[k];
                    const bool in1 = v >= b1 && v <= b1 + 32767;
                    L.col16.push_back(in1 ? (uint16_t)(v - b1) : (uint16_t)(0x8000u | (uint32_t)(v - b2)));
                }
            } else {
                L.ccol[i] = ~(int32_t)wide.size();
                wide.insert(wide.end(), L.col.begin() + k0, L.col.begin() + k1);
            }
        }
        // every stored column must decode back to itself
        for (int32_t i = 0; i < nch; ++i)
            for (int64_t k = L.cptr[i]; k < L.cptr[i + 1]; ++k) {
                int32_t v;
                const int64_t off = k - L.cptr[i];
                if (L.ccol[i] >= 0) {
                    const uint32_t e = L.col16[(size_t)L.ccol[i] + off];
                    v = ((e & 0x8000u) ? L.cbase[2 * (size_t)i + 1] : L.cbase[2 * (size_t)i]) + (int32_t)(e & 0x7fffu);
                } else {
                    v = wide[(size_t)~L.ccol[i] + off];
                }
                if (v != L.col[k] || v < 0 || v >= std::max(nl, 1)) L.encode_ok = false;
            }
        // the offset dictionaries (processing order), checked entry by entry
        L.cdict.assign(nch, -1);
        for (int32_t i = 0; i < nch; ++i) {
            if (!dict_ok[L.cpos[i] / 64]) continue;
            const int32_t blk = (int32_t)(L.dtab.size() / kDictOffsets);
            std::vector<int32_t> offs(1, 0);
            for (int64_t k = L.cptr[i]; k < L.cptr[i + 1]; ++k) {
                const int32_t d = L.col[k] - (L.cpos[i] + (int32_t)((k - L.cptr[i]) % 64));
                if (std::find(offs.begin(), offs.end(), d) == offs.end()) offs.push_back(d);
                if ((int)offs.size() > kDictOffsets) break;
            }
            std::sort(offs.begin(), offs.end());
            if ((int)offs.size() > kDictOffsets || L.clen[i] > kDictSlots) {
                L.encode_ok = false;
                continue;
            }
            L.cdict[i] = blk;
            // the pipelined SpMV reads a word per row and the table instead
            int64_t real = 0;
            for (int32_t lane = 0; lane < 64; ++lane) real += L.rlen[L.cpos[i] + lane];
            L.col_bytes += 64 * 4 + kDictOffsets * 4 - real * (L.ccol[i] >= 0 ? 2 : 4);
            for (int32_t q = 0; q < kDictOffsets; ++q) L.dtab.push_back(q < (int32_t)offs.size() ? offs[q] : 0);
            const int32_t zero = (int32_t)(std::lower_bound(offs.begin(), offs.end(), 0) - offs.begin());
            for (int32_t lane = 0; lane < 64; ++lane) {
                const int32_t t = L.cpos[i] + lane;
                uint32_t wd = 0;
                for (int32_t j = 0; j < kDictSlots; ++j) {
                    int32_t q = zero;  // slots past the chunk length decode to the row itself
                    if (j < L.clen[i]) {
                        const int32_t d = L.col[L.cptr[i] + (int64_t)j * 64 + lane] - t;
                        q = (int32_t)(std::lower_bound(offs.begin(), offs.end(), d) - offs.begin());
                    }
                    if (j < L.unroll) wd |= (uint32_t)q << (4 * j);
                    const int32_t back = t + L.dtab[(size_t)blk * kDictOffsets + q];
                    if (j < L.clen[i] ? back != L.col[L.cptr[i] + (int64_t)j * 64 + lane] : back != t)
                        L.encode_ok = false;
                }
                // with at most 7 slots the top 4 bits hold the row's length
                if (L.unroll < kDictSlots) wd |= (uint32_t)L.rlen[t] << (4 * (kDictSlots - 1));
                L.dword.push_back(wd);
            }
        }
        L.struct_bytes = 0;
        for (int32_t i = 0; i < nch; ++i) {
            L.struct_bytes += 4 + 4 + 1 + 4 + 8 + (L.dtab.empty() ? 0 : 4);
            if (L.cdict[i] < 0 || L.unroll >= kDictSlots)
                for (int32_t lane = 0; lane < 64; ++lane) L.struct_bytes += L.cpos[i] + lane < nl ? 1 : 0;
        }
        L.col.swap(wide);
    } else {
        L.fmt = FMT_CSR;
        L.rowptr.assign(nl + 1, 0);
        for (int32_t t = 0; t < nl; ++t) L.rowptr[t + 1] = L.rowptr[t] + row_len(t);
        L.stored = L.rowptr[nl];
        L.col.resize((size_t)L.stored);
        L.nzmap.resize((size_t)L.stored);
        L.col_bytes = 4 * L.stored;
        L.struct_bytes = 4 * ((int64_t)nl + 1);
        for (int32_t t = 0; t < nl; ++t) {
            const int32_t u = src_row[t];
            for (int32_t e = p->bd_rowptr[u], k = L.rowptr[t]; e < p->bd_rowptr[u + 1]; ++e, ++k) {
                L.col[k] = L.dev_pos[p->bd_colidx[e]];
                L.nzmap[k] = p->bd_nzmap[e];
            }
        }
        // row tiles: at most tile_nnz entries and 4 * workgroup rows; a longer
        // row is a tile of its own
        L.tile_row.assign(1, 0);
        int32_t r0 = 0;
        while (r0 < nl) {
            int32_t r = r0;
            if (L.rowptr[r0 + 1] - L.rowptr[r0] > tile_nnz)
                r = r0 + 1;
            else
                while (r < nl && r - r0 < 4 * kBS && L.rowptr[r + 1] - L.rowptr[r0] <= tile_nnz) ++r;
            L.tile_row.push_back(r);
            r0 = r;
        }
        L.ntiles = (int32_t)L.tile_row.size() - 1;
    }
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
    DevState *st = nullptr;
    double *hist = nullptr;
    int32_t hist_cap = 0;

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
    if (opts.precond == SS_PRECOND_JACOBI) {
        diag.assign((size_t)A->n, 0.0);
        for (int32_t i = 0; i < A->n; ++i)
            for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
                if (A->colidx[k] == i) diag[i] = A->val[k];
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
        for (size_t c = 0; c < nl; ++c) dinv[c] = 1.0 / diag[(size_t)L.l2g[c]];
        if ((rc = upload(s, &s->dinv, dinv.data(), dinv.size())) || (rc = alloc_dev(s, &s->z, nl)) ||
            (rc = alloc_dev(s, &s->part_b2, (size_t)I.grid)))
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

int ss_cg_solve(ss_solver *s, const double *b_dev, double *x_dev, double tol, int32_t maxit, ss_result *res,
                double *hist_host)
{
    if (!s) return fail(SS_EINVAL, "solver is NULL");
    if (!b_dev || !x_dev) return fail(SS_EINVAL, "b or x is NULL");
    if (!(tol >= 0.0) || maxit < 0) return fail(SS_EINVAL, "need tol >= 0 and maxit >= 0");
    int rc = ensure_hist(s, std::min<int64_t>((int64_t)maxit + 1, kHistMax));
    if (rc != SS_OK) return rc;
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
    if (s->opts.precision == SS_FP64) {
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
    if (res) {
        res->status = code;
        res->iterations = f.iter_last;
        res->outer_iterations = outer;
        res->restarts = restarts;
        res->relres = relres;
        res->true_relres = relres;
    }
    if (hist_host) {
        const int32_t cnt = f.status == ST_ZERO_RHS ? 1 : std::min(f.iter_last + 1, s->hist_cap);
        SS_HIP(hipMemcpy(hist_host, s->hist, sizeof(double) * cnt, hipMemcpyDeviceToHost));
    }
    if (code == SS_EBREAKDOWN) fail(SS_EBREAKDOWN, "CG breakdown: (p, A p) <= 0 or non-finite value");
    return code;
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
