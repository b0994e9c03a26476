// Host-side layout builder (see layout.h).
#include "layout.h"

#include <algorithm>
#include <climits>
#include <cstdint>
#include <vector>

#include "ss.h"

namespace ss {

namespace {
constexpr int kSpmvGridMax = 1024;      // persistent SpMV workgroups (4 per CU)
// Up to this many chunks the SpMV grid is 3 workgroups per CU: at 4 a wave
// gets one or two chunks and has little to pipeline (measured: 7% faster
// per iteration at 64^3, equal at 96^3; 4 per CU wins from ~1.4M rows on).
constexpr int kSpmvGridSmall = 768;
constexpr int kSmallChunks = 16384;

// Offset dictionary of a chunk: at most kDictOffsets distinct column - row
// offsets, rows of at most kDictSlots entries (4-bit indices, 8 to a word).
constexpr int kDictOffsets = 16;
// SELL storage holds fewer local positions than this (FP64 vectors under 4 GiB).
constexpr int32_t kSellMaxRows = 1 << 29;
constexpr int kDictSlots = 8;
constexpr int kDictMinPerWg = 24;  // chunks per SpMV workgroup for the dictionaries to pay
// Rows of several load batches: at most 64 offsets (6-bit indices, a batch of
// at most 10 slots in two words).
constexpr int kWideOffsets = 64;
constexpr int kWideSlots = 10;

}  // namespace

// Persistent SpMV grid: one workgroup per 4 chunks (or per CSR tile) at most.
int32_t spmv_grid(bool sell, int32_t units, int32_t opt)
{
    const int32_t work = sell ? (units + kBS / 64 - 1) / (kBS / 64) : units;
    const int32_t dflt = sell && units <= kSmallChunks ? kSpmvGridSmall : kSpmvGridMax;
    return xcd_grid(std::max(1, std::min(work, opt ? opt : dflt)));
}



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
    // (the SELL SpMV addresses its vectors through 32-bit byte offsets)
    const bool sell_ok = maxlen <= 255 && padded < INT32_MAX && nl < kSellMaxRows;
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
        // Wide offset dictionaries (rows of several load batches, all 64 rows
        // of the chunk present): at most 64 distinct column - row offsets,
        // each batch's slots as 6-bit indices in two words per lane, so the
        // SpMV reads 8 B per row and batch and a 256 B table instead of 2 or
        // 4 B per entry.  Checked entry by entry.
        if (L.dtab.empty() && !L.one_batch && L.unroll <= kWideSlots) {
            int32_t nbmax = 0;
            for (int32_t i = 0; i < nch; ++i) nbmax = std::max(nbmax, (L.clen[i] + L.unroll - 1) / L.unroll);
            std::vector<int32_t> offs;
            for (int32_t i = 0; i < nch; ++i) {
                if (L.cpos[i] + 64 > nl) continue;
                offs.assign(1, 0);  // padding and clamped slots decode to the row itself
                bool ok = true;
                for (int64_t k = L.cptr[i]; k < L.cptr[i + 1] && ok; ++k) {
                    const int32_t d = L.col[k] - (L.cpos[i] + (int32_t)((k - L.cptr[i]) % 64));
                    if (std::find(offs.begin(), offs.end(), d) == offs.end()) {
                        offs.push_back(d);
                        ok = (int)offs.size() <= kWideOffsets;
                    }
                }
                if (!ok) continue;
                std::sort(offs.begin(), offs.end());
                const int32_t blk = (int32_t)(L.dtab.size() / kWideOffsets);
                L.cdict[i] = blk;
                for (int32_t q = 0; q < kWideOffsets; ++q) L.dtab.push_back(q < (int32_t)offs.size() ? offs[q] : 0);
                const int32_t len_c = L.clen[i], nb = (len_c + L.unroll - 1) / L.unroll;
                L.dword.resize(((size_t)blk + 1) * nbmax * 64 * 2, 0u);
                int64_t real = 0;
                for (int32_t lane = 0; lane < 64; ++lane) {
                    const int32_t t = L.cpos[i] + lane;
                    real += L.rlen[t];
                    for (int32_t j = 0; j < nb; ++j) {
                        uint64_t bits = 0;
                        for (int32_t u = 0; u < L.unroll; ++u) {
                            // slots past the chunk repeat its last one, as the SpMV's loads do
                            const int32_t slot = std::min(j * L.unroll + u, len_c - 1);
                            const int32_t d = L.col[L.cptr[i] + (int64_t)slot * 64 + lane] - t;
                            const int32_t q = (int32_t)(std::lower_bound(offs.begin(), offs.end(), d) - offs.begin());
                            if (q >= (int32_t)offs.size() || offs[q] != d) L.encode_ok = false;
                            bits |= (uint64_t)q << (6 * u);
                        }
                        const size_t w = (((size_t)blk * nbmax + j) * 64 + lane) * 2;
                        L.dword[w] = (uint32_t)bits;
                        L.dword[w + 1] = (uint32_t)(bits >> 32);
                    }
                }
                L.col_bytes += (int64_t)nb * 64 * 8 + kWideOffsets * 4 - real * (L.ccol[i] >= 0 ? 2 : 4);
            }
            if (!L.dtab.empty()) L.dict_batches = nbmax;
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

void build_small(const ss_part *p, const Layout &L, const double *val, int32_t width, std::vector<double> &sv,
                 std::vector<uint32_t> &sc)
{
    const int32_t nl = p->n_loc(), uw = (width + 1) / 2;
    sv.assign((size_t)width * nl, 0.0);
    sc.assign((size_t)uw * nl, 0u);
    std::vector<int32_t> src(nl);
    for (int32_t u = 0; u < nl; ++u) src[L.dev_pos[u]] = u;
    for (int32_t t = 0; t < nl; ++t) {
        const int32_t u = src[t], e0 = p->bd_rowptr[u], len = p->bd_rowptr[u + 1] - e0;
        for (int32_t j = 0; j < width; ++j) {
            int32_t c = t;  // padding: the row itself, masked by the length
            if (j < len) {
                c = L.dev_pos[p->bd_colidx[e0 + j]];
                sv[(size_t)j * nl + t] = val[p->bd_nzmap[e0 + j]];
            }
            sc[(size_t)(j / 2) * nl + t] |= (uint32_t)c << (16 * (j & 1));
        }
        sc[(size_t)(uw - 1) * nl + t] |= (uint32_t)len << 16;
    }
}

int64_t layout_check(const ss_part *p, const Layout &L)
{
    const int32_t nl = p->n_loc();
    int64_t bad = 0;
    std::vector<int32_t> src(nl, -1);
    for (int32_t u = 0; u < nl; ++u) {
        const int32_t t = L.dev_pos[u];
        if (t < 0 || t >= nl || src[t] >= 0) return 1;  // not a permutation
        src[t] = u;
    }
    // the entries of device row t, as stored, against the local row src[t]
    auto expect = [&](int32_t t, int32_t j, int32_t col, int32_t nz) {
        const int32_t u = src[t], e = p->bd_rowptr[u] + j;
        if (col != L.dev_pos[p->bd_colidx[e]] || nz != p->bd_nzmap[e]) ++bad;
    };
    if (L.fmt == FMT_SELL) {
        std::vector<char> seen((size_t)std::max(L.nchunks, 1), 0);
        std::vector<int32_t> wide_start;  // ~ccol of the wide chunks
        for (int32_t i = 0; i < L.nchunks; ++i) {
            const int32_t cp = L.cpos[i];
            if (cp % 64 || cp < 0 || cp / 64 >= L.nchunks || seen[cp / 64]) return bad + 1;
            seen[cp / 64] = 1;
            const int32_t len_c = L.clen[i];
            if (L.cptr[i + 1] - L.cptr[i] != 64 * len_c) ++bad;
            for (int32_t lane = 0; lane < 64; ++lane) {
                const int32_t t = cp + lane;
                const int32_t rl = t < nl ? L.rlen[t] : 0;
                if (t < nl && rl != p->bd_rowptr[src[t] + 1] - p->bd_rowptr[src[t]]) ++bad;
                if (rl > len_c) ++bad;
                for (int32_t j = 0; j < len_c; ++j) {
                    const int64_t k = L.cptr[i] + (int64_t)j * 64 + lane;
                    const int64_t off = k - L.cptr[i];
                    int32_t col;
                    if (L.ccol[i] >= 0) {
                        const uint32_t e = L.col16[(size_t)L.ccol[i] + off];
                        col = ((e & 0x8000u) ? L.cbase[2 * (size_t)i + 1] : L.cbase[2 * (size_t)i]) +
                              (int32_t)(e & 0x7fffu);
                    } else {
                        col = L.col[(size_t)~L.ccol[i] + off];
                    }
                    if (j < rl)
                        expect(t, j, col, L.nzmap[k]);
                    else if (L.nzmap[k] != -1 || col < 0 || col >= std::max(nl, 1))
                        ++bad;
                    // a wide dictionary chunk decodes to the same column
                    if (L.dict_batches > 0 && L.cdict[i] >= 0) {
                        const int32_t jb = j / L.unroll, u = j % L.unroll;
                        const size_t w = (((size_t)L.cdict[i] * L.dict_batches + jb) * 64 + lane) * 2;
                        const uint64_t bits = ((uint64_t)L.dword[w + 1] << 32) | L.dword[w];
                        const int32_t q = (int32_t)((bits >> (6 * u)) & 63u);
                        if (t + L.dtab[(size_t)L.cdict[i] * kWideOffsets + q] != col) ++bad;
                    }
                    // a dictionary chunk decodes to the same column
                    if (L.dict_batches == 0 && !L.cdict.empty() && L.cdict[i] >= 0 && j < std::min(len_c, L.unroll)) {
                        const uint32_t wd = L.dword[(size_t)L.cdict[i] * 64 + lane];
                        const int32_t q = (int32_t)((wd >> (4 * j)) & 15u);
                        const int32_t dc = t + L.dtab[(size_t)L.cdict[i] * kDictOffsets + q];
                        if (dc != (j < rl ? col : t)) ++bad;
                    }
                }
            }
        }
    } else {
        if (L.rowptr.size() != (size_t)nl + 1 || L.tile_row.empty() || L.tile_row.back() != nl) return bad + 1;
        for (int32_t t = 0; t < nl; ++t) {
            const int32_t len = L.rowptr[t + 1] - L.rowptr[t];
            if (len != p->bd_rowptr[src[t] + 1] - p->bd_rowptr[src[t]]) {
                ++bad;
                continue;
            }
            for (int32_t j = 0; j < len; ++j) expect(t, j, L.col[(size_t)L.rowptr[t] + j], L.nzmap[(size_t)L.rowptr[t] + j]);
        }
    }
    return bad;
}

}  // namespace ss
