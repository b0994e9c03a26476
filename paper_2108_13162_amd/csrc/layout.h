// Host-side layout of the device data of one partition: the device
// position order of the local positions and the storage of the block-diagonal
// matrix of all local matrices (SELL-64 chunks with their column encodings
// and offset dictionaries, or CSR row tiles), built and verified on the host
// before the upload.  Plain C++ (no HIP), so that it can also be built and
// checked on its own with the host sanitizers.
#pragma once

#include <cstdint>
#include <vector>

#include "launch_shape.h"
#include "ss_internal.h"

namespace ss {

constexpr int kGridLimit = 65536;  // upper bound accepted for a requested SpMV grid

// Persistent SpMV grid: one workgroup per 4 chunks (or per CSR tile) at most.
int32_t spmv_grid(bool sell, int32_t units, int32_t opt);

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
    // SELL offset dictionaries.  One-batch rows: 16 offsets a block, per block
    // and lane one word of 4-bit indices (slots 0..7).  Rows of several load
    // batches (dict_batches > 0): 64 offsets a block, per block, batch and
    // lane two words of 6-bit indices (the batch's slots, at most 10).
    std::vector<int32_t> cdict, dtab;  // dictionary block of each chunk (-1: none); the block's offsets
    std::vector<uint32_t> dword;       // the index words
    int32_t dict_batches = 0;          // several-batch rows: load batches per block (0: the one-batch kind)
    int32_t nchunks = 0, ntiles = 0, tile_nnz = 2048;
    int32_t unroll = 8;               // SELL: entries per lane loaded before use
    int32_t one_batch = 0;            // SELL: no chunk longer than unroll
    int64_t stored = 0;  // entries incl. padding
};

// Device order: all owned interface copies (sub-domain by sub-domain), then
// all other interface copies, then every sub-domain's interior positions, the
// local order kept inside each group.
void build_order(const ss_part *p, Layout &L);

// Matrix storage in device order (SS_MAT_* selection `force`, the SpMV grid
// option `grid_opt`, on which the chunk order depends).  Sets L.encode_ok to
// false if any stored column fails to decode back to itself.
void build_matrix(const ss_part *p, Layout &L, int32_t tile_nnz, int32_t force, int32_t grid_opt);

// Storage of the one-launch small solve: `width` value slots per row,
// slot-major in device order (sv[j * n_loc + t]), zero past the row's length;
// two 16-bit column positions per word (sc[(j / 2) * n_loc + t], padding the
// row itself) with the row's length in the upper half of the last word.
// `width` must be odd and at least the longest row; n_loc <= 65536.
void build_small(const ss_part *p, const Layout &L, const double *val, int32_t width, std::vector<double> &sv,
                 std::vector<uint32_t> &sc);

// Decodes the storage built by build_matrix back to (device row, device
// column, global entry) triples and compares them with the block-diagonal
// CSR of p: every stored entry of every local row exactly once, in the row's
// column order, padding pointing at valid positions.  0 when all hold, else
// the number of violations found.
int64_t layout_check(const ss_part *p, const Layout &L);

}  // namespace ss
