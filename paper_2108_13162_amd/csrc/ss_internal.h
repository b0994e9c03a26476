// Internal declarations shared by the host-side sources of libss.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "ss.h"

namespace ss {

// Records the detail message returned by ss_last_error() and passes the code on.
int fail(int code, const std::string &msg);

// Structural + numerical checks of a CSR matrix (ss_csr contract).
int validate_csr(const ss_csr *A, bool require_symmetric);

// Node partitions.
int partition_box(int32_t n, int32_t dim, const int32_t *grid, const int32_t *boxes, int32_t nparts,
                  std::vector<int32_t> &part);
int partition_rcb(int32_t n, int32_t dim, const double *coords, const double *weights, int32_t nparts,
                  std::vector<int32_t> &part);
int partition_graph(const ss_csr *A, const double *weights, int32_t nparts, std::vector<int32_t> &part);

}  // namespace ss

struct ss_part {
    int32_t n = 0;
    int32_t P = 0;
    int64_t nnz = 0;
    std::vector<int32_t> part;      // [n] node -> sub-domain
    std::vector<int32_t> mult;      // [n] number of sub-domains holding the node
    std::vector<int32_t> sub_off;   // [P+1]
    std::vector<int32_t> n_int;     // [P] interior nodes
    std::vector<int32_t> n_own;     // [P] owned interface nodes
    std::vector<int32_t> l2g;       // [n_loc]
    std::vector<int32_t> gamma;     // [n_gamma]
    std::vector<int32_t> copy_ptr;  // [n_gamma+1]
    std::vector<int32_t> copy_pos;  // [n_copies]
    std::vector<int32_t> g2own;     // [n] owned position of every node
    std::vector<int32_t> bd_rowptr; // [n_loc+1]
    std::vector<int32_t> bd_colidx; // [nnz]
    std::vector<int32_t> bd_nzmap;  // [nnz]
    int32_t n_loc() const { return sub_off.empty() ? 0 : sub_off.back(); }
};

namespace ss {
// Owner-rule split and local numbering; fills every map of `p` from A and p->part.
int build_subdomains(const ss_csr *A, ss_part *p);
}  // namespace ss
