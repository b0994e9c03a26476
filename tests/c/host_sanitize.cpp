// Host-code check under AddressSanitizer and UndefinedBehaviorSanitizer:
// the partitioners (box, weighted RCB, user, graph), the owner-rule split and
// its maps, and the device layout builder (SELL-64 chunks with 16-bit and
// int32 columns and offset dictionaries, CSR row tiles, the one-launch small
// storage), on a set of matrices, with every layout decoded back and compared
// with the block-diagonal CSR.  Built by tests/test_host_sanitize.py with
// g++ -fsanitize=address,undefined together with host_partition.cpp,
// graph_partition.cpp and layout.cpp; prints "ok" and exits 0 when every
// check holds.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "layout.h"
#include "ss.h"
#include "ss_internal.h"

namespace {

int g_fail = 0;
int64_t g_dict_chunks = 0, g_wdict_chunks = 0, g_wide_chunks = 0, g_narrow_chunks = 0, g_csr_layouts = 0;

#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++g_fail;                                                            \
        }                                                                        \
    } while (0)

struct Csr {
    int32_t n = 0;
    std::vector<int32_t> rowptr, colidx;
    std::vector<double> val;
    ss_csr view() const { return ss_csr{n, (int32_t)colidx.size(), rowptr.data(), colidx.data(), val.data()}; }
};

// Symmetric matrix from a neighbour rule on a structured grid (x fastest):
// offsets are (dx, dy, dz) triples; off-diagonals -w, diagonal = 1 + sum of
// |off-diagonals|.
Csr stencil(int mx, int my, int mz, const std::vector<int> &offs, unsigned seed)
{
    std::mt19937 rng(seed);
    std::uniform_real_distribution<double> U(0.5, 2.0);
    Csr A;
    A.n = mx * my * mz;
    std::vector<std::vector<std::pair<int32_t, double>>> rows(A.n);
    auto id = [&](int x, int y, int z) { return x + mx * (y + my * z); };
    for (int z = 0; z < mz; ++z)
        for (int y = 0; y < my; ++y)
            for (int x = 0; x < mx; ++x)
                for (size_t o = 0; o + 2 < offs.size(); o += 3) {
                    const int X = x + offs[o], Y = y + offs[o + 1], Z = z + offs[o + 2];
                    if (X < 0 || Y < 0 || Z < 0 || X >= mx || Y >= my || Z >= mz) continue;
                    const int i = id(x, y, z), j = id(X, Y, Z);
                    if (j <= i) continue;
                    const double w = U(rng);
                    rows[i].push_back({j, -w});
                    rows[j].push_back({i, -w});
                }
    A.rowptr.push_back(0);
    for (int32_t i = 0; i < A.n; ++i) {
        double d = 1.0;
        for (auto &e : rows[i]) d += std::fabs(e.second);
        rows[i].push_back({i, d});
        std::sort(rows[i].begin(), rows[i].end());
        for (auto &e : rows[i]) {
            A.colidx.push_back(e.first);
            A.val.push_back(e.second);
        }
        A.rowptr.push_back((int32_t)A.colidx.size());
    }
    return A;
}

// Random symmetric pattern with long rows for some nodes (CSR tiles, wide chunks).
Csr random_matrix(int32_t n, int per_row, int hubs, unsigned seed)
{
    std::mt19937 rng(seed);
    std::uniform_int_distribution<int32_t> pick(0, n - 1);
    std::vector<std::vector<int32_t>> adj(n);
    auto link = [&](int32_t i, int32_t j) {
        if (i == j) return;
        adj[i].push_back(j);
        adj[j].push_back(i);
    };
    for (int32_t i = 0; i < n; ++i)
        for (int k = 0; k < per_row; ++k) link(i, pick(rng));
    for (int h = 0; h < hubs; ++h)
        for (int k = 0; k < 300; ++k) link(h, pick(rng));
    Csr A;
    A.n = n;
    A.rowptr.push_back(0);
    for (int32_t i = 0; i < n; ++i) {
        adj[i].push_back(i);
        std::sort(adj[i].begin(), adj[i].end());
        adj[i].erase(std::unique(adj[i].begin(), adj[i].end()), adj[i].end());
        for (int32_t j : adj[i]) {
            A.colidx.push_back(j);
            A.val.push_back(j == i ? 2.0 * (double)adj[i].size() : -1.0);
        }
        A.rowptr.push_back((int32_t)A.colidx.size());
    }
    return A;
}

// The maps of a partition: sizes add up, every local entry maps to one global
// entry, and the local matrices sum back to A.
void check_part(const Csr &A, const ss_part *p)
{
    int32_t P = 0, n = 0, nl = 0, ng = 0, nc = 0;
    int64_t nnz = 0;
    CHECK(ss_part_sizes(p, &P, &n, &nl, &ng, &nc, &nnz) == SS_OK);
    CHECK(n == A.n && nnz == (int64_t)A.colidx.size());
    std::vector<int32_t> part(n), sub_off(P + 1), n_int(P), n_own(P), l2g(nl), gamma(ng), cptr(ng + 1), cpos(nc);
    CHECK(ss_part_export(p, part.data(), sub_off.data(), n_int.data(), n_own.data(), l2g.data(), gamma.data(),
                         cptr.data(), cpos.data()) == SS_OK);
    std::vector<int32_t> brp(nl + 1), bci(nnz), bnz(nnz);
    CHECK(ss_part_export_local(p, brp.data(), bci.data(), bnz.data()) == SS_OK);
    CHECK(sub_off[0] == 0 && sub_off[P] == nl && brp[nl] == (int32_t)nnz);
    std::vector<int> used(nnz, 0);
    for (int32_t r = 0; r < nl; ++r)
        for (int32_t e = brp[r]; e < brp[r + 1]; ++e) {
            CHECK(bnz[e] >= 0 && bnz[e] < nnz);
            if (bnz[e] < 0 || bnz[e] >= nnz) continue;
            ++used[bnz[e]];
            CHECK(bci[e] >= 0 && bci[e] < nl);
            // the global entry's row and column are the local ones' global ids
            const int32_t gi = l2g[r], gj = l2g[bci[e]];
            CHECK(A.colidx[bnz[e]] == gj && bnz[e] >= A.rowptr[gi] && bnz[e] < A.rowptr[gi + 1]);
            if (e > brp[r]) CHECK(bci[e - 1] < bci[e]);
        }
    for (int64_t k = 0; k < nnz; ++k) CHECK(used[k] == 1);
    for (int32_t g = 0; g < ng; ++g) {
        CHECK(cptr[g + 1] - cptr[g] >= 2);
        for (int32_t c = cptr[g]; c < cptr[g + 1]; ++c) CHECK(l2g[cpos[c]] == gamma[g]);
    }
}

void check_layouts(const Csr &A, const ss_part *p)
{
    ss::Layout L0;
    ss::build_order(p, L0);
    for (int32_t fmt : {SS_MAT_AUTO, SS_MAT_SELL, SS_MAT_CSR})
        for (int32_t grid : {0, 8, 40, 1024})
            for (int32_t tile : {1024, 2048}) {
                if (fmt != SS_MAT_CSR && tile != 2048) continue;
                ss::Layout L;
                ss::build_order(p, L);
                ss::build_matrix(p, L, tile, fmt, grid);
                CHECK(L.encode_ok);
                CHECK(ss::layout_check(p, L) == 0);
                if (L.fmt == ss::FMT_CSR) ++g_csr_layouts;
                for (int32_t i = 0; i < L.nchunks; ++i) {
                    g_dict_chunks += !L.cdict.empty() && L.cdict[i] >= 0 && L.dict_batches == 0;
                    g_wdict_chunks += !L.cdict.empty() && L.cdict[i] >= 0 && L.dict_batches > 0;
                    (L.ccol[i] >= 0 ? g_narrow_chunks : g_wide_chunks) += 1;
                }
            }
    // the one-launch storage
    int32_t wmax = 0;
    for (int32_t u = 0; u < p->n_loc(); ++u) wmax = std::max(wmax, p->bd_rowptr[u + 1] - p->bd_rowptr[u]);
    if (wmax <= 7 && p->n_loc() <= 65536) {
        const int32_t width = wmax <= 5 ? 5 : 7, uw = (width + 1) / 2, nl = p->n_loc();
        std::vector<double> sv;
        std::vector<uint32_t> sc;
        ss::build_small(p, L0, A.val.data(), width, sv, sc);
        CHECK(sv.size() == (size_t)width * nl && sc.size() == (size_t)uw * nl);
        std::vector<int32_t> src(nl);
        for (int32_t u = 0; u < nl; ++u) src[L0.dev_pos[u]] = u;
        for (int32_t t = 0; t < nl; ++t) {
            const int32_t u = src[t], len = (int32_t)(sc[(size_t)(uw - 1) * nl + t] >> 16);
            CHECK(len == p->bd_rowptr[u + 1] - p->bd_rowptr[u]);
            for (int32_t j = 0; j < width; ++j) {
                const int32_t c = (int32_t)((sc[(size_t)(j / 2) * nl + t] >> (16 * (j & 1))) & 0xffffu);
                if (j < len) {
                    const int32_t e = p->bd_rowptr[u] + j;
                    CHECK(c == L0.dev_pos[p->bd_colidx[e]]);
                    CHECK(sv[(size_t)j * nl + t] == A.val[p->bd_nzmap[e]]);
                } else {
                    CHECK(c == t && sv[(size_t)j * nl + t] == 0.0);
                }
            }
        }
    }
}

void run(const char *name, const Csr &A, int32_t method, int32_t nparts, int32_t dim, const int32_t *grid,
         const int32_t *boxes, const double *coords, const int32_t *user)
{
    const ss_csr v = A.view();
    ss_part *p = nullptr;
    const int rc = ss_partition(&v, method, nparts, dim, grid, boxes, coords, nullptr, user, &p);
    CHECK(rc == SS_OK);
    if (rc != SS_OK) {
        std::fprintf(stderr, "%s: %s\n", name, ss_last_error());
        return;
    }
    check_part(A, p);
    check_layouts(A, p);
    ss_part_destroy(p);
    std::printf("%s: n=%d parts=%d\n", name, A.n, nparts);
}

}  // namespace

int main()
{
    {
        const Csr A = stencil(37, 29, 1, {1, 0, 0, 0, 1, 0}, 1);  // 2D 5-point
        const int32_t grid[2] = {37, 29}, boxes[2] = {3, 2};
        run("poisson2d_box", A, SS_PART_BOX, 6, 2, grid, boxes, nullptr, nullptr);
        std::vector<int32_t> user(A.n);
        std::mt19937 rng(3);
        for (auto &u : user) u = (int32_t)(rng() % 5);
        user[0] = 4;
        run("poisson2d_user", A, SS_PART_USER, 7, 0, nullptr, nullptr, nullptr, user.data());  // parts 5, 6 empty
        run("poisson2d_graph", A, SS_PART_GRAPH, 5, 0, nullptr, nullptr, nullptr, nullptr);
    }
    {
        const Csr A = stencil(24, 24, 24, {1, 0, 0, 0, 1, 0, 0, 0, 1}, 2);  // 3D 7-point, dictionaries at grid 8
        const int32_t grid[3] = {24, 24, 24}, boxes[3] = {2, 2, 2};
        run("diffusion3d_box", A, SS_PART_BOX, 8, 3, grid, boxes, nullptr, nullptr);
        std::vector<double> coords(3 * (size_t)A.n);
        for (int32_t i = 0; i < A.n; ++i) {
            coords[3 * i] = i % 24;
            coords[3 * i + 1] = (i / 24) % 24;
            coords[3 * i + 2] = i / 576;
        }
        run("diffusion3d_rcb", A, SS_PART_RCB, 11, 3, nullptr, nullptr, coords.data(), nullptr);
    }
    {
        std::vector<int> offs;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx)
                    if (dx || dy || dz) offs.insert(offs.end(), {dx, dy, dz});
        const Csr A = stencil(11, 9, 10, offs, 4);  // 27-point: several load batches per row
        const int32_t grid[3] = {11, 9, 10}, boxes[3] = {2, 3, 2};
        run("stencil27_box", A, SS_PART_BOX, 12, 3, grid, boxes, nullptr, nullptr);
    }
    {
        const Csr A = random_matrix(3000, 3, 3, 5);  // hubs of > 255 entries: CSR tiles, far columns
        run("random_graph", A, SS_PART_GRAPH, 6, 0, nullptr, nullptr, nullptr, nullptr);
        std::vector<int32_t> user(A.n);
        for (int32_t i = 0; i < A.n; ++i) user[i] = (int32_t)((i * 7) % 4);
        run("random_user", A, SS_PART_USER, 4, 0, nullptr, nullptr, nullptr, user.data());
    }
    {
        // invalid inputs are rejected without touching memory out of range
        Csr A = stencil(5, 5, 1, {1, 0, 0, 0, 1, 0}, 6);
        ss_csr v = A.view();
        ss_part *p = nullptr;
        const int32_t grid[2] = {5, 5}, boxes[2] = {2, 2};
        CHECK(ss_partition(&v, SS_PART_BOX, 3, 2, grid, boxes, nullptr, nullptr, nullptr, &p) == SS_EINVAL);
        CHECK(ss_partition(&v, SS_PART_GRAPH, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr, &p) == SS_EINVAL);
        A.colidx[3] = 1000;
        v = A.view();
        CHECK(ss_partition(&v, SS_PART_GRAPH, 2, 0, nullptr, nullptr, nullptr, nullptr, nullptr, &p) == SS_EINVAL);
        CHECK(p == nullptr);
    }
    // every storage variant was exercised
    CHECK(g_dict_chunks > 0 && g_wdict_chunks > 0 && g_wide_chunks > 0 && g_narrow_chunks > 0 && g_csr_layouts > 0);
    std::printf("chunks checked: %lld with offset dictionaries, %lld with wide (several-batch) dictionaries, "
                "%lld with 16-bit columns, %lld with int32 columns; %lld CSR layouts\n", (long long)g_dict_chunks,
                (long long)g_wdict_chunks, (long long)g_narrow_chunks, (long long)g_wide_chunks,
                (long long)g_csr_layouts);
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
