// Graph partitioning for matrices given without coordinates (SS_PART_GRAPH).
//
// The paper partitions with METIS (Section 3.4): sub-domains of balanced
// size with a small boundary.  This is a multilevel recursive bisection of
// the adjacency graph of A after Karypis and Kumar's published scheme, in
// three phases per bisection:
//   1. coarsening: vertices are paired along their heaviest edge to an
//      unpaired neighbour (visit order from a seeded generator), pairs
//      merged (vertex weights and parallel edge weights added), repeated
//      until the graph is small or stops shrinking;
//   2. initial bisection of the coarsest graph: from several seed vertices,
//      grow side 0 by repeatedly taking the vertex whose move cuts the least
//      edge weight, until side 0 holds its target weight; refine; keep the
//      best;
//   3. uncoarsening: project the bisection level by level and refine it with
//      Fiduccia-Mattheyses passes (move the best-gain boundary vertex that
//      keeps both sides within their weight bound, lock it, keep the best
//      prefix of the moves).
// k parts: bisect with target fractions floor(k/2) : ceil(k/2) (or the
// given part weights), then each side recursively.  Deterministic: the same
// matrix, part count and weights give the same partition.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <queue>
#include <tuple>
#include <vector>

#include "ss_internal.h"

namespace ss {
namespace {

struct Graph {
    int32_t n = 0;
    std::vector<int64_t> xadj;  // [n+1]
    std::vector<int32_t> adj;   // neighbours
    std::vector<int64_t> ew;    // edge weights
    std::vector<int64_t> vw;    // vertex weights
    int64_t total = 0;
};

// xorshift64* (Vigna): a small, fixed generator for the visit orders
struct Rng {
    uint64_t s;
    uint64_t next()
    {
        s ^= s >> 12;
        s ^= s << 25;
        s ^= s >> 27;
        return s * 2685821657736338717ull;
    }
    int32_t below(int32_t m) { return (int32_t)(next() % (uint64_t)m); }
};

constexpr int32_t kCoarsest = 128;  // stop coarsening below this many vertices
constexpr double kImbalance = 1.01; // a side may exceed its target by 1% (3% over three levels)

// 1. heavy-edge matching; cmap[u] = coarse vertex, returns the coarse count
int32_t match_heavy_edges(const Graph &G, Rng &rng, int64_t maxvw, std::vector<int32_t> &cmap)
{
    const int32_t n = G.n;
    std::vector<int32_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    for (int32_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[rng.below(i + 1)]);
    std::vector<int32_t> mate(n, -1);
    for (int32_t u : perm) {
        if (mate[u] >= 0) continue;
        int32_t best = -1;
        int64_t bw = -1;
        for (int64_t e = G.xadj[u]; e < G.xadj[u + 1]; ++e) {
            const int32_t v = G.adj[e];
            if (mate[v] < 0 && v != u && G.vw[u] + G.vw[v] <= maxvw && G.ew[e] > bw) {
                bw = G.ew[e];
                best = v;
            }
        }
        if (best < 0) {
            mate[u] = u;
        } else {
            mate[u] = best;
            mate[best] = u;
        }
    }
    cmap.assign(n, -1);
    int32_t nc = 0;
    for (int32_t u = 0; u < n; ++u)
        if (cmap[u] < 0) {
            cmap[u] = nc;
            cmap[mate[u]] = nc;
            ++nc;
        }
    return nc;
}

// merged graph: coarse vertex weights and parallel edges summed, self loops dropped
Graph contract(const Graph &G, const std::vector<int32_t> &cmap, int32_t nc)
{
    Graph C;
    C.n = nc;
    C.vw.assign(nc, 0);
    C.total = G.total;
    std::vector<int32_t> m1(nc, -1), m2(nc, -1);
    for (int32_t u = 0; u < G.n; ++u) {
        const int32_t c = cmap[u];
        C.vw[c] += G.vw[u];
        if (m1[c] < 0)
            m1[c] = u;
        else
            m2[c] = u;
    }
    C.xadj.assign((size_t)nc + 1, 0);
    C.adj.reserve(G.adj.size() / 2 + 1);
    C.ew.reserve(G.adj.size() / 2 + 1);
    std::vector<int64_t> slot(nc, -1);  // position of edge (c, cv) in C.adj, valid if >= row start
    for (int32_t c = 0; c < nc; ++c) {
        const int64_t start = (int64_t)C.adj.size();
        for (int32_t u : {m1[c], m2[c]}) {
            if (u < 0) continue;
            for (int64_t e = G.xadj[u]; e < G.xadj[u + 1]; ++e) {
                const int32_t cv = cmap[G.adj[e]];
                if (cv == c) continue;
                if (slot[cv] >= start) {
                    C.ew[slot[cv]] += G.ew[e];
                } else {
                    slot[cv] = (int64_t)C.adj.size();
                    C.adj.push_back(cv);
                    C.ew.push_back(G.ew[e]);
                }
            }
        }
        C.xadj[c + 1] = (int64_t)C.adj.size();
    }
    return C;
}

int64_t cut_of(const Graph &G, const std::vector<uint8_t> &side)
{
    int64_t cut = 0;
    for (int32_t u = 0; u < G.n; ++u)
        for (int64_t e = G.xadj[u]; e < G.xadj[u + 1]; ++e)
            if (side[u] != side[G.adj[e]]) cut += G.ew[e];
    return cut / 2;
}

// 3. Fiduccia-Mattheyses refinement of a bisection under the weight bounds
// maxw[0], maxw[1].  A state is better when it is within the bounds (or
// closer to them) and, among those, has the smaller cut.
void fm_refine(const Graph &G, std::vector<uint8_t> &side, const int64_t maxw[2], int passes)
{
    const int32_t n = G.n;
    std::vector<int64_t> id(n, 0), ed(n, 0);
    int64_t w[2] = {0, 0};
    for (int32_t u = 0; u < n; ++u) {
        w[side[u]] += G.vw[u];
        for (int64_t e = G.xadj[u]; e < G.xadj[u + 1]; ++e)
            (side[G.adj[e]] == side[u] ? id[u] : ed[u]) += G.ew[e];
    }
    int64_t cut = 0;
    for (int32_t u = 0; u < n; ++u) cut += ed[u];
    cut /= 2;
    auto excess = [&](const int64_t *ww) {
        return std::max<int64_t>(0, ww[0] - maxw[0]) + std::max<int64_t>(0, ww[1] - maxw[1]);
    };
    std::vector<uint32_t> ver(n, 0);
    std::vector<uint8_t> locked(n, 0);
    using Entry = std::tuple<int64_t, int32_t, uint32_t>;  // gain, -vertex, version
    const int32_t limit = std::max<int32_t>(25, std::min<int32_t>(n / 20, 400));
    for (int pass = 0; pass < passes; ++pass) {
        std::priority_queue<Entry> heap[2];
        for (int32_t u = 0; u < n; ++u)
            if (ed[u] > 0 || excess(w) > 0) heap[side[u]].push(Entry(ed[u] - id[u], -u, ver[u]));
        std::vector<int32_t> moves;
        int64_t best_cut = cut, best_exc = excess(w);
        size_t best_len = 0;
        int32_t since = 0;
        for (;;) {
            // the best valid entry of each side
            int32_t cand[2] = {-1, -1};
            int64_t gain[2] = {0, 0};
            for (int s = 0; s < 2; ++s)
                while (!heap[s].empty()) {
                    const auto [g, mu, vr] = heap[s].top();
                    const int32_t u = -mu;
                    if (locked[u] || side[u] != s || vr != ver[u]) {
                        heap[s].pop();
                        continue;
                    }
                    cand[s] = u;
                    gain[s] = g;
                    break;
                }
            // a side over its bound must give; otherwise the better gain whose
            // move keeps the receiving side within its bound
            int from = -1;
            for (int s = 0; s < 2; ++s)
                if (w[s] > maxw[s] && cand[s] >= 0) from = s;
            if (from < 0) {
                for (int s = 0; s < 2; ++s) {
                    if (cand[s] < 0 || w[1 - s] + G.vw[cand[s]] > maxw[1 - s]) continue;
                    if (from < 0 || gain[s] > gain[from]) from = s;
                }
            }
            if (from < 0) break;
            const int32_t u = cand[from];
            heap[from].pop();
            const int to = 1 - from;
            side[u] = (uint8_t)to;
            locked[u] = 1;
            w[from] -= G.vw[u];
            w[to] += G.vw[u];
            cut -= ed[u] - id[u];
            std::swap(id[u], ed[u]);
            for (int64_t e = G.xadj[u]; e < G.xadj[u + 1]; ++e) {
                const int32_t v = G.adj[e];
                if (side[v] == to) {
                    id[v] += G.ew[e];
                    ed[v] -= G.ew[e];
                } else {
                    id[v] -= G.ew[e];
                    ed[v] += G.ew[e];
                }
                if (!locked[v]) {
                    ++ver[v];
                    heap[side[v]].push(Entry(ed[v] - id[v], -v, ver[v]));
                }
            }
            moves.push_back(u);
            const int64_t exc = excess(w);
            if (exc < best_exc || (exc == best_exc && cut < best_cut)) {
                best_exc = exc;
                best_cut = cut;
                best_len = moves.size();
                since = 0;
            } else if (++since > limit) {
                break;
            }
        }
        // undo the moves after the best prefix
        for (size_t t = moves.size(); t > best_len; --t) {
            const int32_t u = moves[t - 1];
            const int from = side[u], to = 1 - from;
            side[u] = (uint8_t)to;
            w[from] -= G.vw[u];
            w[to] += G.vw[u];
            cut -= ed[u] - id[u];
            std::swap(id[u], ed[u]);
            for (int64_t e = G.xadj[u]; e < G.xadj[u + 1]; ++e) {
                const int32_t v = G.adj[e];
                if (side[v] == to) {
                    id[v] += G.ew[e];
                    ed[v] -= G.ew[e];
                } else {
                    id[v] -= G.ew[e];
                    ed[v] += G.ew[e];
                }
            }
        }
        for (int32_t u : moves) locked[u] = 0;
        if (best_len == 0) break;
    }
}

// 2. grow side 0 from seed until it holds target0: always take the side-1
// vertex adjacent to side 0 whose move cuts the least edge weight (when none
// is adjacent, the lowest-index side-1 vertex)
void grow_bisection(const Graph &G, int32_t seed, int64_t target0, std::vector<uint8_t> &side)
{
    const int32_t n = G.n;
    side.assign(n, 1);
    std::vector<int64_t> gain(n, 0);  // edge weight to side 0 minus to side 1
    for (int32_t u = 0; u < n; ++u)
        for (int64_t e = G.xadj[u]; e < G.xadj[u + 1]; ++e) gain[u] -= G.ew[e];
    using Entry = std::pair<int64_t, int32_t>;  // gain, -vertex
    std::priority_queue<Entry> heap;
    int32_t lowest = 0;  // no side-1 vertex below it
    int64_t w0 = 0;
    int32_t next = seed;
    while (w0 < target0) {
        while (next < 0 && !heap.empty()) {
            const auto [g, mu] = heap.top();
            heap.pop();
            if (side[-mu] == 1 && g == gain[-mu]) next = -mu;
        }
        if (next < 0) {
            while (lowest < n && side[lowest] == 0) ++lowest;
            if (lowest == n) break;
            next = lowest;
        }
        const int32_t u = next;
        next = -1;
        side[u] = 0;
        w0 += G.vw[u];
        for (int64_t e = G.xadj[u]; e < G.xadj[u + 1]; ++e) {
            const int32_t v = G.adj[e];
            gain[v] += 2 * G.ew[e];
            if (side[v] == 1) heap.push(Entry(gain[v], -v));
        }
    }
}

// multilevel bisection of G; side 0 gets the fraction f0 of the weight
std::vector<uint8_t> bisect(const Graph &G0, double f0, Rng &rng)
{
    std::vector<Graph> levels;
    std::vector<std::vector<int32_t>> maps;
    levels.push_back(G0);
    while (levels.back().n > kCoarsest) {
        const Graph &G = levels.back();
        const int64_t maxvw = std::max<int64_t>(1, (int64_t)(1.5 * (double)G.total / kCoarsest));
        std::vector<int32_t> cmap;
        const int32_t nc = match_heavy_edges(G, rng, maxvw, cmap);
        if (nc > (int32_t)(0.95 * G.n)) break;
        Graph C = contract(G, cmap, nc);
        maps.push_back(std::move(cmap));
        levels.push_back(std::move(C));
    }
    const double W = (double)G0.total;
    const int64_t t0 = (int64_t)(f0 * W + 0.5), t1 = G0.total - t0;
    auto bounds = [&](const Graph &G, int64_t *maxw) {
        int64_t vmax = 0;
        for (int64_t v : G.vw) vmax = std::max(vmax, v);
        maxw[0] = std::max<int64_t>((int64_t)(kImbalance * (double)t0), t0 + vmax);
        maxw[1] = std::max<int64_t>((int64_t)(kImbalance * (double)t1), t1 + vmax);
        // a side with a positive target keeps some weight (vertex weights >= 1)
        if (t1 > 0) maxw[0] = std::min<int64_t>(maxw[0], G.total - 1);
        if (t0 > 0) maxw[1] = std::min<int64_t>(maxw[1], G.total - 1);
    };
    // initial bisection of the coarsest graph: several seeds, the best kept
    const Graph &Cg = levels.back();
    int64_t maxw[2];
    bounds(Cg, maxw);
    std::vector<uint8_t> best, trial;
    int64_t best_cut = INT64_MAX, best_exc = INT64_MAX;
    const int trials = Cg.n > 1 ? 8 : 1;
    for (int t = 0; t < trials; ++t) {
        grow_bisection(Cg, Cg.n > 0 ? rng.below(Cg.n) : 0, t0, trial);
        fm_refine(Cg, trial, maxw, 4);
        int64_t w[2] = {0, 0};
        for (int32_t u = 0; u < Cg.n; ++u) w[trial[u]] += Cg.vw[u];
        const int64_t exc = std::max<int64_t>(0, w[0] - maxw[0]) + std::max<int64_t>(0, w[1] - maxw[1]);
        const int64_t cut = cut_of(Cg, trial);
        if (exc < best_exc || (exc == best_exc && cut < best_cut)) {
            best_exc = exc;
            best_cut = cut;
            best = trial;
        }
    }
    // project and refine level by level
    std::vector<uint8_t> side = std::move(best);
    for (size_t l = levels.size() - 1; l > 0; --l) {
        const Graph &F = levels[l - 1];
        const std::vector<int32_t> &cmap = maps[l - 1];
        std::vector<uint8_t> fine(F.n);
        for (int32_t u = 0; u < F.n; ++u) fine[u] = side[cmap[u]];
        side.swap(fine);
        bounds(F, maxw);
        fm_refine(F, side, maxw, 4);
    }
    return side;
}

// the subgraph induced by the vertices with side == s; ids[] its original ids
Graph induced(const Graph &G, const std::vector<uint8_t> &side, uint8_t s, const std::vector<int32_t> &ids,
              std::vector<int32_t> &sub_ids)
{
    std::vector<int32_t> local(G.n, -1);
    Graph H;
    sub_ids.clear();
    for (int32_t u = 0; u < G.n; ++u)
        if (side[u] == s) {
            local[u] = H.n++;
            sub_ids.push_back(ids[u]);
            H.vw.push_back(G.vw[u]);
            H.total += G.vw[u];
        }
    H.xadj.assign((size_t)H.n + 1, 0);
    for (int32_t u = 0; u < G.n; ++u) {
        if (side[u] != s) continue;
        for (int64_t e = G.xadj[u]; e < G.xadj[u + 1]; ++e)
            if (side[G.adj[e]] == s) {
                H.adj.push_back(local[G.adj[e]]);
                H.ew.push_back(G.ew[e]);
            }
        H.xadj[local[u] + 1] = (int64_t)H.adj.size();
    }
    return H;
}

void recurse(const Graph &G, const std::vector<int32_t> &ids, const std::vector<double> &tw, int32_t p0, int32_t np,
             Rng &rng, std::vector<int32_t> &part)
{
    if (np == 1 || G.n == 0) {
        for (int32_t u = 0; u < G.n; ++u) part[ids[u]] = p0;
        return;
    }
    const int32_t kl = np / 2;
    double wl = 0.0, wt = 0.0;
    for (int32_t t = 0; t < np; ++t) {
        wt += tw[p0 + t];
        if (t < kl) wl += tw[p0 + t];
    }
    const std::vector<uint8_t> side = bisect(G, wl / wt, rng);
    std::vector<int32_t> ids0, ids1;
    const Graph G0 = induced(G, side, 0, ids, ids0);
    const Graph G1 = induced(G, side, 1, ids, ids1);
    recurse(G0, ids0, tw, p0, kl, rng, part);
    recurse(G1, ids1, tw, p0 + kl, np - kl, rng, part);
}

}  // namespace

int partition_graph(const ss_csr *A, const double *weights, int32_t nparts, std::vector<int32_t> &part)
{
    std::vector<double> tw(nparts, 1.0);
    if (weights)
        for (int32_t t = 0; t < nparts; ++t) {
            if (!(weights[t] > 0.0) || !std::isfinite(weights[t]))
                return fail(SS_EINVAL, "GRAPH partition: weights must be positive and finite");
            tw[t] = weights[t];
        }
    // the adjacency graph of A: every off-diagonal stored entry an edge of weight 1
    Graph G;
    G.n = A->n;
    G.xadj.assign((size_t)A->n + 1, 0);
    G.adj.reserve((size_t)A->nnz);
    for (int32_t i = 0; i < A->n; ++i) {
        for (int32_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
            if (A->colidx[k] != i) G.adj.push_back(A->colidx[k]);
        G.xadj[i + 1] = (int64_t)G.adj.size();
    }
    G.ew.assign(G.adj.size(), 1);
    G.vw.assign(A->n, 1);
    G.total = A->n;
    std::vector<int32_t> ids(A->n);
    std::iota(ids.begin(), ids.end(), 0);
    part.assign(A->n, 0);
    Rng rng{0x9e3779b97f4a7c15ull};
    recurse(G, ids, tw, 0, nparts, rng, part);
    return SS_OK;
}

}  // namespace ss
