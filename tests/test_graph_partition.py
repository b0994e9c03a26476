"""SS_PART_GRAPH: multilevel graph partitioning of matrices without
coordinates (CPU only).

The paper partitions with METIS, which is not available; the library's
partitioner is a heuristic with no oracle counterpart.  It is pinned to what
graph theory fixes: every node in one part, the balance bound it promises,
cuts within a small factor of the known optimum on grids (and exactly optimal
where that is forced), far below a random partition's, determinism.  Its
output then feeds the same owner-rule split as every other method, checked
bit-exact against the oracle's split of the same partition."""
import math

import numpy as np
import pytest

import oracle as O
import paper_2108_13162_amd as ss
from workloads import CSR, config, diffusion3d_lognormal, poisson2d, random_spd_csr


def _cut(A, part):
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    return int(np.sum(part[rows] != part[A.colidx]) // 2)


def _graph_part(A, k, weights=None):
    p = ss.ss_partition(A, ss.SS_PART_GRAPH, k, weights=weights)
    return p, ss.ss_part_export(p)["part"]


def _balance_bound(k):
    # 1% per bisection level, plus one vertex of rounding per level
    return 1.01 ** math.ceil(math.log2(k)) if k > 1 else 1.0


def _chain(n):
    D = np.diag(np.full(n, 2.0)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)
    rows, cols = np.nonzero(D)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return CSR(n, np.cumsum(rp).astype(np.int32), cols.astype(np.int32), D[rows, cols])


@pytest.mark.parametrize("name,k", [("p64", 2), ("p64", 4), ("p64", 7), ("d24", 8), ("rnd", 5), ("hex", 16)])
def test_valid_and_balanced(name, k):
    A = {"p64": lambda: poisson2d(64), "d24": lambda: diffusion3d_lognormal(24, 2),
         "rnd": lambda: random_spd_csr(3000, 6.0, 4), "hex": lambda: config(3, size=24).A}[name]()
    _, part = _graph_part(A, k)
    assert part.shape == (A.n,) and part.min() >= 0 and part.max() < k
    sizes = np.bincount(part, minlength=k)
    assert sizes.min() > 0
    assert sizes.max() <= _balance_bound(k) * A.n / k + math.ceil(math.log2(k)) + 1, sizes


def test_cut_near_optimal_on_grids():
    # 64 x 64 grid: 2 parts need 64 cut edges, 4 parts 128 (2 x 2 boxes)
    A = poisson2d(64)
    assert _cut(A, _graph_part(A, 2)[1]) <= 1.2 * 64
    assert _cut(A, _graph_part(A, 4)[1]) <= 1.3 * 128
    # 24^3 grid into 8: 2 x 2 x 2 boxes cut 3 * 24^2 = 1728 edges
    B = diffusion3d_lognormal(24, 2)
    assert _cut(B, _graph_part(B, 8)[1]) <= 1.3 * 1728


def test_chain_is_cut_into_segments():
    # a path of 1000 nodes: k parts need k - 1 cut edges
    A = _chain(1000)
    for k in (2, 4, 5):
        _, part = _graph_part(A, k)
        assert _cut(A, part) == k - 1, k


def test_far_below_random_partition():
    A = random_spd_csr(4000, 8.0, 6)
    _, part = _graph_part(A, 8)
    rnd = np.random.default_rng(0).integers(0, 8, A.n)
    assert _cut(A, part) < 0.7 * _cut(A, rnd)
    G = diffusion3d_lognormal(20, 3)
    _, part = _graph_part(G, 8)
    rnd = np.random.default_rng(1).integers(0, 8, G.n)
    assert _cut(G, part) < 0.1 * _cut(G, rnd)


def test_deterministic():
    A = config(3, size=20).A
    a = _graph_part(A, 6)[1]
    b = _graph_part(A, 6)[1]
    assert np.array_equal(a, b)


def test_disconnected_components_are_not_cut():
    # two disjoint 32 x 32 grids: the 2-way cut is 0
    P = poisson2d(32)
    n = P.n
    rp = np.concatenate([P.rowptr, P.rowptr[1:] + P.rowptr[-1]]).astype(np.int32)
    ci = np.concatenate([P.colidx, P.colidx + n]).astype(np.int32)
    A = CSR(2 * n, rp, ci, np.concatenate([P.val, P.val]))
    _, part = _graph_part(A, 2)
    assert _cut(A, part) == 0
    assert np.bincount(part).tolist() == [n, n]


def test_edgeless_matrix():
    n = 1000
    A = CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, 3.0))
    _, part = _graph_part(A, 8)
    sizes = np.bincount(part, minlength=8)
    assert sizes.min() > 0 and sizes.max() <= _balance_bound(8) * n / 8 + 4


def test_part_weights():
    A = poisson2d(64)
    w = np.array([1.0, 2.0, 3.0, 2.0])
    _, part = _graph_part(A, 4, weights=w)
    sizes = np.bincount(part, minlength=4)
    want = A.n * w / w.sum()
    assert np.all(np.abs(sizes - want) <= 0.04 * want + 3), (sizes, want)
    with pytest.raises(ss.SSError):
        _graph_part(A, 4, weights=np.array([1.0, -1.0, 1.0, 1.0]))


@pytest.mark.parametrize("k", [1, 3, 8])
def test_split_of_graph_partition_matches_oracle(k):
    # the owner-rule split and interface maps of a GRAPH partition, bit-exact
    A = config(3, size=16).A
    p, part = _graph_part(A, k)
    e = ss.ss_part_export(p)
    sd = O.split(A.rowptr, A.colidx, part, k)
    for key in ("sub_off", "n_int", "n_own", "l2g", "gamma", "copy_ptr", "copy_pos"):
        assert np.array_equal(e[key], getattr(sd, key)), key


def test_one_node_per_part_and_single_node():
    A = poisson2d(4)
    _, part = _graph_part(A, A.n)
    assert sorted(part.tolist()) == list(range(A.n))
    one = CSR(1, np.array([0, 1], dtype=np.int32), np.array([0], dtype=np.int32), np.array([2.0]))
    p, part = _graph_part(one, 1)
    assert part.tolist() == [0] and ss.ss_part_sizes(p)["n_gamma"] == 0
