"""Offset-dictionary chunks of the pipelined SpMV, through the C-ABI.

The dictionaries are used when every chunk is one batch of at most 8 entries
(rows of 5, 7 and 8 entries here: with 8 the row length is read as usual,
with fewer it rides in the dictionary word)
and each SpMV workgroup gets at least 24 chunks; a small `spmv_grid` brings
small matrices there, so that the dictionary chunks, the other chunks of the
same workgroup ranges and the switch between the two loops all run at test
sizes.  The product is bitwise the oracle's (columns are rebuilt exactly), and
the solves meet the plain-CG bars."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import paper_2108_13162_amd as ss
from workloads import CSR, diffusion3d_lognormal, poisson2d, poisson3d, uniform_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _eight_per_row(m):
    """The 7-point Laplacian on m^3 plus one diagonal coupling per node: a node
    with even x couples to (x+1, y+1, z), so interior rows hold 8 entries (9
    distinct column offsets in a chunk) and the dictionary chunks take all 8
    slots of their words, with no room for the row length."""
    A = poisson3d(m)
    S = sp.csr_matrix((A.val, A.colidx, A.rowptr), shape=(A.n, A.n))
    ids = np.arange(A.n)
    x, y = ids % m, (ids // m) % m
    i = ids[(x % 2 == 0) & (x + 1 < m) & (y + 1 < m)]
    j = i + 1 + m
    C = sp.coo_matrix((np.full(i.size, -1.0), (i, j)), shape=S.shape)
    D = sp.coo_matrix((np.ones(2 * i.size), (np.r_[i, j], np.r_[i, j])), shape=S.shape)
    S = (S + C + C.T + D).tocsr()
    S.sort_indices()
    return CSR(A.n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))


def _systems():
    A3 = diffusion3d_lognormal(40, seed=21, sigma=1.0)
    A2 = poisson2d(200)
    A8 = _eight_per_row(40)
    return [
        ("lognormal 40^3, 8 boxes", A3, O.box_partition((40, 40, 40), (2, 2, 2)), 8, (40, 40, 40), (2, 2, 2)),
        ("Poisson 200^2, 4 boxes", A2, O.box_partition((200, 200), (2, 2)), 4, (200, 200), (2, 2)),
        ("8 entries a row, 40^3, 8 boxes", A8, O.box_partition((40, 40, 40), (2, 2, 2)), 8, (40, 40, 40), (2, 2, 2)),
    ]


def test_eight_per_row_system():
    # the system the U = 8 dictionary cases run on: rows of at most 8 entries,
    # most of them full, symmetric and diagonally dominant
    A = _systems()[2][1]
    lens = np.diff(A.rowptr)
    assert lens.max() == 8 and (lens == 8).mean() > 0.4
    S = sp.csr_matrix((A.val, A.colidx, A.rowptr), shape=(A.n, A.n))
    assert abs(S - S.T).max() == 0
    assert np.all(S.diagonal() >= abs(S).sum(axis=1).A1 - S.diagonal())


def _bytes(s):
    return ss.ss_cg_time_spmv(s, 2)[1]


# grids leaving each workgroup at least 24 chunks (1000, 625 and 1000 chunks)
@pytest.mark.parametrize("which,grid", [(0, 8), (0, 16), (0, 40), (1, 8), (1, 16), (1, 24), (2, 8), (2, 16), (2, 40)])
def test_dictionary_apply_and_solve(which, grid):
    name, A, part, P, g, boxes = _systems()[which]
    p = ss.ss_partition(A, ss.SS_PART_BOX, P, grid=g, boxes=boxes)
    s = ss.ss_cg_setup(A, p, ss.default_opts(spmv_grid=grid))
    plain = ss.ss_cg_setup(A, p, ss.default_opts(spmv_grid=1024))  # too few chunks a workgroup
    # the dictionaries are in use: the CG step reads less column data
    assert _bytes(s) < _bytes(plain), name
    sd = O.split(A.rowptr, A.colidx, part, P)
    rng = np.random.default_rng(grid)
    for x in (rng.standard_normal(A.n), rng.integers(-4, 5, A.n).astype(np.float64)):
        y = ss.ss_cg_apply(s, torch.tensor(x, device=DEV)).cpu().numpy()
        assert np.array_equal(y, O.ss_spmv(A, sd, x)), name
    b = uniform_rhs(A.n, 31)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, torch.tensor(b, device=DEV), x, tol=1e-10, maxit=5000)
    xo, ro = O.ss_cg(A, sd, b, tol=1e-10, maxit=5000, hist=False)
    # a coarse grid groups the dot-product partials differently from the
    # oracle's sequential sums; on the ill-conditioned lognormal system that
    # moves CG's count by a few per cent (557 vs 562 measured at grid 8)
    assert r.status == ss.SS_OK
    assert abs(r.iterations - ro.iterations) <= max(2, 0.02 * ro.iterations), (r.iterations, ro.iterations)
    true = np.linalg.norm(b - O.csr_matvec(A, x.cpu().numpy())) / np.linalg.norm(b)
    assert true <= 1e-10, true


@pytest.mark.parametrize("prec", [ss.SS_FP32_RU, ss.SS_FP32_IR])
def test_dictionary_fp32_modes(prec):
    # the FP32 inner CG runs the same dictionary chunks with FP32 values
    name, A, part, P, g, boxes = _systems()[0]
    p = ss.ss_partition(A, ss.SS_PART_BOX, P, grid=g, boxes=boxes)
    s = ss.ss_cg_setup(A, p, ss.default_opts(spmv_grid=16, precision=prec))
    b = uniform_rhs(A.n, 32)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, torch.tensor(b, device=DEV), x, tol=1e-10, maxit=20000)
    assert r.status == ss.SS_OK, r.status
    true = np.linalg.norm(b - O.csr_matvec(A, x.cpu().numpy())) / np.linalg.norm(b)
    assert true <= 1e-10, true
    xr = O.solve_reference(A, b)
    assert np.linalg.norm(x.cpu().numpy() - xr) / np.linalg.norm(xr) <= 1e-7
