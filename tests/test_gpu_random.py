"""Randomized apply parity through the C-ABI: random SPD matrices (1 to 80k
rows; the large ones couple rows far apart, so their chunks take int32
columns), random partitions given as part arrays (1 to 9 parts, some empty,
scattered or in contiguous blocks), both storage formats, integer and float
data.  The sub-structured product must equal the oracle's on the same
partition bit for bit: both sides round each product, add a local row left to
right in column order and add an interface node's copies in ascending
sub-domain order."""
import numpy as np
import pytest

import oracle as O
import paper_2108_13162_amd as ss
from workloads import random_spd_csr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(40000, 80000)) if seed % 6 == 5 else int(rng.integers(1, 3000))
    A = random_spd_csr(n, float(rng.uniform(0.0, 12.0)), seed=2000 + seed, integer=seed % 3 == 0)
    P = int(rng.integers(1, 10))
    part = rng.integers(0, P, size=n).astype(np.int32)
    if seed % 5 == 4 and P > 1:
        part[part == P // 2] = 0  # an empty part in the middle
    if seed % 2 == 0:
        part = np.sort(part)  # contiguous blocks: few interface nodes
    fmt = ss.SS_MAT_CSR if seed % 4 == 3 else ss.SS_MAT_SELL
    return A, P, part, fmt


@pytest.mark.parametrize("seed", range(30))
def test_random_apply_bitwise(seed):
    A, P, part, fmt = _case(seed)
    p = ss.ss_partition(A, ss.SS_PART_USER, P, user_part=part)
    s = ss.ss_cg_setup(A, p, ss.default_opts(matrix_format=fmt))
    sd = O.split(A.rowptr, A.colidx, part, P)
    rng = np.random.default_rng(seed)
    for x in (rng.standard_normal(A.n), rng.integers(-5, 6, A.n).astype(np.float64)):
        y = ss.ss_cg_apply(s, torch.tensor(x, device=DEV)).cpu().numpy()
        want = O.ss_spmv(A, sd, x)
        assert np.array_equal(y, want), (seed, A.n, P, fmt, float(np.max(np.abs(y - want))))


@pytest.mark.parametrize("seed", range(12))
def test_random_solve(seed):
    # CG to 1e-10 on the same random systems and partitions: the oracle's
    # sub-structured CG on the same partition sets the iteration count (the
    # two differ only in dot-product summation order) and the error floor
    A, P, part, fmt = _case(seed)
    p = ss.ss_partition(A, ss.SS_PART_USER, P, user_part=part)
    s = ss.ss_cg_setup(A, p, ss.default_opts(matrix_format=fmt))
    sd = O.split(A.rowptr, A.colidx, part, P)
    b = np.random.default_rng(100 + seed).uniform(-1.0, 1.0, A.n)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, torch.tensor(b, device=DEV), x, tol=1e-10, maxit=5000)
    xo, ro = O.ss_cg(A, sd, b, tol=1e-10, maxit=5000, hist=False)
    assert r.status == ss.SS_OK and ro.status == O.OK
    assert abs(r.iterations - ro.iterations) <= 2, (r.iterations, ro.iterations)
    xg = x.cpu().numpy()
    true = np.linalg.norm(b - O.csr_matvec(A, xg)) / np.linalg.norm(b)
    assert true <= 1e-10, true
    xr = O.solve_reference(A, b)
    err = np.linalg.norm(xg - xr) / np.linalg.norm(xr)
    err_o = np.linalg.norm(xo - xr) / np.linalg.norm(xr)
    assert err <= max(1e-9, 10 * err_o), (err, err_o)
