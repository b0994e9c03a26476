"""The one-launch solve of small systems (SS_PATH_SMALL) against the oracle
and against the streaming path of the same solver options.

One workgroup runs Algorithm 3 (M = I) with the matrix in registers and x, r,
p in LDS.  Its products are the same row sums as the other kernels (stored
column order, separately rounded products and sums); the dot products are
sums over all positions in another fixed order, so iterates agree with the
oracle within the spread that the summation order alone causes."""
import numpy as np
import pytest

import oracle as O
import paper_2108_13162_amd as ss
from workloads import CSR, config, diffusion3d_lognormal, poisson2d, random_spd_csr, uniform_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _solve(s, b, x0=None, **kw):
    x = _t(x0) if x0 is not None else torch.zeros(len(b), dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, _t(b), x, **kw)
    return x.cpu().numpy(), r


def _case(kind):
    """(name, A, library partition, oracle sub-domains)"""
    if kind == "cfg1":
        w = config(1)  # 64 x 64 Poisson, 2 x 2 boxes: 4224 positions, 6 rows a thread
        return "poisson64_box2x2", w.A, ss.partition_workload(w), O.split(
            w.A.rowptr, w.A.colidx, O.box_partition(w.grid, w.boxes), 4)
    if kind.startswith("p2d"):
        m = int(kind[3:])
        A = poisson2d(m)
        return kind, A, ss.ss_partition(A, ss.SS_PART_BOX, 6, grid=(m, m), boxes=(3, 2)), O.split(
            A.rowptr, A.colidx, O.box_partition((m, m), (3, 2)), 6)
    if kind.startswith("d3d"):
        M = int(kind[3:])
        A = diffusion3d_lognormal(M, seed=M)
        return kind, A, ss.ss_partition(A, ss.SS_PART_BOX, 8, grid=(M, M, M), boxes=(2, 2, 2)), O.split(
            A.rowptr, A.colidx, O.box_partition((M, M, M), (2, 2, 2)), 8)
    if kind == "random":
        A = random_spd_csr(900, 3.0, seed=12)
        A = _trim(A, 7)
        part = np.random.default_rng(12).integers(0, 5, A.n).astype(np.int32)
        return kind, A, ss.ss_partition(A, ss.SS_PART_USER, 5, user_part=part), O.split(
            A.rowptr, A.colidx, part, 5)
    raise ValueError(kind)


def _trim(A, width):
    """Keep the diagonal and the off-diagonals of the first columns so that
    every row holds at most `width` entries, symmetrically, and restore
    diagonal dominance."""
    D = A.to_dense()
    n = A.n
    keep = np.zeros_like(D, dtype=bool)
    cnt = np.ones(n, dtype=int)
    for i in range(n):
        keep[i, i] = True
        for j in np.nonzero(D[i])[0]:
            if j > i and cnt[i] < width and cnt[j] < width:
                keep[i, j] = keep[j, i] = True
                cnt[i] += 1
                cnt[j] += 1
    D = np.where(keep, D, 0.0)
    np.fill_diagonal(D, 0.0)
    np.fill_diagonal(D, np.abs(D).sum(1) + 1.0)
    rows, cols = np.nonzero(D)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return CSR(n, np.cumsum(rp).astype(np.int32), cols.astype(np.int32), D[rows, cols])


KINDS = ["cfg1", "p2d8", "p2d31", "p2d45", "p2d60", "d3d8", "d3d12", "d3d14", "random"]


@pytest.fixture(scope="module")
def cases():
    return {k: _case(k) for k in KINDS}


def test_small_path_is_chosen(cases):
    for k, (name, A, p, sd) in cases.items():
        s = ss.ss_cg_setup(A, p)
        assert s.path() == ss.SS_PATH_SMALL, name
        assert ss.ss_cg_setup(A, p, ss.default_opts(small_solver=ss.SS_SMALL_OFF)).path() == ss.SS_PATH_STREAM
    # not chosen: larger systems, other precisions, the preconditioner
    w = config(5, size=24)
    p = ss.partition_workload(w)
    assert ss.ss_cg_setup(w.A, p).path() == ss.SS_PATH_STREAM
    name, A, p, sd = cases["cfg1"]
    assert ss.ss_cg_setup(A, p, ss.default_opts(precision=ss.SS_FP32_RU)).path() == ss.SS_PATH_STREAM
    assert ss.ss_cg_setup(A, p, ss.default_opts(precond=ss.SS_PRECOND_JACOBI)).path() == ss.SS_PATH_STREAM
    with pytest.raises(ss.SSError):
        ss.ss_cg_setup(A, p, ss.default_opts(small_solver=7))


def _hist_diff(h, ref):
    # residual estimates below 1e-13 are rounding noise once CG has converged
    m = ref > 1e-13
    return np.max(np.abs(h[m] - ref[m]) / ref[m])


def _spread(A, sd, b, k):
    xg, rg = O.cg(A, b, tol=0.0, maxit=k)
    xs, rs = O.ss_cg(A, sd, b, tol=0.0, maxit=k)
    return np.linalg.norm(xg - xs) / np.linalg.norm(xs), _hist_diff(rg.hist, rs.hist)


@pytest.mark.parametrize("k", [1, 10, 50])
def test_fixed_k_iterates_match_oracle(cases, k):
    for kind, (name, A, p, sd) in cases.items():
        b = uniform_rhs(A.n, 40 + k)
        s = ss.ss_cg_setup(A, p)
        x, r = _solve(s, b, tol=0.0, maxit=k, hist=True)
        xo, ro = O.ss_cg(A, sd, b, tol=0.0, maxit=k)
        assert r.status == ss.SS_NOT_CONVERGED and r.iterations == ro.iterations == k, name
        dx_o, dh_o = _spread(A, sd, b, k)
        dx = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        dh = _hist_diff(r.hist, ro.hist)
        assert dx <= max(1e-12, 10 * dx_o), (name, dx, dx_o)
        assert dh <= max(1e-12, 10 * dh_o), (name, dh, dh_o)
        # against the oracle with Dot2 dot products: no further than either
        # sequential oracle order (2x margin, 1e-15 floor)
        xd, _ = O.ss_cg_dot2(A, sd, b, tol=0.0, maxit=k)
        nd = np.linalg.norm(xd)
        e_gpu = np.linalg.norm(x - xd) / nd
        e_seq = max(np.linalg.norm(xo - xd) / nd, np.linalg.norm(O.cg(A, b, tol=0.0, maxit=k)[0] - xd) / nd)
        print(f"{name} k={k}: to the Dot2 oracle: gpu {e_gpu:.2e}, sequential orders up to {e_seq:.2e}")
        assert e_gpu <= max(1e-15, 2 * e_seq), (name, e_gpu, e_seq)


def test_solves_match_oracle_and_stream_path(cases):
    for kind, (name, A, p, sd) in cases.items():
        b = uniform_rhs(A.n, 3)
        s = ss.ss_cg_setup(A, p)
        x, r = _solve(s, b, tol=1e-10, maxit=20000, hist=True)
        xo, ro = O.ss_cg(A, sd, b, tol=1e-10, maxit=20000)
        true = np.linalg.norm(b - O.csr_matvec(A, x)) / np.linalg.norm(b)
        assert r.status == ss.SS_OK and true <= 1e-10, (name, r, true)
        assert abs(r.relres - true) <= 1e-6 * true + 1e-16
        assert abs(r.iterations - ro.iterations) <= 2, (name, r.iterations, ro.iterations)
        ref = O.solve_reference(A, b)
        err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
        erro = np.linalg.norm(xo - ref) / np.linalg.norm(ref)
        assert err <= max(1e-9, 2 * erro), (name, err, erro)
        assert len(r.hist) == r.iterations + 1 and np.all(np.isfinite(r.hist))
        # the streaming path of the same matrix: the same method
        s2 = ss.ss_cg_setup(A, p, ss.default_opts(small_solver=ss.SS_SMALL_OFF))
        x2, r2 = _solve(s2, b, tol=1e-10, maxit=20000)
        assert r2.status == ss.SS_OK and abs(r2.iterations - r.iterations) <= 2
        # bitwise reproducible run to run
        x3, r3 = _solve(s, b, tol=1e-10, maxit=20000, hist=True)
        assert np.array_equal(x3, x) and r3.iterations == r.iterations and np.array_equal(r3.hist, r.hist)


def test_tight_tolerance_accuracy(cases):
    name, A, p, sd = cases["cfg1"]
    b = uniform_rhs(A.n, 101)
    x, r = _solve(ss.ss_cg_setup(A, p), b, tol=1e-13, maxit=20000)
    ref = O.solve_reference(A, b)
    assert r.status == ss.SS_OK and np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_edge_cases(cases):
    name, A, p, sd = cases["p2d31"]
    s = ss.ss_cg_setup(A, p)
    n = A.n
    # b = 0: x = 0 after 0 iterations
    x, r = _solve(s, np.zeros(n), x0=np.ones(n), tol=1e-10)
    assert r.status == ss.SS_OK and r.iterations == 0 and not x.any() and r.relres == 0.0
    b = uniform_rhs(n, 8)
    # maxit 0 and 1
    x, r = _solve(s, b, tol=1e-10, maxit=0)
    assert r.status == ss.SS_NOT_CONVERGED and r.iterations == 0 and not x.any()
    x, r = _solve(s, b, tol=1e-10, maxit=1, hist=True)
    xo, ro = O.ss_cg(A, sd, b, tol=1e-10, maxit=1)
    assert r.status == ss.SS_NOT_CONVERGED and r.iterations == 1
    assert np.linalg.norm(x - xo) <= 1e-13 * np.linalg.norm(xo)
    # converged initial guess: no iteration
    xs, _ = O.ss_cg(A, sd, b, tol=1e-13, maxit=20000)
    x, r = _solve(s, b, x0=xs, tol=1e-10)
    assert r.status == ss.SS_OK and r.iterations == 0 and np.array_equal(x, xs)
    # NaN in b: breakdown
    bn = b.copy()
    bn[5] = np.nan
    _, r = _solve(s, bn, tol=1e-10)
    assert r.status == ss.SS_EBREAKDOWN
    # an indefinite matrix: (p, A p) <= 0
    neg = CSR(A.n, A.rowptr, A.colidx, -A.val)
    pn = ss.ss_partition(neg, ss.SS_PART_BOX, 6, grid=(31, 31), boxes=(3, 2))
    sn = ss.ss_cg_setup(neg, pn)
    assert sn.path() == ss.SS_PATH_SMALL
    _, r = _solve(sn, b, tol=1e-10)
    assert r.status == ss.SS_EBREAKDOWN
    # a 1 x 1 system: one iteration
    one = CSR(1, np.array([0, 1], dtype=np.int32), np.array([0], dtype=np.int32), np.array([4.0]))
    s1 = ss.ss_cg_setup(one, ss.ss_partition(one, ss.SS_PART_USER, 1, user_part=np.zeros(1)))
    assert s1.path() == ss.SS_PATH_SMALL
    x, r = _solve(s1, np.array([2.0]), tol=1e-14)
    assert r.status == ss.SS_OK and r.iterations == 1 and x[0] == 0.5


def test_set_values_reaches_the_one_launch_solve(cases):
    # new values (same pattern): the one-launch solve uses them -- bitwise the
    # solve of a solver set up on the new matrix
    name, A, p, sd = cases["d3d12"]
    d = np.random.default_rng(2).uniform(0.5, 2.0, A.n)
    rows = A.row_of_nz()
    A2 = CSR(A.n, A.rowptr, A.colidx, d[rows] * A.val * d[A.colidx])
    b = uniform_rhs(A.n, 4)
    s = ss.ss_cg_setup(A, p)
    ss.ss_cg_set_values(s, _t(A2.val))
    x, r = _solve(s, b, tol=1e-10, maxit=5000)
    s2 = ss.ss_cg_setup(A2, p)
    assert s2.path() == s.path() == ss.SS_PATH_SMALL
    x2, r2 = _solve(s2, b, tol=1e-10, maxit=5000)
    assert r.status == ss.SS_OK and r.iterations == r2.iterations and np.array_equal(x, x2)
    assert np.linalg.norm(b - O.csr_matvec(A2, x)) <= 1e-10 * np.linalg.norm(b)


def test_setup_rejects_another_pattern():
    # same n and nnz, different pattern: a 6 x 4 grid against a 4 x 6 one
    A = poisson2d(6, 4)
    B = poisson2d(4, 6)
    assert A.n == B.n and A.nnz == B.nnz and not np.array_equal(A.colidx, B.colidx)
    p = ss.ss_partition(A, ss.SS_PART_GRAPH, 2)
    with pytest.raises(ss.SSError) as e:
        ss.ss_cg_setup(B, p)
    assert e.value.code == ss.SS_EINVAL
    ss.ss_cg_setup(A, p)  # the matrix it was built from is accepted
