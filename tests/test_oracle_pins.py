"""Pins the oracle to facts fixed by the paper and by mathematics (CPU only).

Each test checks the oracle against something other than itself: the paper's
printed CSR example, closed-form partition counts, exact integer arithmetic,
a textbook/library routine (numpy's solver, Cholesky), Krylov optimality of
CG iterates, the finite-termination and Chebyshev convergence bounds of CG,
and finite differences for the adjoint gradient.
"""
import math
import os
from itertools import combinations

import numpy as np
import pytest

import oracle as O
from workloads import (CSR, config, diffusion3d_lognormal, diffusion3d_grf, grid_coords, poisson2d,
                       random_spd_csr, rcb_weights, uniform_rhs)


def _dense_to_csr(D: np.ndarray, keep_zeros: bool = False) -> CSR:
    n = D.shape[0]
    mask = np.ones_like(D, dtype=bool) if keep_zeros else (D != 0)
    rows, cols = np.nonzero(mask)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    return CSR(n, np.cumsum(rowptr).astype(np.int32), cols.astype(np.int32), D[rows, cols].astype(np.float64))


# ----------------------------------------------------------------------------
# CSR storage: the example of Section 2.2
# ----------------------------------------------------------------------------

def _read_golden(path):
    out = {"matrix": []}
    mode = None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line == "matrix":
                mode = "matrix"
                continue
            head, *rest = line.split()
            if head in ("AA", "JA", "IA", "pattern"):
                out[head] = rest
                mode = None
            elif mode == "matrix":
                out["matrix"].append([float(t) for t in line.split()])
    return out


def test_paper_csr_example(golden_dir):
    g = _read_golden(os.path.join(golden_dir, "paper_csr_example.txt"))
    D = np.array(g["matrix"])
    AA = np.array([float(t) for t in g["AA"]])
    JA = np.array([int(t) for t in g["JA"]])
    IA = np.array([int(t) for t in g["IA"]])
    n = D.shape[0]
    nnz = len(AA)
    # the paper's definition: IA(n+1) = nnz + 1, 1-based
    assert IA[-1] == nnz + 1 and len(IA) == n + 1
    # the listed pattern is the nonzero set of the printed matrix
    pat = sorted(tuple(int(v) for v in t.split("/")) for t in g["pattern"])
    assert pat == sorted((i + 1, j + 1) for i, j in zip(*np.nonzero(D)))
    # 0-based arrays, as the oracle stores them
    A = CSR(n, (IA - 1).astype(np.int32), (JA - 1).astype(np.int32), AA)
    assert np.array_equal(A.to_dense(), D)
    # matvec on integer data is exact: compare with integer matrix product
    x = np.array([3.0, -1.0, 4.0, 1.0, -5.0])
    assert np.array_equal(O.csr_matvec(A, x), (D.astype(np.int64) @ x.astype(np.int64)).astype(float))
    # every unit vector extracts a column
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        assert np.array_equal(O.csr_matvec(A, e), D[:, j])


# ----------------------------------------------------------------------------
# partitions and maps: closed forms
# ----------------------------------------------------------------------------

def test_box_4x4_2x2_by_hand():
    A = poisson2d(4)
    part = O.box_partition((4, 4), (2, 2))
    assert part.reshape(4, 4).tolist() == [[0, 0, 1, 1], [0, 0, 1, 1], [2, 2, 3, 3], [2, 2, 3, 3]]
    sd = O.split(A.rowptr, A.colidx, part, 4)
    assert np.diff(sd.sub_off).tolist() == [8, 6, 6, 4]
    assert len(sd.gamma) == 7
    assert np.bincount(sd.mult).tolist() == [0, 9, 6, 1]
    # the cross point (2,2) -> id 10 is shared by sub-domains 1, 2, 3
    g = list(sd.gamma).index(10)
    cps = sd.copy_pos[sd.copy_ptr[g]:sd.copy_ptr[g + 1]]
    owners = [int(np.searchsorted(sd.sub_off, c, side="right") - 1) for c in cps]
    assert owners == [1, 2, 3]


def test_box_64x64_2x2_counts():
    A = poisson2d(64)
    sd = O.split(A.rowptr, A.colidx, O.box_partition((64, 64), (2, 2)), 4)
    assert np.diff(sd.sub_off).tolist() == [1088, 1056, 1056, 1024]
    assert len(sd.gamma) == 127
    assert np.bincount(sd.mult).tolist() == [0, 3969, 126, 1]


@pytest.mark.parametrize("M", [5, 6, 9, 16])
def test_box_2d_closed_form(M):
    # 2 boxes per axis, cut at c = floor(M/2).  With the owner rule a node
    # joins the lower neighbour's sub-domain once per axis where it sits on
    # the first row/column of an upper box: m = 1 + #such axes.
    A = poisson2d(M)
    sd = O.split(A.rowptr, A.colidx, O.box_partition((M, M), (2, 2)), 4)
    hist = np.bincount(sd.mult, minlength=4)
    assert hist[2] == 2 * (M - 1) and hist[3] == 1
    assert sd.n_loc == M * M + hist[2] + 2 * hist[3]


@pytest.mark.parametrize("M", [4, 7, 12])
def test_box_3d_closed_form(M):
    A = diffusion3d_lognormal(M, seed=1)
    sd = O.split(A.rowptr, A.colidx, O.box_partition((M, M, M), (2, 2, 2)), 8)
    hist = np.bincount(sd.mult, minlength=5)
    for k in (1, 2, 3):
        assert hist[1 + k] == math.comb(3, k) * (M - 1) ** (3 - k)
    assert sd.n_loc == M ** 3 + sum((m - 1) * hist[m] for m in range(1, 5))


def _brute_force_split(A: CSR, part, P):
    """Set-based rendering of the owner rule, one entry at a time."""
    rows = A.row_of_nz()
    V = [set() for _ in range(P)]
    for i in range(A.n):
        V[part[i]].add(i)
    entries = [set() for _ in range(P)]
    for k in range(A.nnz):
        i, j = int(rows[k]), int(A.colidx[k])
        o = part[i] if i == j else min(part[i], part[j])
        V[o].update((i, j))
        entries[o].add(k)
    return V, entries


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_split_brute_force_random_partition(seed):
    rng = np.random.default_rng(seed)
    A = random_spd_csr(60, 4.0, seed=seed)
    P = 5
    part = rng.integers(0, P, size=A.n).astype(np.int32)
    sd = O.split(A.rowptr, A.colidx, part, P)
    V, entries = _brute_force_split(A, part, P)
    mult = np.zeros(A.n, dtype=int)
    for s in range(P):
        for i in V[s]:
            mult[i] += 1
    assert np.array_equal(sd.mult, mult)
    for s in range(P):
        loc = sd.l2g[sd.sub_off[s]:sd.sub_off[s + 1]].tolist()
        interior = sorted(i for i in V[s] if mult[i] == 1)
        owned = sorted(i for i in V[s] if mult[i] > 1 and part[i] == s)
        ghost = sorted(i for i in V[s] if mult[i] > 1 and part[i] != s)
        assert loc == interior + owned + ghost
        assert sd.n_int[s] == len(interior) and sd.n_own[s] == len(owned)
        # local matrix rows hold exactly the entries owned by s
        lo, hi = sd.sub_off[s], sd.sub_off[s + 1]
        got = sorted(sd.bd_nzmap[sd.bd_rowptr[lo]:sd.bd_rowptr[hi]].tolist())
        assert got == sorted(entries[s])


@pytest.mark.parametrize("P,how", [(4, "box"), (9, "box"), (7, "user"), (1, "box")])
def test_local_matrices_sum_to_global(P, how):
    # sum_s R_s^T A_s R_s == A, entry by entry and bitwise (Section 3.4:
    # S_33 = S_33^(1) + S_33^(2); elsewhere each entry lives in one sub-domain)
    m = 13
    A = CSR(*_lognormal2d(m))
    if how == "box":
        b = int(round(math.sqrt(P)))
        part = O.box_partition((m, m), (b, b))
    else:
        part = np.random.default_rng(3).integers(0, P, size=A.n).astype(np.int32)
    sd = O.split(A.rowptr, A.colidx, part, P)
    vbd = sd.bd_values(A.val)
    rows_bd = np.repeat(np.arange(sd.n_loc), np.diff(sd.bd_rowptr))
    G = np.zeros((A.n, A.n))
    cnt = np.zeros((A.n, A.n), dtype=int)
    np.add.at(G, (sd.l2g[rows_bd], sd.l2g[sd.bd_colidx]), vbd)
    np.add.at(cnt, (sd.l2g[rows_bd], sd.l2g[sd.bd_colidx]), 1)
    D = A.to_dense()
    assert np.array_equal(G, D)
    assert cnt.max() == 1 and cnt.sum() == A.nnz
    # every local matrix is symmetric
    L = np.zeros((sd.n_loc, sd.n_loc))
    L[rows_bd, sd.bd_colidx] = vbd
    assert np.array_equal(L, L.T)


def _lognormal2d(m):
    from workloads.generators import diffusion2d_lognormal
    A = diffusion2d_lognormal(m, np.random.default_rng(7))
    return A.n, A.rowptr, A.colidx, A.val


def test_rcb_invariants():
    M = 14
    coords = grid_coords((M, M, M))
    w = rcb_weights(16, seed=3)
    part = O.rcb_partition(coords, w)
    n = len(part)
    assert part.min() == 0 and part.max() == 15

    # recompute every bisection independently from the finished partition:
    # the left half of [lo,hi) has the expected size and lies entirely
    # before the right half along the widest axis (ties by global id)
    def check(ids, lo, hi):
        if hi - lo == 1:
            assert np.all(part[ids] == lo)
            return
        mid = (lo + hi) // 2
        sub = coords[ids]
        axis = int(np.argmax(sub.max(0) - sub.min(0)))
        left = ids[part[ids] < mid]
        right = ids[part[ids] >= mid]
        expect = int(math.floor(len(ids) * sum(w[lo:mid]) / sum(w[lo:hi]) + 0.5))
        assert len(left) == expect
        key = lambda i: (coords[i, axis], i)  # noqa: E731
        if len(left) and len(right):
            assert max(map(key, left)) < min(map(key, right))
        check(left, lo, mid)
        check(right, mid, hi)

    check(np.arange(n), 0, 16)
    sizes = np.bincount(part)
    share = sizes / n
    assert np.all(np.abs(share - w / w.sum()) < 0.01)


# ----------------------------------------------------------------------------
# sub-structured SpMV and dots on integer data: exact
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["box2x2", "box3x3", "user7", "rcb6"])
def test_ss_spmv_integer_exact(kind):
    m = 17
    A = poisson2d(m)
    if kind == "box2x2":
        part, P = O.box_partition((m, m), (2, 2)), 4
    elif kind == "box3x3":
        part, P = O.box_partition((m, m), (3, 3)), 9
    elif kind == "user7":
        part, P = np.random.default_rng(1).integers(0, 7, A.n).astype(np.int32), 7
    else:
        part, P = O.rcb_partition(grid_coords((m, m)), np.ones(6)), 6
    sd = O.split(A.rowptr, A.colidx, part, P)
    rng = np.random.default_rng(11)
    x = rng.integers(-2**20, 2**20, size=A.n)
    exact = A.to_dense().astype(np.int64) @ x
    y = O.ss_spmv(A, sd, x.astype(float))
    assert np.array_equal(y, exact.astype(float))
    # assembled copies agree on every position, not just the owned ones
    q = O.ss_spmv_local(sd, A.val, O.gather(sd, x.astype(float)))
    assert np.array_equal(q, exact[sd.l2g].astype(float))
    # weighted local dot counts every node once
    u = rng.integers(-2**15, 2**15, size=A.n)
    v = rng.integers(-2**15, 2**15, size=A.n)
    assert O.owned_dot(sd, O.gather(sd, u.astype(float)), O.gather(sd, v.astype(float))) == float(u @ v)


def test_iface_sum_order_is_ascending_subdomain():
    # values whose FP sum depends on the order: 1e16 + 1 - 1e16
    A = poisson2d(4)
    sd = O.split(A.rowptr, A.colidx, O.box_partition((4, 4), (2, 2)), 4)
    q = np.zeros(sd.n_loc)
    g = list(sd.gamma).index(10)  # copies in sub-domains 1, 2, 3
    cps = sd.copy_pos[sd.copy_ptr[g]:sd.copy_ptr[g + 1]]
    q[cps] = [1e16, 1.0, -1e16]
    out = O.iface_sum(sd, q)
    assert np.all(out[cps] == ((1e16 + 1.0) - 1e16))


# ----------------------------------------------------------------------------
# CG (Algorithm 3, M = I)
# ----------------------------------------------------------------------------

def test_cg_tiny_vs_library_and_cholesky():
    for seed in range(4):
        A = random_spd_csr(48, 5.0, seed=seed)
        b = uniform_rhs(A.n, 50 + seed)
        D = A.to_dense()
        ref = np.linalg.solve(D, b)
        xc, st = O.chol_solve(D, b)
        assert st == O.OK
        assert np.linalg.norm(xc - ref) <= 1e-13 * np.linalg.norm(ref)
        x, res = O.cg(A, b, tol=1e-14)
        assert res.status == O.OK
        assert np.linalg.norm(x - xc) <= 1e-12 * np.linalg.norm(xc)
        assert res.true_relres <= 1e-14 * 1.01


def test_cholesky_rejects_indefinite():
    D = np.array([[1.0, 2.0], [2.0, 1.0]])
    _, st = O.chol_solve(D, np.ones(2))
    assert st == O.EBREAKDOWN


@pytest.mark.parametrize("k", [1, 2, 3, 5, 7])
def test_cg_iterates_are_krylov_optimal(k):
    # x_k minimises the A-norm error over x_0 + K_k(A, r_0): the Galerkin
    # condition V^T (b - A x_k) = 0 for an orthonormal basis V of K_k.
    A = random_spd_csr(40, 6.0, seed=5)
    D = A.to_dense()
    b = uniform_rhs(A.n, 9)
    x0 = uniform_rhs(A.n, 10) * 0.1
    xk, res = O.cg(A, b, x0=x0, tol=0.0, maxit=k)
    assert res.iterations == k and res.status == O.NOT_CONVERGED
    r0 = b - D @ x0
    K = np.empty((A.n, k))
    v = r0 / np.linalg.norm(r0)
    for j in range(k):
        K[:, j] = v
        v = D @ v
        v = v / np.linalg.norm(v)
    V, _ = np.linalg.qr(K)
    y = np.linalg.solve(V.T @ D @ V, V.T @ r0)
    ref = x0 + V @ y
    assert np.linalg.norm(xk - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("eigs", [(1.0, 2.0), (1.0, 3.0, 7.0), (2.0, 5.0, 9.0, 20.0)])
def test_cg_finite_termination(eigs):
    # with k distinct eigenvalues CG reaches the exact solution in k steps
    rng = np.random.default_rng(len(eigs))
    n = 24
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.array([eigs[i % len(eigs)] for i in range(n)])
    D = (Q * lam) @ Q.T
    D = (D + D.T) / 2
    A = _dense_to_csr(D, keep_zeros=True)
    b = rng.uniform(-1, 1, n)
    x, res = O.cg(A, b, tol=1e-12, maxit=100)
    assert res.status == O.OK
    assert res.iterations == len(eigs)


def test_cg_one_by_one():
    A = CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([4.0]))
    x, res = O.cg(A, np.array([3.0]), tol=1e-14)
    assert res.iterations == 1 and x[0] == 0.75 and res.status == O.OK


def test_cg_laplacian_chebyshev_bound():
    # 2D Dirichlet 5-point Laplacian on m x m: eigenvalues
    # 4 - 2cos(i pi/(m+1)) - 2cos(j pi/(m+1)), kappa = cot^2(pi/(2(m+1))).
    # CG from x0 = 0 reaches ||r||/||b|| <= tol within
    # ceil(ln(2 sqrt(kappa)/tol) / ln((sqrt(kappa)+1)/(sqrt(kappa)-1))) steps
    # (A-norm bound turned into a residual bound with a factor sqrt(kappa)).
    m = 64
    kappa = 1.0 / math.tan(math.pi / (2 * (m + 1))) ** 2
    assert abs(kappa - 1711.7) < 0.1
    sk = math.sqrt(kappa)
    bound = math.ceil(math.log(2 * sk / 1e-10) / math.log((sk + 1) / (sk - 1)))
    assert bound == 568
    w = config(1)
    x, res = O.cg(w.A, w.b, tol=1e-10)
    assert res.status == O.OK and res.iterations <= bound
    # the spectrum formula itself, on a small grid
    ms = 9
    ev = np.linalg.eigvalsh(poisson2d(ms).to_dense())
    t = np.arange(1, ms + 1) * math.pi / (ms + 1)
    closed = np.sort((4 - 2 * np.cos(t)[:, None] - 2 * np.cos(t)[None, :]).ravel())
    assert np.allclose(ev, closed, atol=1e-12)
    # same for the sub-structured run on its 2x2 boxes
    sd = O.split(w.A.rowptr, w.A.colidx, O.box_partition(w.grid, w.boxes), 4)
    _, res2 = O.ss_cg(w.A, sd, w.b, tol=1e-10)
    assert res2.status == O.OK and res2.iterations <= bound


def test_ss_cg_p1_is_global_cg_bitwise():
    A = diffusion3d_lognormal(10, seed=4)
    b = uniform_rhs(A.n, 4)
    sd = O.split(A.rowptr, A.colidx, np.zeros(A.n, np.int32), 1)
    x1, r1 = O.cg(A, b, tol=1e-10)
    x2, r2 = O.ss_cg(A, sd, b, tol=1e-10)
    assert np.array_equal(x1, x2) and np.array_equal(r1.hist, r2.hist)
    assert r1.iterations == r2.iterations


def test_iteration_count_independent_of_subdomains():
    # Sub-structuring only regroups the SpMV and the dots: in exact arithmetic
    # the iterates are those of global CG, so one iteration count fits every
    # processor count (the paper prints a single #iter per matrix).
    M = 16
    A = diffusion3d_lognormal(M, seed=2)
    b = uniform_rhs(A.n, 102)
    counts = []
    xs = []
    for boxes in [(1, 1, 1), (2, 1, 1), (2, 2, 1), (2, 2, 2), (4, 2, 2)]:
        P = int(np.prod(boxes))
        sd = O.split(A.rowptr, A.colidx, O.box_partition((M, M, M), boxes), P)
        x, res = O.ss_cg(A, sd, b, tol=1e-10)
        assert res.status == O.OK and res.true_relres <= 1e-10
        counts.append(res.iterations)
        xs.append(x)
    assert max(counts) - min(counts) <= 2
    for x in xs[1:]:
        assert np.linalg.norm(x - xs[0]) <= 1e-8 * np.linalg.norm(xs[0])


def test_ss_cg_matches_cholesky_small():
    A = diffusion3d_grf(8, seed=5)
    b = uniform_rhs(A.n, 5)
    sd = O.split(A.rowptr, A.colidx, O.box_partition((8, 8, 8), (2, 2, 2)), 8)
    ref, st = O.chol_solve(A.to_dense(), b)
    x, res = O.ss_cg(A, sd, b, tol=1e-14)
    assert res.status == O.OK
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_cg_edge_cases():
    A = poisson2d(6)
    sd = O.split(A.rowptr, A.colidx, O.box_partition((6, 6), (2, 2)), 4)
    # b = 0 -> x = 0 after zero iterations
    x, res = O.ss_cg(A, sd, np.zeros(A.n), x0=np.ones(A.n))
    assert res.status == O.OK and res.iterations == 0 and not x.any()
    # maxit reached
    x, res = O.ss_cg(A, sd, uniform_rhs(A.n, 1), tol=1e-30, maxit=1)
    assert res.status == O.NOT_CONVERGED and res.iterations == 1
    # NaN in b
    b = uniform_rhs(A.n, 1)
    b[3] = np.nan
    _, res = O.ss_cg(A, sd, b)
    assert res.status == O.EBREAKDOWN
    # indefinite matrix: (p, Sp) <= 0 at the first step
    Ai = CSR(2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.array([1.0, -1.0]))
    _, res = O.cg(Ai, np.array([0.0, 1.0]))
    assert res.status == O.EBREAKDOWN and res.iterations == 0
    # converged initial guess
    xs = O.solve_reference(A, b=uniform_rhs(A.n, 2))
    _, res = O.ss_cg(A, sd, uniform_rhs(A.n, 2), x0=xs, tol=1e-8)
    assert res.iterations == 0 and res.status == O.OK


# ----------------------------------------------------------------------------
# FP32 values + FP64 iterative refinement
# ----------------------------------------------------------------------------

def test_fp32_spmv_exact_on_small_integers():
    A = poisson2d(9)
    x = np.random.default_rng(0).integers(-1000, 1000, A.n)
    y32 = O.csr_matvec_f32(A.rowptr, A.colidx, A.val.astype(np.float32), x.astype(np.float32))
    assert np.array_equal(y32.astype(np.int64), A.to_dense().astype(np.int64) @ x)


def _f32(v: float) -> float:
    """Round a Python float (FP64) to the nearest FP32 value, ties to even."""
    return float(np.float32(v))


def _matvec_f32_by_hand(rowptr, colidx, v32, x32):
    """An independent FP32 CSR product: every product and every running sum
    is computed in FP64 and rounded to FP32 at once.  FP64 holds the exact
    product of two FP32 numbers, and rounding an FP64 sum of two FP32 numbers
    to FP32 equals the FP32 sum (53 >= 2*24 + 2 bits: double rounding is
    innocuous for +, -, *), so this is exact FP32 arithmetic written with
    Python floats."""
    y = np.empty(len(rowptr) - 1, dtype=np.float32)
    for i in range(len(rowptr) - 1):
        s = 0.0
        for k in range(rowptr[i], rowptr[i + 1]):
            s = _f32(s + _f32(float(v32[k]) * float(x32[colidx[k]])))
        y[i] = s
    return y


def test_fp32_matvec_rounds_each_step_in_row_order():
    # 27-point Q1 stiffness with lognormal element coefficients and a random
    # FP32 vector: non-integer data, long rows, plenty of rounding
    A = config(3, size=6).A
    rng = np.random.default_rng(31)
    v32 = A.val.astype(np.float32)
    x32 = rng.uniform(-1.0, 1.0, A.n).astype(np.float32)
    y = O.csr_matvec_f32(A.rowptr, A.colidx, v32, x32)
    assert np.array_equal(y.view(np.uint32), _matvec_f32_by_hand(A.rowptr, A.colidx, v32, x32).view(np.uint32))
    # it is FP32 arithmetic, not an FP64 row sum rounded once at the end
    rows = A.row_of_nz()
    prod64 = v32.astype(np.float64) * x32.astype(np.float64)[A.colidx]
    y64 = np.array([math.fsum(prod64[A.rowptr[i]:A.rowptr[i + 1]]) for i in range(A.n)])
    assert np.count_nonzero(y != y64.astype(np.float32)) > A.n // 10
    # and it meets the recursive-summation bound gamma_k(2^-24) sum |a||x|
    k = np.diff(A.rowptr).astype(np.float64)
    u = 2.0 ** -24
    gam = k * u / (1.0 - k * u)
    absum = np.bincount(rows, weights=np.abs(prod64), minlength=A.n)
    assert np.all(np.abs(y.astype(np.float64) - y64) <= gam * absum)


def test_fp32_iface_sum_adds_copies_in_list_order():
    # one interface node with three copies: (1 + 2^-24) + 2^-24 rounds to 1 at
    # every step in FP32, 2^-24 + 2^-24 + 1 does not, and the FP64 sum of the
    # three rounded once would give 1 + 2^-23
    e = 2.0 ** -24
    q = np.array([1.0, e, e, 7.0], dtype=np.float32)
    out = O.iface_sum_f32([0, 3], [0, 1, 2], q)
    assert np.array_equal(out, np.array([1.0, 1.0, 1.0, 7.0], dtype=np.float32))
    back = O.iface_sum_f32([0, 3], [2, 1, 0], q)
    assert np.array_equal(back, np.array([1.0 + 2 * e] * 3 + [7.0], dtype=np.float32))
    assert np.float32(1.0 + 2 * e) != np.float32(1.0)
    # two nodes, copies scattered: each node gets only its own copies' sum
    q2 = np.array([0.5, 3.0, 0.25, 1.5], dtype=np.float32)
    assert np.array_equal(O.iface_sum_f32([0, 2, 4], [0, 2, 3, 1], q2),
                          np.array([0.75, 4.5, 0.75, 4.5], dtype=np.float32))


def test_fp32_owned_dot_accumulates_in_fp64():
    # FP32 inputs, FP64 products and FP64 sum over the owned positions: the
    # 2^-26 terms vanish in an FP32 accumulation (1 + 2^-26 == 1 in FP32) but
    # all stay in FP64, where this sum is exact
    sd = O.split(poisson2d(4).rowptr, poisson2d(4).colidx, O.box_partition((4, 4), (2, 2)), 4)
    own = O.owned_positions(sd)
    u = np.zeros(sd.n_loc, dtype=np.float32)
    u[own] = 2.0 ** -13
    u[own[0]] = 1.0
    u[np.setdiff1d(np.arange(sd.n_loc), own)] = 1e3   # ghost copies: not counted
    got = O.owned_dot_f32(sd, u, u)
    assert got == 1.0 + (len(own) - 1) * 2.0 ** -26
    assert np.float32(1.0) + np.float32(2.0 ** -26) == np.float32(1.0)
    # non-integer data: within gamma_n(2^-53) of the exact sum of the FP32 products
    rng = np.random.default_rng(5)
    a = rng.uniform(-1, 1, sd.n_loc).astype(np.float32)
    b = rng.uniform(-1, 1, sd.n_loc).astype(np.float32)
    prods = a[own].astype(np.float64) * b[own].astype(np.float64)
    nn = len(own)
    assert abs(O.owned_dot_f32(sd, a, b) - math.fsum(prods)) <= nn * 2.0 ** -53 / (1 - nn * 2.0 ** -53) * np.abs(prods).sum()


def test_ss_spmv_f32_is_local_products_then_assembly():
    # the FP32 sub-structured product: FP32 local row sums (pinned above), then
    # FP32 sums of the interface copies in ascending sub-domain order
    w = config(3, size=8)
    part = O.rcb_partition(w.coords, w.weights)
    sd = O.split(w.A.rowptr, w.A.colidx, part, 16)
    x32 = np.random.default_rng(9).uniform(-1, 1, w.A.n).astype(np.float32)
    y = O.ss_spmv_f32(w.A, sd, x32)
    v32 = sd.bd_values(w.A.val).astype(np.float32)
    ql = _matvec_f32_by_hand(sd.bd_rowptr, sd.bd_colidx, v32, x32[sd.l2g])
    for g in range(len(sd.gamma)):
        cps = sd.copy_pos[sd.copy_ptr[g]:sd.copy_ptr[g + 1]]
        t = 0.0
        for c in cps:
            t = _f32(t + float(ql[c]))
        ql[cps] = t
    own = O.owned_positions(sd)
    ref = np.empty(w.A.n, dtype=np.float32)
    ref[sd.l2g[own]] = ql[own]
    assert np.array_equal(y.view(np.uint32), ref.view(np.uint32))
    # within FP32 rounding of the FP64 global product
    y64 = O.csr_matvec(w.A, x32.astype(np.float64))
    absum = O.csr_matvec(CSR(w.A.n, w.A.rowptr, w.A.colidx, np.abs(w.A.val)), np.abs(x32.astype(np.float64)))
    k = 27 + 8
    assert np.all(np.abs(y - y64) <= (k * 2.0 ** -24 / (1 - k * 2.0 ** -24)) * absum * 1.01 + 1e-30)


def _exact_dot(u, v):
    from fractions import Fraction
    return sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(u, v))


def test_dot2_error_bound_and_cancellation():
    # Dot2 (Ogita, Rump, Oishi 2005): |res - x'y| <= u |x'y| + gamma_n^2 |x|'|y|
    rng = np.random.default_rng(17)
    u = 2.0 ** -53
    for n, scale in ((1, 1.0), (7, 1.0), (500, 1e3), (2000, 1.0)):
        a = rng.uniform(-1, 1, n) * scale
        b = rng.uniform(-1, 1, n)
        ex = _exact_dot(a, b)
        g = n * u / (1 - n * u)
        bound = u * abs(float(ex)) + g * g * float(np.abs(a) @ np.abs(b))
        assert abs(O.dot2(a, b) - float(ex)) <= bound
    # a sum that cancels: the plain left-to-right dot loses everything, Dot2 is exact
    a = np.array([1e16, 1.0, -1e16, 3.0, 1e-3])
    b = np.array([1.0, 1.0, 1.0, 1.0, 1e-3])
    assert O.dot(a, b) != float(_exact_dot(a, b))
    assert O.dot2(a, b) == float(_exact_dot(a, b))
    # ill-conditioned random dots (condition ~1e12): still within the bound
    x = rng.uniform(-1, 1, 300)
    y = rng.uniform(-1, 1, 300)
    x[0], y[0] = 1e12, 1e12 * 0 + 1.0
    x[1], y[1] = -1e12, 1.0
    ex = _exact_dot(x, y)
    g = 300 * u / (1 - 300 * u)
    assert abs(O.dot2(x, y) - float(ex)) <= u * abs(float(ex)) + g * g * float(np.abs(x) @ np.abs(y))


def test_owned_dot2_counts_owned_positions_once():
    A = diffusion3d_lognormal(6, seed=4)
    sd = O.split(A.rowptr, A.colidx, O.box_partition((6, 6, 6), (2, 2, 2)), 8)
    rng = np.random.default_rng(1)
    xg, yg = rng.uniform(-1, 1, A.n), rng.uniform(-1, 1, A.n)
    got = O.owned_dot2(sd, O.gather(sd, xg), O.gather(sd, yg))
    ex = _exact_dot(xg, yg)  # each node counted once: the global dot
    g = A.n * 2.0 ** -53
    assert abs(got - float(ex)) <= 2.0 ** -53 * abs(float(ex)) + g * g * float(np.abs(xg) @ np.abs(yg))


def test_cg_dot2_is_cg():
    # the CG of Algorithm 3 with Dot2 dots: P = 1 equals the unsplit CG bit
    # for bit, solves match Cholesky, the Laplacian meets its Chebyshev bound,
    # and the count does not depend on the sub-domains
    M = 10
    A = diffusion3d_lognormal(M, seed=3, sigma=0.5)
    b = uniform_rhs(A.n, 5)
    sd1 = O.split(A.rowptr, A.colidx, np.zeros(A.n, dtype=np.int32), 1)
    x1, r1 = O.ss_cg_dot2(A, sd1, b, tol=1e-12)
    xg, rg = O.cg_dot2(A, b, tol=1e-12)
    assert r1.iterations == rg.iterations and np.array_equal(x1, xg)
    ref, _ = O.chol_solve(A.to_dense(), b)
    assert np.linalg.norm(xg - ref) <= 1e-9 * np.linalg.norm(ref) and r1.true_relres <= 1e-12
    its = set()
    for boxes, P in (((2, 2, 2), 8), ((2, 1, 1), 2), ((3, 2, 1), 6)):
        sd = O.split(A.rowptr, A.colidx, O.box_partition((M, M, M), boxes), P)
        _, r = O.ss_cg_dot2(A, sd, b, tol=1e-10)
        assert r.status == O.OK and r.true_relres <= 1e-10
        its.add(r.iterations)
    assert max(its) - min(its) <= 2
    w = config(1)
    _, rp = O.cg_dot2(w.A, w.b, tol=1e-10, maxit=10000)
    assert rp.status == O.OK and rp.iterations <= 568


def test_ir_reaches_fp64_accuracy():
    M = 10
    A = diffusion3d_lognormal(M, seed=3, sigma=0.5)
    b = uniform_rhs(A.n, 103)
    sd = O.split(A.rowptr, A.colidx, O.box_partition((M, M, M), (2, 2, 1)), 4)
    ref, _ = O.chol_solve(A.to_dense(), b)
    x, res = O.ss_ir(A, sd, b, tol=1e-10, inner_tol=1e-4)
    assert res.status == O.OK and res.true_relres <= 1e-10 and res.outer >= 2
    kappa = np.linalg.cond(A.to_dense())
    assert np.linalg.norm(x - ref) <= 2 * kappa * 1e-10 * np.linalg.norm(ref)
    # a single FP32 inner solve alone cannot get there: FP32 rounding of b
    # already limits it near 1e-7 relative
    assert np.max(np.abs(b - b.astype(np.float32))) > 1e-10


# ----------------------------------------------------------------------------
# Jacobi-preconditioned CG (Algorithm 3 with M = diag A)
# ----------------------------------------------------------------------------

def test_pcg_equals_cg_on_the_symmetrically_scaled_system():
    # With M = D, PCG on A x = b produces x_k = D^{-1/2} y_k where y_k are the
    # CG iterates on (D^{-1/2} A D^{-1/2}) y = D^{-1/2} b (the textbook
    # equivalence); checked after k steps on a small lognormal system
    M = 6
    A = diffusion3d_lognormal(M, seed=7, sigma=1.0)
    b = uniform_rhs(A.n, 107)
    D = A.to_dense()
    s = 1.0 / np.sqrt(np.diag(D))
    As = _dense_to_csr(D * s[:, None] * s[None, :])
    for k in (1, 3, 8):
        x, rp = O.pcg(A, b, tol=0.0, maxit=k, hist=False)
        y, rc = O.cg(As, s * b, tol=0.0, maxit=k, hist=False)
        assert rp.iterations == rc.iterations == k
        assert np.linalg.norm(x - s * y) <= 1e-11 * np.linalg.norm(x), k


def test_pcg_diagonal_matrix_one_step():
    d = np.array([1.0, 3.0, 0.5, 7.0, 2.0])
    A = _dense_to_csr(np.diag(d))
    b = np.array([1.0, -2.0, 3.0, 0.25, 5.0])
    x, r = O.pcg(A, b, tol=1e-14)
    assert r.status == O.OK and r.iterations == 1
    assert np.allclose(x, b / d, rtol=1e-15)


def test_pcg_accuracy_iterations_and_subdomains():
    M = 12
    A = diffusion3d_lognormal(M, seed=3, sigma=1.0)
    b = uniform_rhs(A.n, 108)
    D = A.to_dense()
    ref = np.linalg.solve(D, b)
    x, r = O.pcg(A, b, tol=1e-12, maxit=10000)
    assert r.status == O.OK and r.true_relres <= 1e-12
    kappa = np.linalg.cond(D)
    assert np.linalg.norm(x - ref) <= 2 * kappa * 1e-12 * np.linalg.norm(ref)
    _, rcg = O.cg(A, b, tol=1e-10, hist=False)
    _, rp = O.pcg(A, b, tol=1e-10, hist=False)
    assert rp.iterations < rcg.iterations
    # sub-structuring regroups the SpMV and the dots only
    its = []
    for boxes in [(1, 1, 1), (2, 2, 1), (2, 2, 2), (3, 2, 2)]:
        P = int(np.prod(boxes))
        sd = O.split(A.rowptr, A.colidx, O.box_partition((M, M, M), boxes), P)
        xs, rs = O.ss_pcg(A, sd, b, tol=1e-10, hist=False)
        its.append(rs.iterations)
        assert rs.status == O.OK and rs.true_relres <= 1e-10
        if P == 1:
            xg, rg = O.pcg(A, b, tol=1e-10, hist=False)
            assert np.array_equal(xs, xg) and rs.iterations == rg.iterations
    assert max(its) - min(its) <= 2, its


def test_pcg_edge_cases():
    A = diffusion3d_lognormal(5, seed=3, sigma=0.5)
    x, r = O.pcg(A, np.zeros(A.n), x0=np.ones(A.n))
    assert r.status == O.OK and r.iterations == 0 and not x.any()
    bn = uniform_rhs(A.n, 3)
    bn[2] = np.nan
    _, r = O.pcg(A, bn)
    assert r.status == O.EBREAKDOWN
    # a non-positive diagonal entry has no Jacobi inverse
    B = CSR(A.n, A.rowptr.copy(), A.colidx.copy(), A.val.copy())
    rows = B.row_of_nz()
    k0 = int(np.nonzero((rows == 0) & (B.colidx == 0))[0][0])
    B.val[k0] = 0.0
    _, r = O.pcg(B, uniform_rhs(A.n, 3))
    assert r.status == O.EINVAL


def _ru_case():
    M = 12
    A = diffusion3d_lognormal(M, seed=3, sigma=0.5)
    b = uniform_rhs(A.n, 104)
    sd = O.split(A.rowptr, A.colidx, O.box_partition((M, M, M), (2, 2, 1)), 4)
    return A, b, sd


def test_ru_reaches_fp64_accuracy_near_fp64_iteration_count():
    # FP32 CG with FP64 residual replacement: the true residual (numpy's own
    # matvec) meets the tolerance, the error is within the FP64 bound, and
    # because the search direction survives every replacement the iteration
    # count stays near FP64 CG's (a restart-based refinement needs clearly more)
    A, b, sd = _ru_case()
    x, res = O.ss_ru(A, sd, b, tol=1e-10, delta=0.1, check_every=8)
    D = A.to_dense()
    true = np.linalg.norm(b - D @ x) / np.linalg.norm(b)
    assert res.status == O.OK and true <= 1e-10 and res.outer >= 1
    assert abs(res.true_relres - true) <= 1e-3 * true
    ref = np.linalg.solve(D, b)
    kappa = np.linalg.cond(D)
    assert np.linalg.norm(x - ref) <= 2 * kappa * 1e-10 * np.linalg.norm(ref)
    _, r64 = O.ss_cg(A, sd, b, tol=1e-10)
    _, rir = O.ss_ir(A, sd, b, tol=1e-10, inner_tol=1e-6)
    assert res.iterations <= 1.05 * r64.iterations + 3, (res.iterations, r64.iterations)
    assert rir.iterations > 1.1 * res.iterations, (rir.iterations, res.iterations)


def test_ru_replacement_matters():
    # with no replacement inside the iteration (delta = 0) only the final
    # true-residual check corrects the FP32 drift: it needs restarts and more
    # iterations, and still ends at the tolerance
    A, b, sd = _ru_case()
    x0, r0 = O.ss_ru(A, sd, b, tol=1e-10, delta=0.0, check_every=8)
    x1, r1 = O.ss_ru(A, sd, b, tol=1e-10, delta=0.1, check_every=8)
    assert r0.status == O.OK and r0.outer == 0 and r0.true_relres <= 1e-10
    assert r1.outer > 0 and r0.iterations > r1.iterations
    # the replacement test only runs every check_every iterations
    x2, r2 = O.ss_ru(A, sd, b, tol=1e-10, delta=0.1, check_every=10 ** 6)
    assert r2.outer == 0 and r2.iterations == r0.iterations and np.array_equal(x2, x0)


def test_ru_edge_cases():
    A, b, sd = _ru_case()
    x, r = O.ss_ru(A, sd, np.zeros(A.n), x0=np.ones(A.n))
    assert r.status == O.OK and r.iterations == 0 and not x.any()
    x, r = O.ss_ru(A, sd, b, maxit=0)
    assert r.status == O.NOT_CONVERGED and r.iterations == 0
    x, r = O.ss_ru(A, sd, b, maxit=5)
    assert r.status == O.NOT_CONVERGED and r.iterations == 5
    bn = b.copy()
    bn[3] = np.nan
    _, r = O.ss_ru(A, sd, bn)
    assert r.status == O.EBREAKDOWN
    _, r = O.ss_ru(A, sd, b, check_every=0)
    assert r.status == O.EINVAL


# ----------------------------------------------------------------------------
# adjoint gradient: finite differences with symmetric perturbations
# ----------------------------------------------------------------------------

def test_adjoint_gradient_fd():
    M = 5
    A = diffusion3d_grf(M, seed=5, smooth=1.0)
    n = A.n
    D = A.to_dense()
    b = uniform_rhs(n, 105)
    xt = np.random.default_rng(205).uniform(-1, 1, n)

    def loss(Dm, bv):
        x, st = O.chol_solve(Dm, bv)
        assert st == O.OK
        return 0.5 * float(np.sum((x - xt) ** 2))

    x, _ = O.chol_solve(D, b)
    lam, _ = O.chol_solve(D, x - xt)
    dvals = O.grad_vals(A, lam, x)
    rows = A.row_of_nz()
    rng = np.random.default_rng(0)
    # directions on the pattern that keep A symmetric: a diagonal entry alone,
    # or an off-diagonal pair (i,j),(j,i) together
    for _ in range(12):
        k = int(rng.integers(A.nnz))
        i, j = int(rows[k]), int(A.colidx[k])
        E = np.zeros_like(D)
        E[i, j] = 1.0
        E[j, i] = 1.0
        eps = 1e-6 * np.abs(A.val).max()
        fd = (loss(D + eps * E, b) - loss(D - eps * E, b)) / (2 * eps)
        kt = k if i == j else int(np.nonzero((rows == j) & (A.colidx == i))[0][0])
        an = dvals[k] if i == j else dvals[k] + dvals[kt]
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    # dL/db = lambda
    for _ in range(4):
        d = rng.standard_normal(n)
        eps = 1e-6
        fd = (loss(D, b + eps * d) - loss(D, b - eps * d)) / (2 * eps)
        assert abs(fd - lam @ d) <= 1e-6 * max(1.0, abs(lam @ d))
