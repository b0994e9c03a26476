"""The all-cores (OpenMP) build of the oracle's CG, used by the benchmark's
CPU baseline and for floor solutions, against the pinned sequential oracle
(CPU only).  On one thread it performs the sequential oracle's operations in
the same order, so the results must be bitwise equal; on several threads only
the dot-product grouping changes."""
import numpy as np

import oracle as O
from workloads import config, diffusion3d_lognormal, uniform_rhs


def _case():
    M = 14
    A = diffusion3d_lognormal(M, seed=21)
    part = O.box_partition((M, M, M), (2, 2, 2))
    return A, O.split(A.rowptr, A.colidx, part, 8), uniform_rhs(A.n, 9)


def test_one_thread_is_the_sequential_oracle_bitwise():
    A, sd, b = _case()
    xs, rs = O.ss_cg(A, sd, b, tol=1e-10, hist=False)
    xo, ro = O.ss_cg_omp(A, sd, b, tol=1e-10, threads=1)
    assert ro.status == rs.status == O.OK and ro.iterations == rs.iterations
    assert np.array_equal(xo, xs) and ro.true_relres == rs.true_relres
    xg, rg = O.cg(A, b, tol=1e-10, hist=False)
    xg1, rg1 = O.cg_omp(A, b, tol=1e-10, threads=1)
    assert np.array_equal(xg1, xg) and rg1.iterations == rg.iterations


def test_threads_solve_the_same_system():
    A, sd, b = _case()
    xs, rs = O.ss_cg(A, sd, b, tol=1e-10, hist=False)
    for th in (2, 4, 7):
        x, r = O.ss_cg_omp(A, sd, b, tol=1e-10, threads=th)
        assert r.status == O.OK and r.true_relres <= 1e-10
        assert abs(r.iterations - rs.iterations) <= max(2, 0.02 * rs.iterations)
        true = np.linalg.norm(b - O.csr_matvec(A, x)) / np.linalg.norm(b)
        assert abs(true - r.true_relres) <= 1e-3 * true
        # the same thread count gives the same bits
        x2, r2 = O.ss_cg_omp(A, sd, b, tol=1e-10, threads=th)
        assert np.array_equal(x, x2)


def test_floor_solution_and_edge_cases():
    w = config(5, size=10)
    x, r = O.cg_omp(w.A, w.b, tol=1e-14, threads=3)
    ref, _ = O.chol_solve(w.A.to_dense(), w.b)
    assert r.status == O.OK and np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
    x0, r0 = O.cg_omp(w.A, np.zeros(w.A.n), x0=np.ones(w.A.n), threads=2)
    assert r0.status == O.OK and r0.iterations == 0 and not x0.any()
    _, rm = O.cg_omp(w.A, w.b, tol=1e-14, maxit=3, threads=2)
    assert rm.status == O.NOT_CONVERGED and rm.iterations == 3
