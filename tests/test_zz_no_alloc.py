"""ss_cg_solve_noalloc against ss_cg_solve through the C-ABI: the same solve
(same kernels in the same order, so bitwise the same x, iteration count and
residual history) with the run state in the library's fixed per-GPU array and
no device allocation.  Two calls in a row, the second on a smaller system (the
one-launch path) with a shorter history; then the limits."""
import numpy as np
import pytest

import paper_2108_13162_amd as ss
from workloads import diffusion3d_lognormal, poisson2d, uniform_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _both(s, b, tol, maxit, hist):
    x1 = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    r1 = ss.ss_cg_solve(s, _t(b), x1, tol=tol, maxit=maxit, hist=hist)
    live = len(s.allocator.live)
    x2 = torch.zeros(len(b), dtype=torch.float64, device=DEV)
    r2 = ss.ss_cg_solve_noalloc(s, _t(b), x2, tol=tol, maxit=maxit, hist=hist)
    assert len(s.allocator.live) == live  # no allocator call
    return x1, r1, x2, r2


def _same(x1, r1, x2, r2):
    assert torch.equal(x1, x2)
    assert (r1.status, r1.iterations, r1.restarts, r1.relres) == (r2.status, r2.iterations, r2.restarts, r2.relres)
    if r1.hist is not None:
        assert np.array_equal(r1.hist, r2.hist)


def test_noalloc_matches_solve_twice():
    # call 1: 20^3 lognormal diffusion in 8 boxes (the streaming path)
    M = 20
    A = diffusion3d_lognormal(M, seed=31)
    s = ss.ss_cg_setup(A, ss.ss_partition(A, ss.SS_PART_BOX, 8, grid=(M, M, M), boxes=(2, 2, 2)))
    assert s.path() == ss.SS_PATH_STREAM
    b = uniform_rhs(A.n, 2)
    x1, r1, x2, r2 = _both(s, b, 1e-10, 6000, True)
    assert r1.status == ss.SS_OK and r1.iterations > 50
    _same(x1, r1, x2, r2)
    # call 2, smaller: 30 x 30 Poisson in 2 x 3 boxes (the one-launch path), shorter history
    B = poisson2d(30)
    s2 = ss.ss_cg_setup(B, ss.ss_partition(B, ss.SS_PART_BOX, 6, grid=(30, 30), boxes=(2, 3)))
    assert s2.path() == ss.SS_PATH_SMALL
    b2 = uniform_rhs(B.n, 3)
    y1, q1, y2, q2 = _both(s2, b2, 1e-10, 300, True)
    assert q1.status == ss.SS_OK and q1.iterations < r1.iterations
    _same(y1, q1, y2, q2)
    # and back to the first solver: the array keeps no state between calls
    x3 = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    r3 = ss.ss_cg_solve_noalloc(s, _t(b), x3, tol=1e-10, maxit=6000, hist=True)
    _same(x1, r1, x3, r3)


def test_noalloc_preconditioned_and_stopped_early():
    M = 16
    A = diffusion3d_lognormal(M, seed=5)
    p = ss.ss_partition(A, ss.SS_PART_BOX, 8, grid=(M, M, M), boxes=(2, 2, 2))
    s = ss.ss_cg_setup(A, p, ss.default_opts(precond=ss.SS_PRECOND_JACOBI))
    b = uniform_rhs(A.n, 4)
    _same(*_both(s, b, 1e-10, 4000, True))
    x1, r1, x2, r2 = _both(s, b, 1e-10, 7, False)
    assert r1.status == ss.SS_NOT_CONVERGED and r1.iterations == 7
    _same(x1, r1, x2, r2)


def test_noalloc_limits():
    M = 12
    A = diffusion3d_lognormal(M, seed=6)
    p = ss.ss_partition(A, ss.SS_PART_BOX, 8, grid=(M, M, M), boxes=(2, 2, 2))
    s = ss.ss_cg_setup(A, p)
    b = _t(uniform_rhs(A.n, 1))
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    with pytest.raises(ss.SSError) as e:
        ss.ss_cg_solve_noalloc(s, b, x, tol=1e-10, maxit=ss.SS_NOALLOC_HIST_MAX, hist=True)
    assert e.value.code == ss.SS_EINVAL
    # without a history any iteration limit is accepted
    r = ss.ss_cg_solve_noalloc(s, b, x, tol=1e-10, maxit=10 * ss.SS_NOALLOC_HIST_MAX)
    assert r.status == ss.SS_OK
    r = ss.ss_cg_solve_noalloc(s, b, x, tol=1e-10, maxit=ss.SS_NOALLOC_HIST_MAX - 1, hist=True)
    assert r.status == ss.SS_OK
    s32 = ss.ss_cg_setup(A, p, ss.default_opts(precision=ss.SS_FP32_RU))
    with pytest.raises(ss.SSError) as e:
        ss.ss_cg_solve_noalloc(s32, b, x, tol=1e-10, maxit=100)
    assert e.value.code == ss.SS_EUNSUPPORTED
    # the regular solve, by contrast, grows its history buffer through the allocator
    live = len(s.allocator.live)
    ss.ss_cg_solve(s, b, x, tol=1e-10, maxit=200000, hist=True)
    assert len(s.allocator.live) > live
