"""Adjoint CG backward (dL/db = A^{-1} g, dL/dA_ij = -lambda_i x_j on the
pattern) through torch.autograd, against the FP64 oracle gradient and central
finite differences along perturbations that keep A symmetric."""
import numpy as np
import pytest

import oracle as O
import paper_2108_13162_amd as ss
from workloads import CSR, config, diffusion3d_grf, uniform_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _transpose_index(A):
    """k -> index of the stored entry (j, i) for entry k = (i, j)."""
    rows = A.row_of_nz()
    key = rows * A.n + A.colidx
    tkey = A.colidx.astype(np.int64) * A.n + rows
    order = np.argsort(key)
    return order[np.searchsorted(key[order], tkey)]


def _loss_and_grads(A, solver, b, xt, tol):
    vals = _t(A.val).requires_grad_(True)
    bt = _t(b).requires_grad_(True)
    x = ss.sscg_solve(vals, bt, solver, tol=tol, adj_tol=tol)
    loss = 0.5 * torch.sum((x - _t(xt)) ** 2)
    loss.backward()
    return float(loss.detach()), vals.grad.cpu().numpy(), bt.grad.cpu().numpy(), x.detach().cpu().numpy()


def test_gradients_match_fp64_reference_small():
    w = config(5, size=8)
    A = w.A
    solver = ss.ss_cg_setup(A, ss.partition_workload(w))
    b, xt = w.b, w.extra["x_target"]
    _, dvals, db, x = _loss_and_grads(A, solver, b, xt, tol=1e-14)
    D = A.to_dense()
    xr, _ = O.chol_solve(D, b)
    lam, _ = O.chol_solve(D, xr - xt)
    ref = O.grad_vals(A, lam, xr)
    assert np.linalg.norm(x - xr) <= 1e-12 * np.linalg.norm(xr)
    assert np.linalg.norm(db - lam) <= 1e-10 * np.linalg.norm(lam)
    assert np.linalg.norm(dvals - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("opts", [{"precond": ss.SS_PRECOND_JACOBI}, {"small_solver": ss.SS_SMALL_OFF}])
def test_gradients_through_other_solve_paths(opts):
    # the same adjoint on a Jacobi-preconditioned solver and on the streaming
    # kernels (the 8^3 system otherwise takes the one-launch solve): both
    # solves converge to the same x and lambda, so the same gradients
    w = config(5, size=8)
    A = w.A
    solver = ss.ss_cg_setup(A, ss.partition_workload(w), ss.default_opts(**opts))
    b, xt = w.b, w.extra["x_target"]
    _, dvals, db, x = _loss_and_grads(A, solver, b, xt, tol=1e-14)
    D = A.to_dense()
    xr, _ = O.chol_solve(D, b)
    lam, _ = O.chol_solve(D, xr - xt)
    ref = O.grad_vals(A, lam, xr)
    assert np.linalg.norm(x - xr) <= 1e-12 * np.linalg.norm(xr)
    assert np.linalg.norm(db - lam) <= 1e-10 * np.linalg.norm(lam)
    assert np.linalg.norm(dvals - ref) <= 1e-10 * np.linalg.norm(ref)


def test_gradients_full_size_central_fd():
    # 64^3 smoothed-GRF diffusion, 8 boxes: loss 0.5 ||x - x_t||^2
    w = config(5)
    A = w.A
    solver = ss.ss_cg_setup(A, ss.partition_workload(w))
    b, xt = w.b, w.extra["x_target"]
    tol = 1e-13
    L0, dvals, db, x = _loss_and_grads(A, solver, b, xt, tol=tol)
    tr = _transpose_index(A)
    rows = A.row_of_nz()
    rng = np.random.default_rng(0)

    def loss_at(vals, bv):
        ss.ss_cg_set_values(solver, _t(vals))
        xx = torch.zeros(A.n, dtype=torch.float64, device=DEV)
        r = ss.ss_cg_solve(solver, _t(bv), xx, tol=tol, maxit=100000)
        assert r.status == ss.SS_OK
        return 0.5 * float(torch.sum((xx - _t(xt)) ** 2))

    for trial in range(8):
        # symmetric direction on the pattern: random on the upper triangle,
        # mirrored; a diagonal entry moves alone
        d = rng.standard_normal(A.nnz)
        d = np.where(rows <= A.colidx, d, d[tr])
        # Central differences carry an O(eps^2) truncation term that this
        # ill-conditioned system makes large (about 8e-4 relative at a step of
        # 1e-6 ||vals||_inf, identical on the CPU oracle); one Richardson step,
        # (4 D(eps) - D(2 eps)) / 3, removes it, leaving O(eps^4).
        eps = 1e-7 * np.abs(A.val).max() / np.abs(d).max()
        d1 = (loss_at(A.val + eps * d, b) - loss_at(A.val - eps * d, b)) / (2 * eps)
        d2 = (loss_at(A.val + 2 * eps * d, b) - loss_at(A.val - 2 * eps * d, b)) / (4 * eps)
        fd = (4.0 * d1 - d2) / 3.0
        an = float(dvals @ d)
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-12, (trial, fd, an)
    ss.ss_cg_set_values(solver, _t(A.val))
    for trial in range(4):
        # the loss is quadratic in b: central differences are exact up to rounding
        d = rng.standard_normal(A.n)
        eps = 1e-6
        fd = (loss_at(A.val, b + eps * d) - loss_at(A.val, b - eps * d)) / (2 * eps)
        an = float(db @ d)
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-12, (trial, fd, an)


def test_gradcheck_symmetric_parameterisation():
    # torch.autograd.gradcheck over the independent (upper-triangle) entries,
    # mapped to both triangles so that A stays symmetric
    A = diffusion3d_grf(4, seed=5, smooth=1.0)
    part = ss.ss_partition(A, ss.SS_PART_BOX, 4, grid=(4, 4, 4), boxes=(2, 2, 1))
    solver = ss.ss_cg_setup(A, part)
    rows = A.row_of_nz()
    upper = np.nonzero(rows <= A.colidx)[0]
    tr = _transpose_index(A)
    src = np.where(rows <= A.colidx, np.arange(A.nnz), tr)
    upos = np.full(A.nnz, -1)
    upos[upper] = np.arange(len(upper))
    gather = torch.tensor(upos[src], device=DEV)
    theta = _t(A.val[upper]).requires_grad_(True)
    b = _t(uniform_rhs(A.n, 9)).requires_grad_(True)

    def f(th, bb):
        return ss.sscg_solve(th[gather], bb, solver, tol=1e-14, adj_tol=1e-14)

    assert torch.autograd.gradcheck(f, (theta, b), eps=1e-6, atol=1e-7, rtol=1e-5)
