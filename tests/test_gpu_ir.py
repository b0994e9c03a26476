"""FP32 values + FP64 iterative refinement (SS_FP32_IR) against the oracle's
definition of the same method and against the FP64 accuracy bar.

The FP32 inner SpMV and vector updates are evaluated exactly as the oracle
writes them (FP32 products and sums in row order, FP64 updates rounded to
FP32); only the FP64 dot-product summation orders differ."""
import numpy as np
import pytest

import oracle as O
import paper_2108_13162_amd as ss
from workloads import config, diffusion3d_lognormal, uniform_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


TIN = 1e-5  # inner tolerance used on both sides


def _ir(A, p, **kw):
    kw.setdefault("inner_tol", TIN)
    return ss.ss_cg_setup(A, p, ss.default_opts(precision=ss.SS_FP32_IR, **kw))


@pytest.fixture(scope="module")
def q1():
    w = config(3, size=20)  # Q1 hexahedra, 20^3 unknowns, 16 weighted RCB parts
    sd = O.split(w.A.rowptr, w.A.colidx, O.rcb_partition(w.coords, w.weights), 16)
    return w, ss.partition_workload(w), sd


@pytest.mark.parametrize("k", [1, 5])
def test_first_inner_steps_match_oracle(q1, k):
    w, p, sd = q1
    A, b = w.A, w.b
    s = _ir(A, p, inner_maxit=k, max_outer=1)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, _t(b), x, tol=1e-10, maxit=100000)
    xo, ro = O.ss_ir(A, sd, b, tol=1e-10, inner_tol=TIN, inner_maxit=k, max_outer=1)
    assert r.status == ss.SS_NOT_CONVERGED and ro.status == O.NOT_CONVERGED
    assert r.iterations == ro.iterations == k and r.outer_iterations == ro.outer == 1
    xg = x.cpu().numpy()
    if k == 1:
        # the FP32 product is the oracle's bit for bit; only the FP64 dot
        # orders of ||r|| and (p, A p) differ, so each entry of d = fl32(alpha
        # p) is at most one FP32 rounding (2^-23 relative) from the oracle's
        # (x = ||r|| d); 2x covers a rare flip of fl32(r / ||r||) itself
        assert np.linalg.norm(xg - xo) <= 2 * 2.0 ** -23 * np.linalg.norm(xo)
    else:
        # roundings that flip propagate through the FP32 recurrences
        assert np.linalg.norm(xg - xo) <= 1e-5 * np.linalg.norm(xo)


def test_ir_solve_reaches_fp64_residual(q1):
    w, p, sd = q1
    A, b = w.A, w.b
    s = _ir(A, p)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, _t(b), x, tol=1e-10, maxit=100000, hist=True)
    xo, ro = O.ss_ir(A, sd, b, tol=1e-10, inner_tol=TIN)
    xg = x.cpu().numpy()
    true = np.linalg.norm(b - O.csr_matvec(A, xg)) / np.linalg.norm(b)
    assert r.status == ss.SS_OK and true <= 1e-10, (r, true)
    assert r.outer_iterations >= 2 and abs(r.outer_iterations - ro.outer) <= 1
    assert abs(r.iterations - ro.iterations) <= max(5, 0.1 * ro.iterations), (r.iterations, ro.iterations)
    # error against the FP64 floor solution, stated and bounded like FP64 CG's
    xref = O.solve_reference(A, b)
    err = np.linalg.norm(xg - xref) / np.linalg.norm(xref)
    x64, r64 = O.ss_cg(A, sd, b, tol=1e-10)
    err64 = np.linalg.norm(x64 - xref) / np.linalg.norm(xref)
    print(f"IR: {r.iterations} inner / {r.outer_iterations} outer iterations, true relres {true:.2e}, "
          f"error {err:.2e} (FP64 CG: {r64.iterations} iterations, error {err64:.2e})")
    assert err <= max(1e-9, 10 * err64)
    assert r.hist is not None and np.all(np.isfinite(r.hist))


def test_ir_solution_error_1e9(q1):
    w, p, sd = q1
    s = _ir(w.A, p)
    x = torch.zeros(w.A.n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, _t(w.b), x, tol=1e-13, maxit=100000)
    assert r.status == ss.SS_OK
    xref = O.solve_reference(w.A, w.b)
    assert np.linalg.norm(x.cpu().numpy() - xref) <= 1e-9 * np.linalg.norm(xref)


def test_ir_edge_cases():
    A = diffusion3d_lognormal(9, seed=3, sigma=0.5)
    p = ss.ss_partition(A, ss.SS_PART_BOX, 8, grid=(9, 9, 9), boxes=(2, 2, 2))
    s = _ir(A, p)
    n = A.n
    x = torch.ones(n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, torch.zeros(n, dtype=torch.float64, device=DEV), x)
    assert r.status == ss.SS_OK and r.iterations == 0 and not x.cpu().numpy().any()
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, _t(uniform_rhs(n, 1)), x, tol=1e-10, maxit=3)
    assert r.status == ss.SS_NOT_CONVERGED and r.iterations == 3
    bn = uniform_rhs(n, 2)
    bn[0] = np.nan
    r = ss.ss_cg_solve(s, _t(bn), torch.zeros(n, dtype=torch.float64, device=DEV))
    assert r.status == ss.SS_EBREAKDOWN
    with pytest.raises(ss.SSError):
        ss.ss_cg_setup(A, p, ss.default_opts(precision=ss.SS_FP32_IR, inner_tol=2.0))
