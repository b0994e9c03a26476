"""FP32 CG with FP64 residual replacement (SS_FP32_RU) against the oracle's
definition of the same method (oracle.ss_ru, with the same replacement
threshold and the same test interval = the polled chunk length).

The FP32 SpMV and the FP64-evaluated, FP32-rounded vector updates are the
oracle's; only the FP64 dot summation orders differ, so replacement points
and iteration counts can shift slightly."""
import numpy as np
import pytest

import oracle as O
import paper_2108_13162_amd as ss
from workloads import config, diffusion3d_lognormal, uniform_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CHUNK = 8


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _ru(A, p, **kw):
    kw.setdefault("check_every", CHUNK)
    return ss.ss_cg_setup(A, p, ss.default_opts(precision=ss.SS_FP32_RU, **kw))


@pytest.fixture(scope="module")
def q1():
    w = config(3, size=20)  # Q1 hexahedra, 20^3 unknowns, 16 weighted RCB parts
    sd = O.split(w.A.rowptr, w.A.colidx, O.rcb_partition(w.coords, w.weights), 16)
    return w, ss.partition_workload(w), sd


@pytest.mark.parametrize("k", [1, 5])
def test_first_steps_match_oracle(q1, k):
    # no replacement before the first chunk end: plain FP32 CG steps
    w, p, sd = q1
    s = _ru(w.A, p)
    x = torch.zeros(w.A.n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, _t(w.b), x, tol=1e-10, maxit=k)
    xo, ro = O.ss_ru(w.A, sd, w.b, tol=1e-10, maxit=k, check_every=CHUNK)
    assert r.status == ss.SS_NOT_CONVERGED and ro.status == O.NOT_CONVERGED
    assert r.iterations == ro.iterations == k
    xg = x.cpu().numpy()
    if k == 1:
        # r = fl32(b), p = r and q = A32 p are the oracle's bit for bit; alpha
        # differs only by the FP64 dot orders, so each entry of x = d =
        # fl32(alpha p) is the oracle's or one FP32 rounding (2^-23 relative) away
        assert np.all(np.abs(xg - xo) <= 2.0 ** -23 * np.abs(xo)), np.max(np.abs(xg - xo) / np.abs(xo))
    else:
        # roundings that flip propagate through the FP32 recurrences
        assert np.linalg.norm(xg - xo) <= 1e-5 * np.linalg.norm(xo)


def test_ru_solve_matches_oracle(q1):
    w, p, sd = q1
    A, b = w.A, w.b
    s = _ru(A, p)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, _t(b), x, tol=1e-10, maxit=100000, hist=True)
    xo, ro = O.ss_ru(A, sd, b, tol=1e-10, check_every=CHUNK)
    xg = x.cpu().numpy()
    true = np.linalg.norm(b - O.csr_matvec(A, xg)) / np.linalg.norm(b)
    assert r.status == ss.SS_OK and true <= 1e-10, (r, true)
    assert abs(r.relres - true) <= 1e-3 * true
    assert r.outer_iterations >= 1 and abs(r.outer_iterations - ro.outer) <= 2, (r.outer_iterations, ro.outer)
    assert abs(r.iterations - ro.iterations) <= max(3, 0.05 * ro.iterations), (r.iterations, ro.iterations)
    xref = O.solve_reference(A, b)
    x64, r64 = O.ss_cg(A, sd, b, tol=1e-10)
    err = np.linalg.norm(xg - xref) / np.linalg.norm(xref)
    err64 = np.linalg.norm(x64 - xref) / np.linalg.norm(xref)
    print(f"RU: {r.iterations} iterations, {r.outer_iterations} replacements, true relres {true:.2e}, "
          f"error {err:.2e} (FP64 CG: {r64.iterations} iterations, error {err64:.2e}; oracle RU {ro.iterations})")
    assert err <= max(1e-9, 10 * err64)
    assert r.iterations <= 1.1 * r64.iterations + 5
    assert r.hist is not None and np.all(np.isfinite(r.hist))


def test_ru_graph_and_eager_identical(q1):
    w, p, sd = q1
    out = []
    for g in (1, 0):
        s = _ru(w.A, p, use_graph=g)
        x = torch.zeros(w.A.n, dtype=torch.float64, device=DEV)
        r = ss.ss_cg_solve(s, _t(w.b), x, tol=1e-10, maxit=100000)
        out.append((x.cpu().numpy(), r.iterations, r.outer_iterations))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1:] == out[1][1:]


def test_ru_solution_error_1e9(q1):
    w, p, sd = q1
    s = _ru(w.A, p)
    x = torch.zeros(w.A.n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, _t(w.b), x, tol=1e-13, maxit=100000)
    assert r.status == ss.SS_OK
    xref = O.solve_reference(w.A, w.b)
    assert np.linalg.norm(x.cpu().numpy() - xref) <= 1e-9 * np.linalg.norm(xref)


def test_ru_edge_cases():
    A = diffusion3d_lognormal(9, seed=3, sigma=0.5)
    p = ss.ss_partition(A, ss.SS_PART_BOX, 8, grid=(9, 9, 9), boxes=(2, 2, 2))
    s = _ru(A, p)
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
    # delta = 0: no replacement inside the iteration, the final check restarts
    s0 = _ru(A, p, ru_delta=0.0)
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s0, _t(uniform_rhs(n, 1)), x, tol=1e-10, maxit=100000)
    assert r.status == ss.SS_OK and r.outer_iterations == 0
    with pytest.raises(ss.SSError):
        _ru(A, p, ru_delta=1.5)


def test_full_size_cfg3_ru():
    # Q1 hexahedra on 96^3 unknowns (23.4M entries), 16 uneven RCB parts
    w = config(3)
    A, b = w.A, w.b
    p = ss.partition_workload(w)
    s = ss.ss_cg_setup(A, p, ss.default_opts(precision=ss.SS_FP32_RU))
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, _t(b), x, tol=1e-10, maxit=100000)
    xg = x.cpu().numpy()
    true = np.linalg.norm(b - O.csr_matvec(A, xg)) / np.linalg.norm(b)
    assert r.status == ss.SS_OK and true <= 1e-10, (r, true)
    print(f"cfg3 RU: {r.iterations} iterations, {r.outer_iterations} replacements, true relres {true:.2e}")
