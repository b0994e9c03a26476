"""Band-row and band-column CG (Algorithms 1 and 2, Sections 4.2 and 4.3) on
one device, against the oracle, through the C-ABI.

The products are evaluated in the oracle's order and rounding (band-row: the
global row sums; band-column: each row's band partial sums added in band
order), so ss_cg_apply must reproduce the oracle's product exactly; the CG
iterates differ from the oracle's only by the dot-product summation orders."""
import numpy as np
import pytest

import oracle as O
import paper_2108_13162_amd as ss
from workloads import CSR, config, diffusion3d_lognormal, uniform_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _apply(s, x):
    return ss.ss_cg_apply(s, _t(x)).cpu().numpy()


def _oracle_apply(A, kind, nbands, x):
    return O.csr_matvec(A, x) if kind == ss.SS_BAND_ROW else O.band_col_spmv(A, nbands, x)


@pytest.mark.parametrize("kind", [ss.SS_BAND_ROW, ss.SS_BAND_COL])
@pytest.mark.parametrize("nbands", [1, 2, 7, 64])
def test_apply_matches_oracle_exactly(kind, nbands):
    # 40^3 diffusion: 1000 chunks of 64 rows, bands not dividing n
    A = diffusion3d_lognormal(40, seed=5, sigma=1.0)
    x = np.random.default_rng(nbands).standard_normal(A.n)
    s = ss.ss_band_setup(A, kind, nbands)
    got = _apply(s, x)
    want = _oracle_apply(A, kind, nbands, x)
    assert np.array_equal(got, want), np.max(np.abs(got - want))


def test_band_column_grouping_reaches_the_device():
    # row 0 = [1e16, -1e16, 1]; two bands (column 0 | columns 1-2): by band the
    # 1 is absorbed (0), left to right it survives (1)
    D = np.array([[1e16, -1e16, 1.0], [-1e16, 3.0, 0.0], [1.0, 0.0, 2.0]])
    rows, cols = np.nonzero(D)
    rp = np.zeros(4, dtype=np.int32)
    np.add.at(rp, rows + 1, 1)
    A = CSR(3, np.cumsum(rp).astype(np.int32), cols.astype(np.int32), D[rows, cols])
    x = np.ones(3)
    assert _apply(ss.ss_band_setup(A, ss.SS_BAND_ROW, 2), x)[0] == 1.0
    assert _apply(ss.ss_band_setup(A, ss.SS_BAND_COL, 2), x)[0] == 0.0
    assert _apply(ss.ss_band_setup(A, ss.SS_BAND_COL, 1), x)[0] == 1.0


def test_full_size_apply_matches_oracle_exactly():
    # 128^3 lognormal diffusion (2.1M rows), 8 bands
    w = config(2)
    x = np.random.default_rng(3).standard_normal(w.A.n)
    for kind in (ss.SS_BAND_ROW, ss.SS_BAND_COL):
        s = ss.ss_band_setup(w.A, kind, 8)
        got = _apply(s, x)
        want = _oracle_apply(w.A, kind, 8, x)
        assert np.array_equal(got, want), kind
        del s


@pytest.mark.parametrize("kind,nbands", [(ss.SS_BAND_ROW, 1), (ss.SS_BAND_ROW, 4), (ss.SS_BAND_COL, 3),
                                         (ss.SS_BAND_COL, 16)])
def test_solve_matches_oracle(kind, nbands):
    w = config(1)
    A, b = w.A, w.b
    s = ss.ss_band_setup(A, kind, nbands)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, _t(b), x, tol=1e-10, maxit=5000, hist=True)
    xo, ro = O.band_cg(A, kind, nbands, b, tol=1e-10, maxit=5000)
    xg = x.cpu().numpy()
    assert r.status == ss.SS_OK and ro.status == O.OK
    assert abs(r.iterations - ro.iterations) <= 2, (r.iterations, ro.iterations)
    assert r.true_relres <= 1e-10
    err = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    assert err <= 1e-9, err
    # residual history: within 10x the spread the summation order alone
    # causes on this system (oracle, several band counts vs the unsplit CG)
    _, ru = O.cg(A, b, tol=1e-10, maxit=5000)
    k = min(len(r.hist), len(ro.hist), len(ru.hist))
    spread = 0.0
    for nb in (2, 5, 9):
        _, rb = O.band_cg(A, kind, nb, b, tol=1e-10, maxit=5000)
        kk = min(k, len(rb.hist))
        spread = max(spread, np.max(np.abs(rb.hist[:kk] - ru.hist[:kk]) / ru.hist[:kk]))
    dh = np.max(np.abs(r.hist[:k] - ro.hist[:k]) / ro.hist[:k])
    print(f"kind {kind} nbands {nbands}: hist gpu-oracle {dh:.2e}, oracle spread {spread:.2e}")
    assert dh <= max(1e-10, 10 * spread), (dh, spread)


@pytest.mark.parametrize("k", [1, 10])
def test_fixed_k_iterates(k):
    # k iterations from x = 0 against the oracle, bar: 1e-12 relative or 10x the
    # oracle's own spread (band splitting vs unsplit CG differ in summation order)
    A = diffusion3d_lognormal(24, seed=9, sigma=1.0)
    b = uniform_rhs(A.n, 3)
    for kind in (ss.SS_BAND_ROW, ss.SS_BAND_COL):
        s = ss.ss_band_setup(A, kind, 5)
        x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
        r = ss.ss_cg_solve(s, _t(b), x, tol=0.0, maxit=k)
        xo, ro = O.band_cg(A, kind, 5, b, tol=0.0, maxit=k)
        xu, _ = O.cg(A, b, tol=0.0, maxit=k)
        assert r.status == ss.SS_NOT_CONVERGED and r.iterations == k
        spread = np.linalg.norm(xu - xo) / np.linalg.norm(xo)
        dx = np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo)
        assert dx <= max(1e-12, 10 * spread), (kind, dx, spread)


def test_band_setup_rejects_unsupported_options():
    A = config(1).A
    with pytest.raises(ss.SSError) as e:
        ss.ss_band_setup(A, ss.SS_BAND_COL, 4, ss.default_opts(precision=ss.SS_FP32_IR))
    assert e.value.code == ss.SS_EUNSUPPORTED
    with pytest.raises(ss.SSError) as e:
        ss.ss_band_setup(A, ss.SS_BAND_COL, 4, ss.default_opts(matrix_format=ss.SS_MAT_CSR))
    assert e.value.code == ss.SS_EUNSUPPORTED
    for kind, nb in [(5, 2), (ss.SS_BAND_ROW, 0), (ss.SS_BAND_COL, A.n + 1)]:
        with pytest.raises(ss.SSError) as e:
            ss.ss_band_setup(A, kind, nb)
        assert e.value.code == ss.SS_EINVAL
