"""Pins the band-splitting part of the oracle (CPU only).

Algorithms 1 and 2 cut A into row bands and column bands; Sections 4.2 and
4.3 give the products and dot products of CG on them.  The oracle is checked
against bands worked out by hand on the paper's example matrix (Section 2.2),
against the defining identities (the bands reassemble A entry for entry),
against exact integer arithmetic, and against the unsplit CG and a dense
Cholesky solve.
"""
import os

import numpy as np
import pytest

import oracle as O
from workloads import CSR, config, random_spd_csr, uniform_rhs

from test_oracle_pins import _dense_to_csr, _read_golden


def _paper_matrix(golden_dir) -> CSR:
    g = _read_golden(os.path.join(golden_dir, "paper_csr_example.txt"))
    return _dense_to_csr(np.array(g["matrix"]))


# ----------------------------------------------------------------------------
# Algorithms 1 and 2 on the paper's 5 x 5 example, two bands: m = 5 // 2 = 2,
# the last band takes the remaining 3 rows / columns.
# ----------------------------------------------------------------------------

def test_row_bands_of_paper_example(golden_dir):
    A = _paper_matrix(golden_dir)
    rp, ci, v, nc = O.band_extract(A, O.BAND_ROW, 2, 0)
    assert nc == 5
    assert rp.tolist() == [0, 2, 4]
    assert ci.tolist() == [0, 1, 1, 2]
    assert v.tolist() == [-5, 14, 8, 1]
    rp, ci, v, nc = O.band_extract(A, O.BAND_ROW, 2, 1)
    assert rp.tolist() == [0, 2, 5, 7]
    assert ci.tolist() == [0, 2, 1, 3, 4, 2, 4]
    assert v.tolist() == [2, 10, 4, 2, 9, 15, 7]


def test_column_bands_of_paper_example(golden_dir):
    A = _paper_matrix(golden_dir)
    # columns 0-1: every row, local column = global column
    rp, ci, v, nc = O.band_extract(A, O.BAND_COL, 2, 0)
    assert nc == 2
    assert rp.tolist() == [0, 2, 3, 4, 5, 5]
    assert ci.tolist() == [0, 1, 1, 0, 1]
    assert v.tolist() == [-5, 14, 8, 2, 4]
    # columns 2-4, renumbered from 0
    rp, ci, v, nc = O.band_extract(A, O.BAND_COL, 2, 1)
    assert nc == 3
    assert rp.tolist() == [0, 0, 1, 2, 4, 6]
    assert ci.tolist() == [0, 0, 1, 2, 0, 2]
    assert v.tolist() == [1, 10, 2, 9, 15, 7]


def test_band_column_product_of_paper_example_is_exact(golden_dir):
    A = _paper_matrix(golden_dir)
    D = A.to_dense().astype(np.int64)
    x = np.array([3, -1, 4, 1, -5])
    for nb in range(1, 6):
        y = O.band_col_spmv(A, nb, x.astype(float))
        assert np.array_equal(y, (D @ x).astype(float)), nb


# ----------------------------------------------------------------------------
# The bands reassemble A, whatever n and the band count
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("n,nb", [(1, 1), (7, 1), (7, 3), (7, 7), (50, 4), (61, 8)])
def test_bands_tile_the_matrix(n, nb):
    A = random_spd_csr(n, 3.0, seed=n * 31 + nb)
    m = n // nb
    rows, cols, vals = [], [], []
    tot = 0
    for p in range(nb):
        rp, ci, v, nc = O.band_extract(A, O.BAND_ROW, nb, p)
        lo = p * m
        width = n - lo if p == nb - 1 else m
        assert len(rp) - 1 == width and nc == n
        tot += len(ci)
        for i in range(width):
            for k in range(rp[i], rp[i + 1]):
                rows.append(lo + i)
                cols.append(ci[k])
                vals.append(v[k])
    assert tot == A.nnz
    # concatenated row bands are A itself, in storage order
    assert np.array_equal(np.array(cols), A.colidx) and np.array_equal(np.array(vals), A.val)
    ent = {}
    for p in range(nb):
        rp, ci, v, nc = O.band_extract(A, O.BAND_COL, nb, p)
        lo = p * m
        assert len(rp) - 1 == n and nc == (n - lo if p == nb - 1 else m)
        for i in range(n):
            prev = -1
            for k in range(rp[i], rp[i + 1]):
                assert 0 <= ci[k] < nc and ci[k] > prev  # local, sorted
                prev = ci[k]
                key = (i, lo + ci[k])
                assert key not in ent
                ent[key] = v[k]
    # every stored entry in exactly one column band, same value
    want = {(i, int(A.colidx[k])): A.val[k] for i in range(n) for k in range(A.rowptr[i], A.rowptr[i + 1])}
    assert ent == want


def test_band_count_out_of_range_is_rejected():
    A = random_spd_csr(10, 2.0, seed=1)
    for nb, p in [(0, 0), (11, 0), (3, 3), (3, -1)]:
        with pytest.raises(ValueError):
            O.band_extract(A, O.BAND_ROW, nb, p)
    with pytest.raises(ValueError):
        O.band_cg(A, O.BAND_COL, 11, np.ones(10))


# ----------------------------------------------------------------------------
# Products and dot products
# ----------------------------------------------------------------------------

def test_band_column_product_integer_data_exact():
    rng = np.random.default_rng(5)
    A = random_spd_csr(120, 5.0, seed=9, integer=True)
    D = A.to_dense().astype(np.int64)
    x = rng.integers(-20, 21, size=120)
    for nb in (1, 2, 7, 120):
        assert np.array_equal(O.band_col_spmv(A, nb, x.astype(float)), (D @ x).astype(float))


def test_band_column_product_groups_sums_by_band():
    # row 0 = [1e16, -1e16, 1], two bands: column 0 | columns 1-2.  Summed by
    # band, 1e16 + (-1e16 + 1) = 0 (the 1 is absorbed); left to right it is 1.
    D = np.array([[1e16, -1e16, 1.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    A = _dense_to_csr(D)
    x = np.ones(3)
    assert O.csr_matvec(A, x)[0] == 1.0
    assert O.band_col_spmv(A, 2, x)[0] == 0.0
    assert O.band_col_spmv(A, 1, x)[0] == 1.0


def test_band_column_product_one_band_is_the_row_sum():
    A = random_spd_csr(200, 6.0, seed=2)
    x = np.random.default_rng(0).standard_normal(200)
    assert np.array_equal(O.band_col_spmv(A, 1, x), O.csr_matvec(A, x))


def test_band_column_product_within_rounding_of_dense():
    A = random_spd_csr(300, 6.0, seed=3)
    x = np.random.default_rng(1).standard_normal(300)
    D = np.abs(A.to_dense())
    exact = A.to_dense() @ x
    bound = 8 * 2.0 ** -53 * (D @ np.abs(x))  # a handful of roundings per row
    for nb in (2, 5, 300):
        assert np.all(np.abs(O.band_col_spmv(A, nb, x) - exact) <= bound)


def test_band_dot():
    rng = np.random.default_rng(4)
    u, v = rng.integers(-1000, 1000, 97), rng.integers(-1000, 1000, 97)
    for nb in (1, 3, 97):
        assert O.band_dot(nb, u.astype(float), v.astype(float)) == float(u @ v)
    a, b = rng.standard_normal(97), rng.standard_normal(97)
    assert O.band_dot(1, a, b) == O.dot(a, b)
    # band sums in band order: 3 bands of 32, 32, 33
    want = 0.0
    for lo, hi in [(0, 32), (32, 64), (64, 97)]:
        s = 0.0
        for i in range(lo, hi):
            s = s + a[i] * b[i]
        want = want + s
    assert O.band_dot(3, a, b) == want


# ----------------------------------------------------------------------------
# CG with the band splittings
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("kind", [O.BAND_ROW, O.BAND_COL])
def test_one_band_is_the_unsplit_cg(kind):
    w = config(1)
    x0, r0 = O.cg(w.A, w.b)
    x1, r1 = O.band_cg(w.A, kind, 1, w.b)
    assert r1.status == O.OK and r1.iterations == r0.iterations
    assert np.array_equal(x1, x0) and np.array_equal(r1.hist, r0.hist)


@pytest.mark.parametrize("kind,nb", [(O.BAND_ROW, 3), (O.BAND_ROW, 8), (O.BAND_COL, 2), (O.BAND_COL, 8)])
def test_band_cg_solves_small_spd(kind, nb):
    A = random_spd_csr(60, 4.0, seed=nb + 10 * kind)
    b = uniform_rhs(60, 7)
    xs, st = O.chol_solve(A.to_dense(), b)
    assert st == O.OK
    x, r = O.band_cg(A, kind, nb, b, tol=1e-12, maxit=2000)
    assert r.status == O.OK and r.true_relres <= 1e-11
    assert np.max(np.abs(x - xs)) <= 1e-9 * np.max(np.abs(xs))


@pytest.mark.parametrize("kind", [O.BAND_ROW, O.BAND_COL])
def test_band_cg_follows_the_unsplit_iteration(kind):
    # the splitting only regroups sums: same iterates up to rounding
    w = config(1)
    x0, r0 = O.cg(w.A, w.b)
    x1, r1 = O.band_cg(w.A, kind, 4, w.b)
    assert r1.status == O.OK and abs(r1.iterations - r0.iterations) <= 1
    assert r1.true_relres <= 1e-10
    assert np.max(np.abs(x1 - x0)) <= 1e-9 * np.max(np.abs(x0))
    k = min(len(r0.hist), len(r1.hist), 100)
    assert np.allclose(r1.hist[:k], r0.hist[:k], rtol=1e-8, atol=0)
