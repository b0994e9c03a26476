"""Oracle for the sub-structured CG -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation (numpy for the integer
partition maps, sequential C in FP64 for the arithmetic).  Only tests/, the
smoke check and the bench's CPU-baseline leg may import, call or link it; the
HIP library never does, and the two share no code.  Both sides only share the
seeded input generators of the ``workloads`` package.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .partition import SubDomains, box_partition, partition_workload, rcb_partition, split  # noqa: F401
from . import build as _build

OK, NOT_CONVERGED, EINVAL, ENOMEM, EBREAKDOWN = 0, 1, -1, -2, -4

_lib = None
_lib_omp = None


def lib_omp():
    """The all-cores build (OpenMP) of the CG, for the benchmark's CPU baseline."""
    global _lib_omp
    if _lib_omp is None:
        if (not os.path.exists(_build.LIB_OMP)
                or os.path.getmtime(_build.LIB_OMP) < os.path.getmtime(_build.SRC_OMP)):
            _build.build()
        L = C.CDLL(_build.LIB_OMP)
        i64, i32, dbl, P = C.c_int64, C.c_int32, C.c_double, C.c_void_p
        L.orc_ss_cg_omp.argtypes = [P, i64, P, P, P, P, P, dbl, i32, i32, P, P, P]
        L.orc_cg_omp.argtypes = [i64, P, P, P, P, P, dbl, i32, i32, P, P, P]
        L.orc_omp_max_threads.restype = C.c_int
        _lib_omp = L
    return _lib_omp


def lib():
    global _lib
    if _lib is None:
        if (not os.path.exists(_build.LIB)
                or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = C.CDLL(_build.LIB)
        i64, i32, dbl = C.c_int64, C.c_int32, C.c_double
        P = C.c_void_p
        L.orc_csr_matvec.argtypes = [i64, P, P, P, P, P]
        L.orc_csr_matvec_f32.argtypes = [i64, P, P, P, P, P]
        L.orc_iface_sum.argtypes = [i64, P, P, P]
        L.orc_iface_sum_f32.argtypes = [i64, P, P, P]
        L.orc_owned_dot_f32.argtypes = [i32, P, P, P, P, P]
        L.orc_owned_dot_f32.restype = dbl
        L.orc_ss_spmv_f32.argtypes = [P, P, P]
        L.orc_dot.argtypes = [i64, P, P]
        L.orc_dot.restype = dbl
        L.orc_owned_dot.argtypes = [i32, P, P, P, P, P]
        L.orc_owned_dot.restype = dbl
        L.orc_ss_spmv.argtypes = [P, P, P]
        L.orc_cg.argtypes = [i64, P, P, P, P, P, dbl, i32, P, P, P, P]
        L.orc_ss_cg.argtypes = [P, i64, P, P, P, P, P, dbl, i32, P, P, P, P]
        L.orc_ss_cg_dot2.argtypes = [P, i64, P, P, P, P, P, dbl, i32, P, P, P, P]
        L.orc_cg_dot2.argtypes = [i64, P, P, P, P, P, dbl, i32, P, P, P, P]
        L.orc_dot2.argtypes = [i64, P, P]
        L.orc_dot2.restype = dbl
        L.orc_owned_dot2.argtypes = [i32, P, P, P, P, P]
        L.orc_owned_dot2.restype = dbl
        L.orc_pcg.argtypes = [i64, P, P, P, P, P, dbl, i32, P, P, P, P]
        L.orc_ss_pcg.argtypes = [P, i64, P, P, P, P, P, dbl, i32, P, P, P, P]
        L.orc_ss_ir.argtypes = [P, i64, P, P, P, P, P, dbl, i32, dbl, i32, i32, P, P, P, P]
        L.orc_ss_ru.argtypes = [P, i64, P, P, P, P, P, dbl, i32, dbl, i32, P, P, P, P]
        L.orc_grad_vals.argtypes = [i64, P, P, P, P, P]
        L.orc_chol_solve.argtypes = [i64, P, P, P]
        L.orc_band_size.argtypes = [i64, P, P, i32, i32, i32, P, P, P]
        L.orc_band_extract.argtypes = [i64, P, P, P, i32, i32, i32, P, P, P]
        L.orc_band_col_spmv.argtypes = [i64, P, P, P, i32, P, P, P]
        L.orc_band_dot.argtypes = [i64, i32, P, P]
        L.orc_band_dot.restype = dbl
        L.orc_band_cg.argtypes = [i64, P, P, P, i32, i32, P, P, dbl, i32, P, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class _OrcSub(C.Structure):
    _fields_ = [
        ("P", C.c_int32), ("n_loc", C.c_int32),
        ("sub_off", C.c_void_p), ("n_int", C.c_void_p), ("n_own", C.c_void_p), ("l2g", C.c_void_p),
        ("ngamma", C.c_int32),
        ("copy_ptr", C.c_void_p), ("copy_pos", C.c_void_p),
        ("bd_rowptr", C.c_void_p), ("bd_colidx", C.c_void_p),
        ("bd_val", C.c_void_p), ("bd_val32", C.c_void_p),
    ]


class _Sub:
    """Keeps the arrays behind an orc_sub alive."""

    def __init__(self, sd: SubDomains, val: np.ndarray):
        self.keep = [sd.sub_off, sd.n_int, sd.n_own, sd.l2g, sd.copy_ptr, sd.copy_pos,
                     sd.bd_rowptr, sd.bd_colidx]
        self.v64 = _f64(sd.bd_values(val))
        self.v32 = self.v64.astype(np.float32)  # round to nearest even
        self.s = _OrcSub(sd.nparts, sd.n_loc, _p(sd.sub_off), _p(sd.n_int), _p(sd.n_own), _p(sd.l2g),
                         len(sd.gamma), _p(sd.copy_ptr), _p(sd.copy_pos), _p(sd.bd_rowptr),
                         _p(sd.bd_colidx), _p(self.v64), _p(self.v32))

    def ref(self):
        return C.byref(self.s)


@dataclass
class Result:
    status: int
    iterations: int
    relres: float
    true_relres: float
    hist: Optional[np.ndarray] = None
    outer: int = 0       # IR: outer corrections; RU: residual replacements inside the iteration


# ----------------------------------------------------------------------------
# building blocks
# ----------------------------------------------------------------------------

def csr_matvec(A, x: np.ndarray) -> np.ndarray:
    x = _f64(x)
    y = np.empty(A.n)
    lib().orc_csr_matvec(A.n, _p(_i32(A.rowptr)), _p(_i32(A.colidx)), _p(_f64(A.val)), _p(x), _p(y))
    return y


def csr_matvec_f32(rowptr, colidx, val32, x32) -> np.ndarray:
    n = len(rowptr) - 1
    x32 = np.ascontiguousarray(x32, dtype=np.float32)
    v = np.ascontiguousarray(val32, dtype=np.float32)
    y = np.empty(n, dtype=np.float32)
    lib().orc_csr_matvec_f32(n, _p(_i32(rowptr)), _p(_i32(colidx)), _p(v), _p(x32), _p(y))
    return y


def iface_sum(sd: SubDomains, q: np.ndarray) -> np.ndarray:
    q = _f64(q).copy()
    lib().orc_iface_sum(len(sd.gamma), _p(sd.copy_ptr), _p(sd.copy_pos), _p(q))
    return q


def iface_sum_f32(copy_ptr, copy_pos, q32) -> np.ndarray:
    """FP32 interface assembly on explicit copy lists (sequential, list order)."""
    q = np.ascontiguousarray(q32, dtype=np.float32).copy()
    cp = _i32(copy_ptr)
    lib().orc_iface_sum_f32(len(cp) - 1, _p(cp), _p(_i32(copy_pos)), _p(q))
    return q


def dot(u, v) -> float:
    u, v = _f64(u), _f64(v)
    return lib().orc_dot(len(u), _p(u), _p(v))


def owned_dot(sd: SubDomains, u, v) -> float:
    u, v = _f64(u), _f64(v)
    return lib().orc_owned_dot(sd.nparts, _p(sd.sub_off), _p(sd.n_int), _p(sd.n_own), _p(u), _p(v))


def owned_dot_f32(sd: SubDomains, u32, v32) -> float:
    """Weighted local dot of FP32 vectors, accumulated in FP64."""
    u = np.ascontiguousarray(u32, dtype=np.float32)
    v = np.ascontiguousarray(v32, dtype=np.float32)
    return lib().orc_owned_dot_f32(sd.nparts, _p(sd.sub_off), _p(sd.n_int), _p(sd.n_own), _p(u), _p(v))


def gather(sd: SubDomains, v: np.ndarray) -> np.ndarray:
    return _f64(v)[sd.l2g]


def owned_positions(sd: SubDomains) -> np.ndarray:
    return np.concatenate([np.arange(sd.sub_off[s], sd.sub_off[s] + sd.n_int[s] + sd.n_own[s])
                           for s in range(sd.nparts)]).astype(np.int64)


def scatter_owned(sd: SubDomains, loc: np.ndarray, n: int) -> np.ndarray:
    out = np.empty(n)
    pos = owned_positions(sd)
    out[sd.l2g[pos]] = loc[pos]
    return out


def ss_spmv_local(sd: SubDomains, val: np.ndarray, x_loc: np.ndarray) -> np.ndarray:
    """Sub-structured SpMV on concatenated local vectors (assembled result)."""
    S = _Sub(sd, val)
    x_loc = _f64(x_loc)
    q = np.empty(sd.n_loc)
    lib().orc_ss_spmv(S.ref(), _p(x_loc), _p(q))
    return q


def ss_spmv_f32(A, sd: SubDomains, x32: np.ndarray) -> np.ndarray:
    """y = A32 x32 in FP32 through the sub-structured path, global numbering:
    the inner product of the FP32 modes (values rounded to FP32)."""
    S = _Sub(sd, A.val)
    xl = np.ascontiguousarray(np.asarray(x32, dtype=np.float32)[sd.l2g])
    q = np.empty(sd.n_loc, dtype=np.float32)
    lib().orc_ss_spmv_f32(S.ref(), _p(xl), _p(q))
    out = np.empty(A.n, dtype=np.float32)
    pos = owned_positions(sd)
    out[sd.l2g[pos]] = q[pos]
    return out


def ss_spmv(A, sd: SubDomains, x: np.ndarray) -> np.ndarray:
    """y = A x in global numbering through the sub-structured path."""
    q = ss_spmv_local(sd, A.val, gather(sd, x))
    return scatter_owned(sd, q, A.n)


# ----------------------------------------------------------------------------
# solvers
# ----------------------------------------------------------------------------

def cg(A, b, x0=None, tol: float = 1e-10, maxit: int = 10000, hist: bool = True) -> tuple:
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    h = np.full(maxit + 1, np.nan)
    it, rel, tr = C.c_int32(), C.c_double(), C.c_double()
    st = lib().orc_cg(A.n, _p(_i32(A.rowptr)), _p(_i32(A.colidx)), _p(_f64(A.val)), _p(b), _p(x), tol, maxit,
                      _p(h), C.byref(it), C.byref(rel), C.byref(tr))
    return x, Result(st, it.value, rel.value, tr.value, h[: it.value + 1] if hist else None)


def ss_cg(A, sd: SubDomains, b, x0=None, tol: float = 1e-10, maxit: int = 10000, hist: bool = True) -> tuple:
    S = _Sub(sd, A.val)
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    h = np.full(maxit + 1, np.nan)
    it, rel, tr = C.c_int32(), C.c_double(), C.c_double()
    st = lib().orc_ss_cg(S.ref(), A.n, _p(_i32(A.rowptr)), _p(_i32(A.colidx)), _p(_f64(A.val)), _p(b), _p(x),
                         tol, maxit, _p(h), C.byref(it), C.byref(rel), C.byref(tr))
    return x, Result(st, it.value, rel.value, tr.value, h[: it.value + 1] if hist else None)


def dot2(u, v) -> float:
    """Dot product as accurate as in twice the working precision (Dot2)."""
    u, v = _f64(u), _f64(v)
    return lib().orc_dot2(len(u), _p(u), _p(v))


def owned_dot2(sd: SubDomains, u, v) -> float:
    u, v = _f64(u), _f64(v)
    return lib().orc_owned_dot2(sd.nparts, _p(sd.sub_off), _p(sd.n_int), _p(sd.n_own), _p(u), _p(v))


def cg_dot2(A, b, x0=None, tol: float = 1e-10, maxit: int = 10000, hist: bool = True) -> tuple:
    """cg with Dot2 dot products."""
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    h = np.full(maxit + 1, np.nan)
    it, rel, tr = C.c_int32(), C.c_double(), C.c_double()
    st = lib().orc_cg_dot2(A.n, _p(_i32(A.rowptr)), _p(_i32(A.colidx)), _p(_f64(A.val)), _p(b), _p(x), tol,
                           maxit, _p(h), C.byref(it), C.byref(rel), C.byref(tr))
    return x, Result(st, it.value, rel.value, tr.value, h[: it.value + 1] if hist else None)


def ss_cg_dot2(A, sd: SubDomains, b, x0=None, tol: float = 1e-10, maxit: int = 10000, hist: bool = True) -> tuple:
    """ss_cg with Dot2 dot products: the reference for CG with exactly rounded dots."""
    S = _Sub(sd, A.val)
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    h = np.full(maxit + 1, np.nan)
    it, rel, tr = C.c_int32(), C.c_double(), C.c_double()
    st = lib().orc_ss_cg_dot2(S.ref(), A.n, _p(_i32(A.rowptr)), _p(_i32(A.colidx)), _p(_f64(A.val)), _p(b),
                              _p(x), tol, maxit, _p(h), C.byref(it), C.byref(rel), C.byref(tr))
    return x, Result(st, it.value, rel.value, tr.value, h[: it.value + 1] if hist else None)


def pcg(A, b, x0=None, tol: float = 1e-10, maxit: int = 10000, hist: bool = True) -> tuple:
    """Jacobi-preconditioned CG on the global matrix (Algorithm 3, M = diag A)."""
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    h = np.full(maxit + 1, np.nan)
    it, rel, tr = C.c_int32(), C.c_double(), C.c_double()
    st = lib().orc_pcg(A.n, _p(_i32(A.rowptr)), _p(_i32(A.colidx)), _p(_f64(A.val)), _p(b), _p(x), tol, maxit,
                       _p(h), C.byref(it), C.byref(rel), C.byref(tr))
    return x, Result(st, it.value, rel.value, tr.value, h[: it.value + 1] if hist else None)


def ss_pcg(A, sd: SubDomains, b, x0=None, tol: float = 1e-10, maxit: int = 10000, hist: bool = True) -> tuple:
    """Sub-structured Jacobi-preconditioned CG (every copy holds the global 1/a_ii)."""
    S = _Sub(sd, A.val)
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    h = np.full(maxit + 1, np.nan)
    it, rel, tr = C.c_int32(), C.c_double(), C.c_double()
    st = lib().orc_ss_pcg(S.ref(), A.n, _p(_i32(A.rowptr)), _p(_i32(A.colidx)), _p(_f64(A.val)), _p(b), _p(x),
                          tol, maxit, _p(h), C.byref(it), C.byref(rel), C.byref(tr))
    return x, Result(st, it.value, rel.value, tr.value, h[: it.value + 1] if hist else None)


def ss_ir(A, sd: SubDomains, b, x0=None, tol: float = 1e-10, maxit: int = 100000,
          inner_tol: float = 1e-6, inner_maxit: int = 100000, max_outer: int = 50) -> tuple:
    S = _Sub(sd, A.val)
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    it, outer, rel, tr = C.c_int32(), C.c_int32(), C.c_double(), C.c_double()
    st = lib().orc_ss_ir(S.ref(), A.n, _p(_i32(A.rowptr)), _p(_i32(A.colidx)), _p(_f64(A.val)), _p(b), _p(x),
                         tol, maxit, inner_tol, inner_maxit, max_outer, C.byref(it), C.byref(outer),
                         C.byref(rel), C.byref(tr))
    return x, Result(st, it.value, rel.value, tr.value, None, outer.value)


def ss_ru(A, sd: SubDomains, b, x0=None, tol: float = 1e-10, maxit: int = 100000, delta: float = 0.1,
          check_every: int = 32) -> tuple:
    """FP32 CG with FP64 residual replacement (see orc_ss_ru); Result.outer =
    replacements made inside the iteration."""
    S = _Sub(sd, A.val)
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    it, nref, rel, tr = C.c_int32(), C.c_int32(), C.c_double(), C.c_double()
    st = lib().orc_ss_ru(S.ref(), A.n, _p(_i32(A.rowptr)), _p(_i32(A.colidx)), _p(_f64(A.val)), _p(b), _p(x),
                         tol, maxit, delta, check_every, C.byref(it), C.byref(nref), C.byref(rel), C.byref(tr))
    return x, Result(st, it.value, rel.value, tr.value, None, nref.value)


# ----------------------------------------------------------------------------
# band splittings (Algorithms 1 and 2)
# ----------------------------------------------------------------------------

BAND_ROW, BAND_COL = 0, 1


def band_extract(A, kind: int, nbands: int, p: int) -> tuple:
    """Band p of nbands (kind BAND_ROW or BAND_COL) as (rowptr, colidx, val, ncols)."""
    rp, ci, v = _i32(A.rowptr), _i32(A.colidx), _f64(A.val)
    nr, nc, nz = C.c_int64(), C.c_int64(), C.c_int64()
    st = lib().orc_band_size(A.n, _p(rp), _p(ci), kind, nbands, p, C.byref(nr), C.byref(nc), C.byref(nz))
    if st != OK:
        raise ValueError(f"band_extract: status {st}")
    brp = np.empty(nr.value + 1, dtype=np.int32)
    bci = np.empty(max(nz.value, 1), dtype=np.int32)
    bv = np.empty(max(nz.value, 1))
    lib().orc_band_extract(A.n, _p(rp), _p(ci), _p(v), kind, nbands, p, _p(brp), _p(bci), _p(bv))
    return brp, bci[: nz.value], bv[: nz.value], nc.value


def band_col_spmv(A, nbands: int, x) -> np.ndarray:
    x = _f64(x)
    y, tmp = np.empty(A.n), np.empty(A.n)
    lib().orc_band_col_spmv(A.n, _p(_i32(A.rowptr)), _p(_i32(A.colidx)), _p(_f64(A.val)), nbands, _p(x), _p(y),
                            _p(tmp))
    return y


def band_dot(nbands: int, u, v) -> float:
    u, v = _f64(u), _f64(v)
    return lib().orc_band_dot(len(u), nbands, _p(u), _p(v))


def band_cg(A, kind: int, nbands: int, b, x0=None, tol: float = 1e-10, maxit: int = 10000,
            hist: bool = True) -> tuple:
    """CG (Algorithm 3, M = I) with the band-row or band-column splitting."""
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    h = np.full(maxit + 1, np.nan)
    it, rel, tr = C.c_int32(), C.c_double(), C.c_double()
    st = lib().orc_band_cg(A.n, _p(_i32(A.rowptr)), _p(_i32(A.colidx)), _p(_f64(A.val)), kind, nbands, _p(b),
                           _p(x), tol, maxit, _p(h), C.byref(it), C.byref(rel), C.byref(tr))
    if st == EINVAL:
        raise ValueError("band_cg: bad band count or kind")
    return x, Result(st, it.value, rel.value, tr.value, h[: it.value + 1] if hist else None)


def grad_vals(A, lam, x) -> np.ndarray:
    lam, x = _f64(lam), _f64(x)
    d = np.empty(A.nnz)
    lib().orc_grad_vals(A.n, _p(_i32(A.rowptr)), _p(_i32(A.colidx)), _p(lam), _p(x), _p(d))
    return d


def chol_solve(D: np.ndarray, b) -> tuple:
    a = np.array(D, dtype=np.float64, order="C", copy=True)
    b = _f64(b)
    x = np.empty(len(b))
    st = lib().orc_chol_solve(len(b), _p(a), _p(b), _p(x))
    return x, st


def ss_cg_omp(A, sd: SubDomains, b, x0=None, tol: float = 1e-10, maxit: int = 100000, threads: int = 0) -> tuple:
    """The sub-structured CG of ss_cg on `threads` OpenMP threads (0: default)."""
    S = _Sub(sd, A.val)
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    it, rel, tr = C.c_int32(), C.c_double(), C.c_double()
    st = lib_omp().orc_ss_cg_omp(S.ref(), A.n, _p(_i32(A.rowptr)), _p(_i32(A.colidx)), _p(_f64(A.val)), _p(b),
                                 _p(x), tol, maxit, threads, C.byref(it), C.byref(rel), C.byref(tr))
    return x, Result(st, it.value, rel.value, tr.value)


def cg_omp(A, b, x0=None, tol: float = 1e-10, maxit: int = 100000, threads: int = 0) -> tuple:
    """CG on the global matrix on `threads` OpenMP threads (0: default)."""
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    it, rel, tr = C.c_int32(), C.c_double(), C.c_double()
    st = lib_omp().orc_cg_omp(A.n, _p(_i32(A.rowptr)), _p(_i32(A.colidx)), _p(_f64(A.val)), _p(b), _p(x), tol,
                              maxit, threads, C.byref(it), C.byref(rel), C.byref(tr))
    return x, Result(st, it.value, rel.value, tr.value)


def omp_max_threads() -> int:
    return int(lib_omp().orc_omp_max_threads())


def solve_reference(A, b, tol: float = 1e-14, maxit: int = 200000) -> np.ndarray:
    """Solution to the attainable floor: CG on the global matrix run until
    the recomputed residual stops improving."""
    x, res = cg(A, b, tol=tol, maxit=maxit, hist=False)
    return x
