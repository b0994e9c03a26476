"""Sub-structured Conjugate Gradient on MI355X (gfx950) -- Python binding.

A thin ctypes layer over libss.so (include/ss.h): argument marshalling only.
Every step of the solve runs in the library's HIP kernels; PyTorch provides
the device memory (through an allocator callback into its caching allocator)
and the stream.  There is no CPU fallback: without the built library every
call raises.

Method: Cheik Ahamed & Magoules, "Parallel Sub-Structuring Methods for solving
Sparse Linear Systems on a cluster of GPU" -- CG (Algorithm 3) where every
product by the matrix is a local SpMV per sub-domain plus interface assembly
(Section 4.4), with all sub-domains resident on one GPU.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libss.so")

SS_OK, SS_NOT_CONVERGED, SS_EINVAL, SS_ENOMEM, SS_EDEVICE, SS_EBREAKDOWN, SS_EUNSUPPORTED = 0, 1, -1, -2, -3, -4, -5
SS_PART_BOX, SS_PART_RCB, SS_PART_USER, SS_PART_GRAPH = 0, 1, 2, 3
SS_BAND_ROW, SS_BAND_COL = 0, 1
SS_FP64, SS_FP32_IR, SS_FP32_RU = 0, 1, 2
SS_MAT_AUTO, SS_MAT_SELL, SS_MAT_CSR = 0, 1, 2
SS_PRECOND_NONE, SS_PRECOND_JACOBI = 0, 1
SS_SMALL_AUTO, SS_SMALL_OFF = 0, 1
SS_PATH_STREAM, SS_PATH_SMALL = 0, 1
SS_BATCH_CHUNKED, SS_BATCH_PERSISTENT, SS_BATCH_GRAPH = 0, 1, 2

_ALLOC_T = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t)
_FREE_T = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class ss_csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("rowptr", C.c_void_p), ("colidx", C.c_void_p),
                ("val", C.c_void_p)]


class ss_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("inner_tol", C.c_double), ("ru_delta", C.c_double),
                ("inner_maxit", C.c_int32),
                ("max_outer", C.c_int32), ("check_every", C.c_int32), ("use_graph", C.c_int32),
                ("tile_nnz", C.c_int32), ("matrix_format", C.c_int32), ("spmv_grid", C.c_int32),
                ("precond", C.c_int32),
                ("alloc", _ALLOC_T), ("free", _FREE_T),
                ("alloc_ctx", C.c_void_p), ("small_solver", C.c_int32)]


class ss_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("outer_iterations", C.c_int32),
                ("restarts", C.c_int32), ("relres", C.c_double), ("true_relres", C.c_double)]


class ss_batch_tuning(C.Structure):
    _fields_ = [("tile_granules", C.c_int32), ("grid", C.c_int32), ("unroll", C.c_int32),
                ("check_every", C.c_int32), ("schedule", C.c_int32)]


class ss_batch_trial(C.Structure):
    _fields_ = [("tuning", ss_batch_tuning), ("ms_per_iteration", C.c_double)]


class SSError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code}){': ' + detail if detail else ''}")


_lib = None


def lib() -> C.CDLL:
    """The loaded libss.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    P, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "ss_partition": (C.c_int, [P, i32, i32, i32, P, P, P, P, P, P]),
        "ss_part_sizes": (C.c_int, [P, P, P, P, P, P, P]),
        "ss_part_export": (C.c_int, [P, P, P, P, P, P, P, P, P]),
        "ss_part_export_local": (C.c_int, [P, P, P, P]),
        "ss_part_destroy": (None, [P]),
        "ss_opts_default": (None, [P]),
        "ss_cg_setup": (C.c_int, [P, P, P, P, P]),
        "ss_cg_solve": (C.c_int, [P, P, P, dbl, i32, P, P]),
        "ss_cg_solve_noalloc": (C.c_int, [P, P, P, dbl, i32, P, P]),
        "ss_cg_apply": (C.c_int, [P, P, P]),
        "ss_cg_apply_f32": (C.c_int, [P, P, P]),
        "ss_cg_set_values": (C.c_int, [P, P]),
        "ss_cg_grad_vals": (C.c_int, [P, P, P, P]),
        "ss_cg_time_spmv": (C.c_int, [P, i32, P, P]),
        "ss_cg_info": (C.c_int, [P, P, P, P, P, P]),
        "ss_stream_rate": (C.c_int, [i64, i32, i32, P, P, P]),
        "ss_cg_path": (C.c_int, [P, P]),
        "ss_cg_destroy": (None, [P]),
        "ss_band_size": (C.c_int, [P, i32, i32, i32, P, P, P]),
        "ss_band_extract": (C.c_int, [P, i32, i32, i32, P, P, P]),
        "ss_band_setup": (C.c_int, [P, i32, i32, P, P, P]),
        "ss_batch_setup": (C.c_int, [i32, P, i32, P, P, P]),
        "ss_batch_solve": (C.c_int, [P, P, P, dbl, i32, P, P]),
        "ss_batch_set_tuning": (C.c_int, [P, P]),
        "ss_batch_get_tuning": (C.c_int, [P, P]),
        "ss_batch_tune": (C.c_int, [P, P, i32, i32, P, P, i32, P]),
        "ss_batch_info": (C.c_int, [P, P, P, P, P, P]),
        "ss_batch_launches": (C.c_int, [P, P, P, P]),
        "ss_batch_destroy": (None, [P]),
        "ss_strerror": (C.c_char_p, [C.c_int]),
        "ss_last_error": (C.c_char_p, []),
        "ss_version": (C.c_int, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def strerror(code: int) -> str:
    return lib().ss_strerror(code).decode()


def last_error() -> str:
    return lib().ss_last_error().decode()


def _check(code: int, where: str, ok=(SS_OK,)) -> int:
    if code not in ok:
        raise SSError(code, where, last_error())
    return code


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _HostCSR:
    """Keeps host CSR arrays alive while the C side borrows them."""

    def __init__(self, A):
        self.rowptr, self.colidx, self.val = _i32(A.rowptr), _i32(A.colidx), _f64(A.val)
        self.s = ss_csr(int(A.n), int(self.rowptr[-1]), _ptr(self.rowptr), _ptr(self.colidx), _ptr(self.val))

    def ref(self):
        return C.byref(self.s)


# ----------------------------------------------------------------------------
# partitions
# ----------------------------------------------------------------------------

class Partition:
    def __init__(self, handle: C.c_void_p):
        self.h = handle

    def __del__(self):
        h, self.h = getattr(self, "h", None), None
        if h and _lib is not None:
            _lib.ss_part_destroy(h)

    def sizes(self) -> dict:
        return ss_part_sizes(self)

    def export(self) -> dict:
        return ss_part_export(self)

    def export_local(self) -> dict:
        return ss_part_export_local(self)


def ss_partition(A, method: int, nparts: int, grid=None, boxes=None, coords=None, weights=None,
                 user_part=None) -> Partition:
    """Node partition + owner-rule split of A (host arrays); see ss.h."""
    csr = _HostCSR(A)
    g = None if grid is None else _i32(grid)
    bx = None if boxes is None else _i32(boxes)
    cd = None if coords is None else _f64(coords)
    w = None if weights is None else _f64(weights)
    up = None if user_part is None else _i32(user_part)
    dim = len(g) if g is not None else (cd.shape[1] if cd is not None else 0)
    out = C.c_void_p()
    _check(lib().ss_partition(csr.ref(), int(method), int(nparts), int(dim), _ptr(g), _ptr(bx), _ptr(cd), _ptr(w),
                              _ptr(up), C.byref(out)), "ss_partition")
    return Partition(out)


def ss_part_sizes(p: Partition) -> dict:
    v = [C.c_int32() for _ in range(5)] + [C.c_int64()]
    _check(lib().ss_part_sizes(p.h, *[C.byref(t) for t in v]), "ss_part_sizes")
    keys = ["nparts", "n", "n_loc", "n_gamma", "n_copies", "nnz"]
    return {k: t.value for k, t in zip(keys, v)}


def ss_part_export(p: Partition) -> dict:
    z = ss_part_sizes(p)
    out = {
        "part": np.empty(z["n"], np.int32), "sub_off": np.empty(z["nparts"] + 1, np.int32),
        "n_int": np.empty(z["nparts"], np.int32), "n_own": np.empty(z["nparts"], np.int32),
        "l2g": np.empty(z["n_loc"], np.int32), "gamma": np.empty(z["n_gamma"], np.int32),
        "copy_ptr": np.empty(z["n_gamma"] + 1, np.int32), "copy_pos": np.empty(z["n_copies"], np.int32),
    }
    _check(lib().ss_part_export(p.h, *[_ptr(out[k]) for k in out]), "ss_part_export")
    return out


def ss_part_export_local(p: Partition) -> dict:
    z = ss_part_sizes(p)
    out = {"bd_rowptr": np.empty(z["n_loc"] + 1, np.int32), "bd_colidx": np.empty(z["nnz"], np.int32),
           "bd_nzmap": np.empty(z["nnz"], np.int32)}
    _check(lib().ss_part_export_local(p.h, *[_ptr(out[k]) for k in out]), "ss_part_export_local")
    return out


def partition_workload(w, A=None) -> Partition:
    """Partition for a workloads.Workload recipe (box / rcb / single part)."""
    A = w.A if A is None else A
    if w.method == "box":
        return ss_partition(A, SS_PART_BOX, w.nparts, grid=w.grid, boxes=w.boxes)
    if w.method == "rcb":
        return ss_partition(A, SS_PART_RCB, w.nparts, coords=w.coords, weights=w.weights)
    return ss_partition(A, SS_PART_USER, 1, user_part=np.zeros(A.n, np.int32))


# ----------------------------------------------------------------------------
# solver (device side: torch tensors on the current HIP device)
# ----------------------------------------------------------------------------

def _torch():
    import torch

    return torch


class _TorchAllocator:
    """Device memory for the library from torch's caching allocator."""

    def __init__(self, device):
        self.device = device
        self.live = {}
        self.alloc_cb = _ALLOC_T(self._alloc)
        self.free_cb = _FREE_T(self._free)

    def _alloc(self, ctx, nbytes):
        torch = _torch()
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except RuntimeError:
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _free(self, ctx, ptr):
        self.live.pop(ptr, None)


@dataclass
class Result:
    status: int
    iterations: int
    outer_iterations: int
    restarts: int
    relres: float
    true_relres: float
    hist: Optional[np.ndarray] = None


def default_opts(**kw) -> ss_opts:
    o = ss_opts()
    lib().ss_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Solver:
    def __init__(self, h, allocator, stream, n, nnz):
        self.h = h
        self.allocator = allocator
        self.stream = stream
        self.n = n
        self.nnz = nnz

    def __del__(self):
        h, self.h = getattr(self, "h", None), None
        if h and _lib is not None:
            _lib.ss_cg_destroy(h)

    def close(self):
        self.__del__()

    def path(self) -> int:
        """SS_PATH_STREAM or SS_PATH_SMALL (the whole solve in one launch)."""
        v = C.c_int32()
        _check(lib().ss_cg_path(self.h, C.byref(v)), "ss_cg_path")
        return v.value

    def info(self) -> dict:
        v = [C.c_int32(), C.c_int32(), C.c_int64(), C.c_int32(), C.c_int64()]
        _check(lib().ss_cg_info(self.h, *[C.byref(t) for t in v]), "ss_cg_info")
        return dict(zip(["n", "n_loc", "nnz", "matrix_format", "stored"], [t.value for t in v]))


def _dev_f64(t, n: int, name: str):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 tensor on the GPU")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return C.c_void_p(t.data_ptr())


def _dev_f32(t, n: int, name: str):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 tensor on the GPU")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return C.c_void_p(t.data_ptr())


def ss_cg_setup(A, part: Partition, opts: Optional[ss_opts] = None, device=None) -> Solver:
    """Uploads partition `part` of A to the current device; stream = torch's current stream."""
    torch = _torch()
    if not torch.cuda.is_available():
        raise RuntimeError("ss_cg_setup needs a GPU")
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    o = default_opts() if opts is None else opts
    alloc = _TorchAllocator(dev)
    o.alloc = alloc.alloc_cb
    o.free = alloc.free_cb
    o.alloc_ctx = None
    csr = _HostCSR(A)
    stream = torch.cuda.current_stream(dev)
    out = C.c_void_p()
    with torch.cuda.device(dev):
        _check(lib().ss_cg_setup(csr.ref(), part.h, C.byref(o), C.c_void_p(stream.cuda_stream), C.byref(out)),
               "ss_cg_setup")
    return Solver(out, alloc, stream, int(A.n), int(csr.rowptr[-1]))


def ss_band_extract(A, kind: int, nbands: int, p: int) -> tuple:
    """Band p of nbands (SS_BAND_ROW / SS_BAND_COL) of host CSR A:
    (rowptr, colidx, val, ncols)."""
    csr = _HostCSR(A)
    nr, nc, nz = C.c_int32(), C.c_int32(), C.c_int64()
    _check(lib().ss_band_size(csr.ref(), int(kind), int(nbands), int(p), C.byref(nr), C.byref(nc), C.byref(nz)),
           "ss_band_size")
    rp = np.empty(nr.value + 1, dtype=np.int32)
    ci = np.empty(max(nz.value, 1), dtype=np.int32)
    v = np.empty(max(nz.value, 1))
    _check(lib().ss_band_extract(csr.ref(), int(kind), int(nbands), int(p), _ptr(rp), _ptr(ci), _ptr(v)),
           "ss_band_extract")
    return rp, ci[: nz.value], v[: nz.value], nc.value


def ss_band_setup(A, kind: int, nbands: int, opts: Optional[ss_opts] = None, device=None) -> Solver:
    """CG on A with the band-row or band-column splitting into nbands bands
    (all on one device); solve / apply / time with the ss_cg_* calls."""
    torch = _torch()
    if not torch.cuda.is_available():
        raise RuntimeError("ss_band_setup needs a GPU")
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    o = default_opts() if opts is None else opts
    alloc = _TorchAllocator(dev)
    o.alloc = alloc.alloc_cb
    o.free = alloc.free_cb
    o.alloc_ctx = None
    csr = _HostCSR(A)
    stream = torch.cuda.current_stream(dev)
    out = C.c_void_p()
    with torch.cuda.device(dev):
        _check(lib().ss_band_setup(csr.ref(), int(kind), int(nbands), C.byref(o), C.c_void_p(stream.cuda_stream),
                                   C.byref(out)), "ss_band_setup")
    return Solver(out, alloc, stream, int(A.n), int(csr.rowptr[-1]))


def ss_cg_solve(s: Solver, b, x, tol: float = 1e-10, maxit: int = 10000, hist: bool = False) -> Result:
    """Solves A x = b in place on x (device float64 tensors of length n)."""
    pb, px = _dev_f64(b, s.n, "b"), _dev_f64(x, s.n, "x")
    res = ss_result()
    h = np.full(maxit + 1, np.nan) if hist else None
    code = lib().ss_cg_solve(s.h, pb, px, float(tol), int(maxit), C.byref(res), _ptr(h))
    _check(code, "ss_cg_solve", ok=(SS_OK, SS_NOT_CONVERGED, SS_EBREAKDOWN))
    return Result(res.status, res.iterations, res.outer_iterations, res.restarts, res.relres, res.true_relres,
                  None if h is None else h[: res.iterations + 1])


SS_NOALLOC_HIST_MAX = 32768


def ss_cg_solve_noalloc(s: Solver, b, x, tol: float = 1e-10, maxit: int = 10000, hist: bool = False) -> Result:
    """ss_cg_solve without any device allocation (state in the library's fixed
    per-GPU array; calls that overlap on one GPU race)."""
    pb, px = _dev_f64(b, s.n, "b"), _dev_f64(x, s.n, "x")
    res = ss_result()
    h = np.full(maxit + 1, np.nan) if hist else None
    code = lib().ss_cg_solve_noalloc(s.h, pb, px, float(tol), int(maxit), C.byref(res), _ptr(h))
    _check(code, "ss_cg_solve_noalloc", ok=(SS_OK, SS_NOT_CONVERGED, SS_EBREAKDOWN))
    return Result(res.status, res.iterations, res.outer_iterations, res.restarts, res.relres, res.true_relres,
                  None if h is None else h[: res.iterations + 1])


def ss_cg_apply(s: Solver, x, y=None):
    torch = _torch()
    y = torch.empty_like(x) if y is None else y
    _check(lib().ss_cg_apply(s.h, _dev_f64(x, s.n, "x"), _dev_f64(y, s.n, "y")), "ss_cg_apply")
    return y


def ss_cg_apply_f32(s: Solver, x, y=None):
    """y = A32 x in FP32 (solver set up with SS_FP32_IR or SS_FP32_RU)."""
    torch = _torch()
    y = torch.empty_like(x) if y is None else y
    _check(lib().ss_cg_apply_f32(s.h, _dev_f32(x, s.n, "x"), _dev_f32(y, s.n, "y")), "ss_cg_apply_f32")
    return y


def ss_stream_rate(rows: int, slots: int, reps: int = 20) -> tuple:
    """(ms per launch, bytes per launch) of the CG step's streaming pattern
    without gathers on the current device and stream."""
    torch = _torch()
    ms, nb = C.c_double(), C.c_double()
    stream = torch.cuda.current_stream()
    _check(lib().ss_stream_rate(int(rows), int(slots), int(reps), C.c_void_p(stream.cuda_stream), C.byref(ms),
                                C.byref(nb)), "ss_stream_rate")
    return ms.value, nb.value


def ss_cg_set_values(s: Solver, vals) -> None:
    _check(lib().ss_cg_set_values(s.h, _dev_f64(vals, s.nnz, "vals")), "ss_cg_set_values")


def ss_cg_grad_vals(s: Solver, lam, x, dvals=None):
    torch = _torch()
    dvals = torch.empty(s.nnz, dtype=torch.float64, device=x.device) if dvals is None else dvals
    _check(lib().ss_cg_grad_vals(s.h, _dev_f64(lam, s.n, "lambda"), _dev_f64(x, s.n, "x"),
                                 _dev_f64(dvals, s.nnz, "dvals")), "ss_cg_grad_vals")
    return dvals


def ss_cg_time_spmv(s: Solver, reps: int = 20) -> tuple:
    ms, nbytes = C.c_double(), C.c_double()
    _check(lib().ss_cg_time_spmv(s.h, int(reps), C.byref(ms), C.byref(nbytes)), "ss_cg_time_spmv")
    return ms.value, nbytes.value


# ----------------------------------------------------------------------------
# batched solver
# ----------------------------------------------------------------------------

class Batch:
    """Handle of a batch of independent systems (ss_batch_setup)."""

    def __init__(self, h, allocator, stream, sizes, nrhs):
        self.h = h
        self.allocator = allocator
        self.stream = stream
        self.sizes = np.asarray(sizes, dtype=np.int64)
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)])
        self.nrhs = nrhs
        self.nrows = int(self.offsets[-1])

    def __del__(self):
        h, self.h = getattr(self, "h", None), None
        if h and _lib is not None:
            _lib.ss_batch_destroy(h)

    def close(self):
        self.__del__()

    def path(self) -> int:
        """SS_PATH_STREAM or SS_PATH_SMALL (the whole solve in one launch)."""
        v = C.c_int32()
        _check(lib().ss_cg_path(self.h, C.byref(v)), "ss_cg_path")
        return v.value

    def info(self) -> dict:
        v = [C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()]
        _check(lib().ss_batch_info(self.h, *[C.byref(t) for t in v]), "ss_batch_info")
        return dict(zip(["nsys", "nrhs", "nrows", "nnz", "stored"], [t.value for t in v]))

    def launches(self) -> dict:
        """Host-side launches of the last solve (ss_batch_launches)."""
        v = [C.c_int32(), C.c_int32(), C.c_int32()]
        _check(lib().ss_batch_launches(self.h, *[C.byref(t) for t in v]), "ss_batch_launches")
        return dict(zip(["graphs", "chunks", "kernels"], [t.value for t in v]))


def _tuning_dict(t: ss_batch_tuning) -> dict:
    return {"tile_granules": t.tile_granules, "grid": t.grid, "unroll": t.unroll, "check_every": t.check_every,
            "schedule": t.schedule}


def ss_batch_setup(systems, nrhs: int = 4, opts: Optional[ss_opts] = None, device=None) -> Batch:
    """Uploads the systems (host CSR objects) for nrhs right-hand sides each."""
    torch = _torch()
    if not torch.cuda.is_available():
        raise RuntimeError("ss_batch_setup needs a GPU")
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    o = default_opts() if opts is None else opts
    alloc = _TorchAllocator(dev)
    o.alloc, o.free, o.alloc_ctx = alloc.alloc_cb, alloc.free_cb, None
    host = [_HostCSR(A) for A in systems]
    arr = (ss_csr * len(host))(*[h.s for h in host])
    stream = torch.cuda.current_stream(dev)
    out = C.c_void_p()
    with torch.cuda.device(dev):
        _check(lib().ss_batch_setup(len(host), arr, int(nrhs), C.byref(o), C.c_void_p(stream.cuda_stream),
                                    C.byref(out)), "ss_batch_setup")
    return Batch(out, alloc, stream, [A.n for A in systems], int(nrhs))


def ss_batch_solve(bt: Batch, b, x, tol: float = 1e-10, maxit: int = 100000):
    """Solves every (system, rhs) pair in place on x.  b, x: device float64
    tensors of nrows * nrhs elements, row-major [row][rhs] with the systems'
    rows concatenated.  Returns (per-pair Result list in (system, rhs) order,
    summary Result)."""
    n = bt.nrows * bt.nrhs
    pb, px = _dev_f64(b, n, "b"), _dev_f64(x, n, "x")
    np_ = len(bt.sizes) * bt.nrhs
    res = (ss_result * np_)()
    summ = ss_result()
    code = lib().ss_batch_solve(bt.h, pb, px, float(tol), int(maxit), res, C.byref(summ))
    _check(code, "ss_batch_solve", ok=(SS_OK, SS_NOT_CONVERGED, SS_EBREAKDOWN))
    conv = lambda r: Result(r.status, r.iterations, r.outer_iterations, r.restarts, r.relres, r.true_relres)
    return [conv(r) for r in res], conv(summ)


def ss_batch_tune(bt: Batch, b, iters: int = 8, force: bool = False):
    """Autotuner: returns (chosen tuning dict, list of (tuning dict, ms per iteration))."""
    n = bt.nrows * bt.nrhs
    cap = 64
    trials = (ss_batch_trial * cap)()
    nt = C.c_int32()
    chosen = ss_batch_tuning()
    _check(lib().ss_batch_tune(bt.h, _dev_f64(b, n, "b"), int(iters), int(bool(force)), C.byref(chosen), trials,
                               cap, C.byref(nt)), "ss_batch_tune")
    return _tuning_dict(chosen), [(_tuning_dict(trials[i].tuning), trials[i].ms_per_iteration)
                                  for i in range(nt.value)]


def ss_batch_set_tuning(bt: Batch, tile_granules: int, grid: int, unroll: int, check_every: int,
                        schedule: int = SS_BATCH_CHUNKED) -> None:
    t = ss_batch_tuning(tile_granules, grid, unroll, check_every, schedule)
    _check(lib().ss_batch_set_tuning(bt.h, C.byref(t)), "ss_batch_set_tuning")


def ss_batch_get_tuning(bt: Batch) -> dict:
    t = ss_batch_tuning()
    _check(lib().ss_batch_get_tuning(bt.h, C.byref(t)), "ss_batch_get_tuning")
    return _tuning_dict(t)


def pack_batch(blocks) -> np.ndarray:
    """Host helper: per-system [n_s, nrhs] arrays -> the flat batch layout."""
    return np.ascontiguousarray(np.concatenate([np.asarray(b, dtype=np.float64) for b in blocks], axis=0)).ravel()


# ----------------------------------------------------------------------------
# differentiable solve (adjoint CG)
# ----------------------------------------------------------------------------

def _autograd_function():
    torch = _torch()

    class SSCGSolve(torch.autograd.Function):
        """x = A(vals)^{-1} b through the sub-structured CG, differentiable in
        vals (the global stored entries, in CSR order) and b.

        Backward: one more solve with the same symmetric A gives
        lambda = A^{-1} dL/dx; then dL/db = lambda and, for every stored
        entry k = (i, j) taken as an independent parameter,
        dL/dvals_k = -lambda_i x_j.  A perturbation that keeps A symmetric
        moves the (i, j) and (j, i) entries together; its derivative is the
        sum of the two components.
        """

        @staticmethod
        def forward(ctx, vals, b, solver, tol=1e-10, maxit=100000, adj_tol=None):
            ss_cg_set_values(solver, vals.detach().contiguous())
            x = torch.zeros_like(b)
            res = ss_cg_solve(solver, b.detach().contiguous(), x, tol=tol, maxit=maxit)
            if res.status != SS_OK:
                raise SSError(res.status, "SSCGSolve.forward")
            ctx.solver = solver
            ctx.adj = (tol if adj_tol is None else adj_tol, maxit)
            ctx.save_for_backward(vals, x)
            ctx.forward_result = res
            return x

        @staticmethod
        def backward(ctx, gx):
            vals, x = ctx.saved_tensors
            solver = ctx.solver
            ss_cg_set_values(solver, vals.detach().contiguous())
            lam = torch.zeros_like(x)
            res = ss_cg_solve(solver, gx.detach().contiguous(), lam, tol=ctx.adj[0], maxit=ctx.adj[1])
            if res.status != SS_OK:
                raise SSError(res.status, "SSCGSolve.backward")
            dvals = ss_cg_grad_vals(solver, lam, x) if ctx.needs_input_grad[0] else None
            db = lam if ctx.needs_input_grad[1] else None
            return dvals, db, None, None, None, None

    return SSCGSolve


_SSCGSolve = None


def sscg_solve(vals, b, solver: Solver, tol: float = 1e-10, maxit: int = 100000, adj_tol: Optional[float] = None):
    """Differentiable x = A(vals)^{-1} b on `solver` (set up for A's pattern)."""
    global _SSCGSolve
    if _SSCGSolve is None:
        _SSCGSolve = _autograd_function()
    return _SSCGSolve.apply(vals, b, solver, tol, maxit, adj_tol)
