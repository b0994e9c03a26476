"""Seeded generators of sparse SPD systems in CSR form (0-based, int32 indices).

Grid numbering is x fastest: node id = x + Mx*(y + My*z).  Dirichlet boundary
nodes are eliminated, boundary faces/elements still contribute to the diagonal
of the interior nodes next to them.  Rows hold their columns in ascending order
and every matrix is bitwise symmetric (each off-diagonal value is computed once
per unordered pair and stored at both positions).

Seeds: matrix seed = configuration index, right-hand-side seed = 100 + index,
RCB target weights seed 3, adjoint target seed 205.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclass
class CSR:
    """Compressed sparse row storage: row pointers, column indices, values.

    The paper stores AA (values), JA (column indices) and IA (row pointers),
    1-based (Section 2.2); here the same three arrays are 0-based.
    """

    n: int
    rowptr: np.ndarray  # int32 [n+1]
    colidx: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def row_of_nz(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.rowptr))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n), dtype=self.val.dtype)
        d[self.row_of_nz(), self.colidx] = self.val
        return d


@dataclass
class Workload:
    """One synthetic system plus the recipe for partitioning it."""

    name: str
    A: CSR
    b: np.ndarray
    dim: int = 0
    grid: Tuple[int, ...] = ()  # nodes per axis, (Mx, My[, Mz])
    boxes: Tuple[int, ...] = ()  # boxes per axis for a box partition
    method: str = "box"  # "box" | "rcb" | "user" | "none"
    nparts: int = 1
    coords: Optional[np.ndarray] = None  # [n, dim] for RCB
    weights: Optional[np.ndarray] = None  # [nparts] RCB target weights
    extra: Dict[str, object] = field(default_factory=dict)


# ----------------------------------------------------------------------------
# stencil assembly helper
# ----------------------------------------------------------------------------

def _stencil_csr(shape_zyx: Tuple[int, int, int],
                 entries: Sequence[Tuple[Tuple[int, int, int], np.ndarray]]) -> CSR:
    """CSR from per-offset value arrays on a structured grid.

    ``entries`` is a list of ((dz, dy, dx), values[Mz, My, Mx]) sorted by
    (dz, dy, dx); the value at node u is the entry A[u, u + offset] and is
    dropped where u + offset falls outside the grid.  Sorting the offsets
    lexicographically gives ascending column indices in every row.
    """
    Mz, My, Mx = shape_zyx
    N = Mz * My * Mx
    K = len(entries)
    z, y, x = np.indices((Mz, My, Mx), dtype=np.int64)
    ids = np.arange(N, dtype=np.int64)
    mask = np.empty((N, K), dtype=bool)
    vals = np.empty((N, K), dtype=np.float64)
    cols = np.empty((N, K), dtype=np.int32)
    for k, ((dz, dy, dx), v) in enumerate(entries):
        ok = ((z + dz >= 0) & (z + dz < Mz) & (y + dy >= 0) & (y + dy < My)
              & (x + dx >= 0) & (x + dx < Mx))
        mask[:, k] = ok.ravel()
        vals[:, k] = np.broadcast_to(v, (Mz, My, Mx)).ravel()
        cols[:, k] = (ids + dx + Mx * (dy + My * dz)).astype(np.int32)
    counts = mask.sum(axis=1)
    rowptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    return CSR(N, rowptr.astype(np.int32), cols[mask], vals[mask])


def _faces_to_csr2d(cx: np.ndarray, cy: np.ndarray) -> CSR:
    """5-point operator from x-face and y-face coefficients.

    cx[y, fx] couples nodes (fx-1, y) and (fx, y); cy[fy, x] couples (x, fy-1)
    and (x, fy).  Faces at fx in {0, Mx} / fy in {0, My} touch the boundary.
    a_ii = sum of the four faces of node i, a_ij = -c_face.
    """
    My, Mx1 = cx.shape
    Mx = Mx1 - 1
    diag = ((cx[:, :-1] + cx[:, 1:]) + cy[:-1, :]) + cy[1:, :]
    sh = (1, My, Mx)
    ent = [
        ((0, -1, 0), -cy[:-1, :].reshape(sh)),
        ((0, 0, -1), -cx[:, :-1].reshape(sh)),
        ((0, 0, 0), diag.reshape(sh)),
        ((0, 0, 1), -cx[:, 1:].reshape(sh)),
        ((0, 1, 0), -cy[1:, :].reshape(sh)),
    ]
    return _stencil_csr(sh, ent)


def _faces_to_csr3d(cx: np.ndarray, cy: np.ndarray, cz: np.ndarray) -> CSR:
    """7-point operator from face coefficients (cx: [Mz, My, Mx+1], ...)."""
    Mz, My, Mx1 = cx.shape
    Mx = Mx1 - 1
    diag = (((((cx[:, :, :-1] + cx[:, :, 1:]) + cy[:, :-1, :]) + cy[:, 1:, :])
             + cz[:-1, :, :]) + cz[1:, :, :])
    ent = [
        ((-1, 0, 0), -cz[:-1, :, :]),
        ((0, -1, 0), -cy[:, :-1, :]),
        ((0, 0, -1), -cx[:, :, :-1]),
        ((0, 0, 0), diag),
        ((0, 0, 1), -cx[:, :, 1:]),
        ((0, 1, 0), -cy[:, 1:, :]),
        ((1, 0, 0), -cz[1:, :, :]),
    ]
    return _stencil_csr((Mz, My, Mx), ent)


# ----------------------------------------------------------------------------
# matrices
# ----------------------------------------------------------------------------

def poisson2d(m: int, my: Optional[int] = None) -> CSR:
    """5-point Laplacian on an m x my interior grid: a_ii = 4, a_ij = -1.

    Integer valued, so every sum of products of it with integer vectors is
    exact in FP64 as long as the magnitudes stay below 2**53.
    """
    my = m if my is None else my
    cx = np.ones((my, m + 1))
    cy = np.ones((my + 1, m))
    return _faces_to_csr2d(cx, cy)


def poisson3d(m: int) -> CSR:
    """7-point Laplacian on an m^3 interior grid: a_ii = 6, a_ij = -1 (integer
    valued, x fastest), assembled directly for large grids."""
    N = m * m * m
    ids = np.arange(N, dtype=np.int64)
    x, y, z = ids % m, (ids // m) % m, ids // (m * m)
    # the seven offsets in ascending column order
    offs = [(-m * m, z > 0), (-m, y > 0), (-1, x > 0), (0, None), (1, x < m - 1), (m, y < m - 1),
            (m * m, z < m - 1)]
    mask = np.ones((N, 7), dtype=bool)
    cols = np.empty((N, 7), dtype=np.int32)
    for k, (d, ok) in enumerate(offs):
        if ok is not None:
            mask[:, k] = ok
        cols[:, k] = ids + d
    vals = np.broadcast_to(np.array([-1.0, -1.0, -1.0, 6.0, -1.0, -1.0, -1.0]), (N, 7))
    rowptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(mask.sum(axis=1), out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32")
    return CSR(N, rowptr.astype(np.int32), cols[mask], vals[mask])


def diffusion2d_lognormal(m: int, rng: np.random.Generator, my: Optional[int] = None) -> CSR:
    """5-point variable-coefficient diffusion; faces exp(N(0,1)) drawn x-faces first."""
    my = m if my is None else my
    cx = np.exp(rng.standard_normal((my, m + 1)))
    cy = np.exp(rng.standard_normal((my + 1, m)))
    return _faces_to_csr2d(cx, cy)


def diffusion3d_lognormal(M: int, seed: int, sigma: float = 1.0) -> CSR:
    """7-point diffusion on M^3 with i.i.d. face coefficients exp(N(0, sigma^2)).

    All 3*(M+1)*M^2 faces are drawn, boundary faces included; draw order is
    x-faces [z, y, fx], then y-faces [z, fy, x], then z-faces [fz, y, x].
    """
    rng = np.random.default_rng(seed)
    cx = np.exp(sigma * rng.standard_normal((M, M, M + 1)))
    cy = np.exp(sigma * rng.standard_normal((M, M + 1, M)))
    cz = np.exp(sigma * rng.standard_normal((M + 1, M, M)))
    return _faces_to_csr3d(cx, cy, cz)


def gaussian_random_field(shape: Tuple[int, ...], seed: int, smooth: float = 4.0) -> np.ndarray:
    """White noise N(0,1) smoothed by a Gaussian (sigma=`smooth` nodes, cut at
    3 sigma, reflecting edges), then standardised to mean 0 / std 1."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    g = gaussian_filter(w, sigma=smooth, mode="reflect", truncate=3.0)
    return (g - g.mean()) / g.std()


def diffusion3d_grf(M: int, seed: int, smooth: float = 4.0) -> CSR:
    """7-point diffusion on M^3 with face coefficients exp((g_i + g_j)/2), where
    g is a smoothed Gaussian random field on the (M+2)^3 grid that includes
    the Dirichlet boundary layer."""
    g = gaussian_random_field((M + 2, M + 2, M + 2), seed, smooth)
    gi = g[1:-1, 1:-1, :]  # [M, M, M+2] along x
    cx = np.exp((gi[:, :, :-1] + gi[:, :, 1:]) / 2.0)
    gj = g[1:-1, :, 1:-1]
    cy = np.exp((gj[:, :-1, :] + gj[:, 1:, :]) / 2.0)
    gk = g[:, 1:-1, 1:-1]
    cz = np.exp((gk[:-1, :, :] + gk[1:, :, :]) / 2.0)
    return _faces_to_csr3d(cx, cy, cz)


def q1hex_lognormal(M: int, seed: int, sigma: float = 0.5) -> CSR:
    """Trilinear (Q1) hexahedral FE stiffness of -div(c grad u) on (M+1)^3 unit
    elements, Dirichlet boundary eliminated: M^3 unknowns, 27-point stencil.

    Element coefficients c_e = exp(N(0, sigma^2)), drawn [ez, ey, ex].  The
    unit-cube Q1 Laplacian element matrix is (1/12) * {4 on the diagonal, 0
    between nodes sharing an element edge, -1 between nodes on a face diagonal
    or the body diagonal}.  Assembled: a node pair at offset d shares
    2**(number of zero components of d) elements; axis neighbours get an exact
    0 that stays stored, so every row of an interior node has 27 entries.
    """
    rng = np.random.default_rng(seed)
    ne = M + 1
    C = np.exp(sigma * rng.standard_normal((ne, ne, ne)))

    def el(sz: int, sy: int, sx: int) -> np.ndarray:
        # coefficient of the element with lower corner index (z+sz, y+sy, x+sx)
        return C[sz:sz + M, sy:sy + M, sx:sx + M]

    ent = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                d = (dz, dy, dx)
                nz = sum(1 for t in d if t != 0)
                if nz == 0:
                    acc = None
                    for a in (0, 1):
                        for b in (0, 1):
                            for c in (0, 1):
                                acc = el(a, b, c) if acc is None else acc + el(a, b, c)
                    v = acc / 3.0
                elif nz == 1:
                    v = np.zeros((M, M, M))
                else:
                    # shared elements: per axis, +1 -> shift 1, -1 -> shift 0,
                    # 0 -> both shifts (lower one first)
                    choices = [((1,) if t == 1 else (0,) if t == -1 else (0, 1)) for t in d]
                    acc = None
                    for a in choices[0]:
                        for b in choices[1]:
                            for c in choices[2]:
                                acc = el(a, b, c) if acc is None else acc + el(a, b, c)
                    v = -acc / 12.0
                ent.append((d, v))
    return _stencil_csr((M, M, M), ent)


def random_spd_csr(n: int, avg_offdiag: float, seed: int, integer: bool = False) -> CSR:
    """Random sparse, strictly diagonally dominant symmetric matrix (hence SPD).

    Off-diagonal values U[-1,1] (or integers in [-3,3] when ``integer``),
    diagonal = sum of |off-diagonals| of the row + U[0.5, 1.5] (or +1).
    """
    rng = np.random.default_rng(seed)
    m = int(round(avg_offdiag * n / 2))
    i = rng.integers(0, n, size=m)
    j = rng.integers(0, n, size=m)
    keep = i != j
    i, j = i[keep], j[keep]
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    key = np.unique(lo.astype(np.int64) * n + hi)
    lo, hi = key // n, key % n
    if integer:
        v = rng.integers(-3, 4, size=len(lo)).astype(np.float64)
        v[v == 0] = 1.0
    else:
        v = rng.uniform(-1.0, 1.0, size=len(lo))
    rows = np.concatenate([lo, hi, np.arange(n)])
    cols = np.concatenate([hi, lo, np.arange(n)])
    absrow = np.zeros(n)
    np.add.at(absrow, lo, np.abs(v))
    np.add.at(absrow, hi, np.abs(v))
    diag = absrow + (1.0 if integer else rng.uniform(0.5, 1.5, size=n))
    vals = np.concatenate([v, v, diag])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return CSR(n, rowptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


def batch2d_lognormal(nsys: int, nmin: int, nmax: int, seed: int) -> List[CSR]:
    """Independent 5-point lognormal(0,1) systems on n_k x n_k grids, n_k drawn
    uniformly from the integers in [nmin, nmax]; faces drawn system by system."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=nsys)
    return [diffusion2d_lognormal(int(m), rng) for m in sizes]


# ----------------------------------------------------------------------------
# vectors, coordinates, weights
# ----------------------------------------------------------------------------

def uniform_rhs(n: int, seed: int, k: Optional[int] = None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=n if k is None else (n, k))


def rcb_weights(nparts: int, seed: int = 3, spread: float = 0.3) -> np.ndarray:
    """Target sub-domain weights U[1-spread, 1+spread] (uneven sub-domains)."""
    return np.random.default_rng(seed).uniform(1.0 - spread, 1.0 + spread, size=nparts)


def grid_coords(shape_xyz: Sequence[int]) -> np.ndarray:
    """Integer node coordinates (x, y[, z]) as float64, node id x-fastest."""
    dims = len(shape_xyz)
    grids = np.indices(tuple(reversed(shape_xyz)))  # [z, y, x] order
    cols = [grids[dims - 1 - a].ravel() for a in range(dims)]
    return np.stack(cols, axis=1).astype(np.float64)


# ----------------------------------------------------------------------------
# the five workloads (optionally scaled down for parity runs)
# ----------------------------------------------------------------------------

CONFIG_NAMES = {
    1: "poisson2d_64x64_box2x2",
    2: "diffusion3d_lognormal_128c_box2x2x2",
    3: "q1hex_lognormal_96c_rcb16",
    4: "batch256_diffusion2d_lognormal_32to256_rhs4",
    5: "diffusion3d_grf_64c_box2x2x2_adjoint",
}


def config(idx: int, size: Optional[int] = None, nsys: Optional[int] = None) -> Workload:
    """Workload `idx` (1..5).  ``size`` overrides the grid edge (nodes per axis
    of the interior grid) to get a smaller instance of the same recipe."""
    if idx == 1:
        m = 64 if size is None else size
        A = poisson2d(m)
        return Workload(f"poisson2d_{m}x{m}_box2x2", A, uniform_rhs(A.n, 101), dim=2,
                        grid=(m, m), boxes=(2, 2), method="box", nparts=4)
    if idx == 2:
        M = 128 if size is None else size
        A = diffusion3d_lognormal(M, seed=2)
        return Workload(f"diffusion3d_lognormal_{M}c_box2x2x2", A, uniform_rhs(A.n, 102), dim=3,
                        grid=(M, M, M), boxes=(2, 2, 2), method="box", nparts=8)
    if idx == 3:
        M = 96 if size is None else size
        A = q1hex_lognormal(M, seed=3)
        return Workload(f"q1hex_lognormal_{M}c_rcb16", A, uniform_rhs(A.n, 103), dim=3,
                        grid=(M, M, M), method="rcb", nparts=16,
                        coords=grid_coords((M, M, M)), weights=rcb_weights(16, seed=3))
    if idx == 4:
        ns = 256 if nsys is None else nsys
        hi = 256 if size is None else size
        lo = min(32, hi)
        systems = batch2d_lognormal(ns, lo, hi, seed=4)
        rng = np.random.default_rng(104)
        B = [rng.uniform(-1.0, 1.0, size=(S.n, 4)) for S in systems]
        first = systems[0]
        w = Workload(f"batch{ns}_diffusion2d_lognormal_{lo}to{hi}_rhs4", first, B[0][:, 0],
                     method="none", nparts=1)
        w.extra["systems"] = systems
        w.extra["rhs"] = B
        return w
    if idx == 5:
        M = 64 if size is None else size
        A = diffusion3d_grf(M, seed=5)
        w = Workload(f"diffusion3d_grf_{M}c_box2x2x2_adjoint", A, uniform_rhs(A.n, 105), dim=3,
                     grid=(M, M, M), boxes=(2, 2, 2), method="box", nparts=8)
        w.extra["x_target"] = np.random.default_rng(205).uniform(-1.0, 1.0, size=A.n)
        return w
    raise ValueError(f"unknown configuration {idx}")
