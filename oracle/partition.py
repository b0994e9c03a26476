"""Oracle (test infrastructure only): partitions and sub-domain maps in numpy.

Only tests/, the smoke check and the bench's CPU-baseline leg may import this
package.  It shares no code with the HIP library.

What is computed follows the sub-structuring splitting of Section 3.4: the
unknowns are split into sub-domains, every sub-domain knows its own nodes plus
the interface nodes it touches (interior sets 1, 2 and interface set 3 of the
block matrix S), and the interface block of the global matrix is the sum of
the sub-domain contributions (S_33 = S_33^(1) + S_33^(2)).  The paper obtains
the node partition from METIS (Section 5.3); here the node partition is a box
(grid) cut, a weighted recursive coordinate bisection or a user array.

The split of an assembled matrix into local matrices is not spelled out in the
paper (it assumes finite-element assembly).  Reading adopted: every stored
entry (i, j) belongs to exactly one sub-domain, o(i,j) = P(i) for i == j and
min(P(i), P(j)) otherwise.  Then sum_s R_s^T A_s R_s == A holds entry by entry
with no floating-point operation.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np


# ----------------------------------------------------------------------------
# node partitions
# ----------------------------------------------------------------------------

def box_partition(grid: Sequence[int], boxes: Sequence[int]) -> np.ndarray:
    """Part of every grid node for a cut of the grid into boxes.

    grid = nodes per axis (x first), node id = x + Mx*(y + My*z).  Along an
    axis with M nodes and B boxes, box b starts at floor(b*M/B); a node with
    coordinate c lies in the last box whose start is <= c.
    Part id = bx + Bx*(by + By*bz).
    """
    grid = [int(g) for g in grid]
    boxes = [int(b) for b in boxes]
    n = int(np.prod(grid))
    ids = np.arange(n, dtype=np.int64)
    part = np.zeros(n, dtype=np.int64)
    stride_node = 1
    stride_part = 1
    for M, B in zip(grid, boxes):
        c = (ids // stride_node) % M
        starts = np.array([(b * M) // B for b in range(B)], dtype=np.int64)
        bidx = np.searchsorted(starts, c, side="right") - 1
        part += bidx * stride_part
        stride_node *= M
        stride_part *= B
    return part.astype(np.int32)


def _seq_sum(values) -> float:
    acc = 0.0
    for v in values:
        acc = acc + float(v)
    return acc


def rcb_partition(coords: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """Weighted recursive coordinate bisection into len(weights) parts.

    A node set S assigned to the part range [lo, hi) is split along the axis of
    largest coordinate extent (ties: lowest axis first); the nodes are ordered
    by (coordinate on that axis, global id) and the first
    floor(|S| * W[lo,mid) / W[lo,hi) + 0.5) go to [lo, mid) with
    mid = (lo + hi) // 2, the rest to [mid, hi).  Weight sums are sequential,
    left to right.  The paper asks for balanced, compact ("spherical")
    sub-structures with small boundaries (Section 3.3); the weights make them
    deliberately uneven.
    """
    coords = np.asarray(coords, dtype=np.float64)
    n = coords.shape[0]
    part = np.full(n, -1, dtype=np.int32)
    w = [float(v) for v in weights]

    def rec(S: np.ndarray, lo: int, hi: int) -> None:
        if hi - lo == 1:
            part[S] = lo
            return
        mid = (lo + hi) // 2
        if len(S) > 0:
            sub = coords[S]
            ext = sub.max(axis=0) - sub.min(axis=0)
            axis = int(np.argmax(ext))
            order = np.lexsort((S, sub[:, axis]))
            S = S[order]
        wl = _seq_sum(w[lo:mid])
        wt = _seq_sum(w[lo:hi])
        nleft = int(np.floor(len(S) * wl / wt + 0.5))
        rec(S[:nleft], lo, mid)
        rec(S[nleft:], mid, hi)

    rec(np.arange(n, dtype=np.int64), 0, len(w))
    return part


# ----------------------------------------------------------------------------
# owner-rule split into sub-domains
# ----------------------------------------------------------------------------

@dataclass
class SubDomains:
    """Sub-domain data in concatenated local numbering.

    Sub-domain s occupies positions [sub_off[s], sub_off[s+1]) and orders its
    nodes as: interior (multiplicity 1) ascending by global id, then interface
    nodes it owns (multiplicity > 1, P(i) == s) ascending, then the other
    interface nodes it touches ("ghost" copies) ascending.  Positions
    [sub_off[s], sub_off[s] + n_int[s] + n_own[s]) are the owned positions.
    """

    nparts: int
    part: np.ndarray  # [n]
    mult: np.ndarray  # [n] multiplicity m_i
    sub_off: np.ndarray  # [P+1]
    n_int: np.ndarray  # [P]
    n_own: np.ndarray  # [P]
    l2g: np.ndarray  # [n_loc]
    gamma: np.ndarray  # [n_gamma] interface nodes, ascending global id
    copy_ptr: np.ndarray  # [n_gamma+1]
    copy_pos: np.ndarray  # [n_copies] positions of the copies, ascending sub-domain
    bd_rowptr: np.ndarray  # [n_loc+1] block-diagonal CSR of all local matrices
    bd_colidx: np.ndarray  # [nnz] concatenated positions
    bd_nzmap: np.ndarray  # [nnz] index of the global stored entry

    @property
    def n_loc(self) -> int:
        return int(self.sub_off[-1])

    def bd_values(self, val: np.ndarray) -> np.ndarray:
        return np.asarray(val)[self.bd_nzmap]


def split(rowptr: np.ndarray, colidx: np.ndarray, part: np.ndarray, nparts: int) -> SubDomains:
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    part = np.asarray(part, dtype=np.int64)
    n = len(part)
    P = int(nparts)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    cols = colidx
    # owner of every stored entry
    owner = np.where(rows == cols, part[rows], np.minimum(part[rows], part[cols]))
    # V_s: nodes of part s, plus both end points of every entry owned by s
    keys = np.unique(np.concatenate([
        part * n + np.arange(n, dtype=np.int64),
        owner * n + rows,
        owner * n + cols,
    ]))
    mem_s = keys // n
    mem_i = keys % n
    mult = np.bincount(mem_i, minlength=n)
    # class of every membership: 0 interior, 1 owned interface, 2 ghost
    cls = np.where(mult[mem_i] == 1, 0, np.where(part[mem_i] == mem_s, 1, 2))
    # local order: by sub-domain, then class, then global id
    order = np.lexsort((mem_i, cls, mem_s))
    pos_of_key = np.empty(len(keys), dtype=np.int64)
    pos_of_key[order] = np.arange(len(keys), dtype=np.int64)
    n_s = np.bincount(mem_s, minlength=P)
    sub_off = np.zeros(P + 1, dtype=np.int64)
    np.cumsum(n_s, out=sub_off[1:])
    n_int = np.bincount(mem_s[cls == 0], minlength=P)
    n_own = np.bincount(mem_s[cls == 1], minlength=P)
    l2g = mem_i[order]

    # interface nodes and the positions of their copies (ascending sub-domain)
    gamma = np.nonzero(mult > 1)[0]
    sel = mult[mem_i] > 1
    gkeys_i = mem_i[sel]
    gkeys_s = mem_s[sel]
    gpos = pos_of_key[sel]
    gorder = np.lexsort((gkeys_s, gkeys_i))
    copy_pos = gpos[gorder]
    copy_ptr = np.zeros(len(gamma) + 1, dtype=np.int64)
    np.cumsum(mult[gamma], out=copy_ptr[1:])

    # local matrices: entry (i, j) of owner s sits in row pos(s,i), column pos(s,j)
    rpos = pos_of_key[np.searchsorted(keys, owner * n + rows)]
    cpos = pos_of_key[np.searchsorted(keys, owner * n + cols)]
    eorder = np.lexsort((cpos, rpos))
    n_loc = int(sub_off[-1])
    bd_rowptr = np.zeros(n_loc + 1, dtype=np.int64)
    np.cumsum(np.bincount(rpos, minlength=n_loc), out=bd_rowptr[1:])

    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)  # noqa: E731
    return SubDomains(
        nparts=P, part=i32(part), mult=i32(mult), sub_off=i32(sub_off), n_int=i32(n_int),
        n_own=i32(n_own), l2g=i32(l2g), gamma=i32(gamma), copy_ptr=i32(copy_ptr),
        copy_pos=i32(copy_pos), bd_rowptr=i32(bd_rowptr), bd_colidx=i32(cpos[eorder]),
        bd_nzmap=i32(np.arange(len(rows))[eorder]),
    )


def partition_workload(w, part: Optional[np.ndarray] = None) -> np.ndarray:
    """Node partition for a workloads.Workload recipe."""
    if part is not None:
        return np.asarray(part, dtype=np.int32)
    if w.method == "box":
        return box_partition(w.grid, w.boxes)
    if w.method == "rcb":
        return rcb_partition(w.coords, w.weights)
    if w.method in ("none", "user"):
        return np.zeros(w.A.n, dtype=np.int32)
    raise ValueError(w.method)
