"""The FP32 product of the mixed-precision modes through the C-ABI
(ss_cg_apply_f32) against the oracle's FP32 sub-structured product, bit for
bit: the values rounded to FP32, every local row summed left to right with
each product and sum rounded to FP32, then the interface copies added in
ascending sub-domain order in FP32 (Section 4.4.1, Algorithms 4 and 5).  The
oracle's FP32 arithmetic is pinned on the CPU against an independent
evaluation (tests/test_oracle_pins.py)."""
import numpy as np
import pytest

import oracle as O
import paper_2108_13162_amd as ss
from workloads import config, diffusion3d_lognormal, uniform_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _x32(n, seed):
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n).astype(np.float32)


def _apply32(s, x32):
    x = torch.tensor(x32, device=DEV)
    return ss.ss_cg_apply_f32(s, x).cpu().numpy()


@pytest.fixture(scope="module")
def q1():
    w = config(3, size=20)  # Q1 hexahedra, 20^3 unknowns, 16 weighted RCB parts
    sd = O.split(w.A.rowptr, w.A.colidx, O.rcb_partition(w.coords, w.weights), 16)
    return w, ss.partition_workload(w), sd


@pytest.mark.parametrize("prec", ["SS_FP32_IR", "SS_FP32_RU"])
def test_apply_f32_bitwise_q1(q1, prec):
    w, p, sd = q1
    s = ss.ss_cg_setup(w.A, p, ss.default_opts(precision=getattr(ss, prec)))
    for seed in (1, 2):
        x32 = _x32(w.A.n, seed)
        y = _apply32(s, x32)
        yo = O.ss_spmv_f32(w.A, sd, x32)
        assert y.dtype == np.float32
        assert np.array_equal(y.view(np.uint32), yo.view(np.uint32)), np.flatnonzero(y != yo)[:10]
    # the comparison tells FP32 arithmetic apart from an FP64 product rounded once
    y64 = O.csr_matvec(w.A, x32.astype(np.float64)).astype(np.float32)
    assert np.count_nonzero(y != y64) > w.A.n // 10


@pytest.mark.parametrize("fmt", ["SS_MAT_SELL", "SS_MAT_CSR"])
def test_apply_f32_bitwise_formats_7pt(fmt):
    # lognormal 7-point diffusion, 3 x 2 x 2 boxes (ragged box sizes), both storages
    M = 23
    A = diffusion3d_lognormal(M, seed=17)
    part = O.box_partition((M, M, M), (3, 2, 2))
    sd = O.split(A.rowptr, A.colidx, part, 12)
    p = ss.ss_partition(A, ss.SS_PART_BOX, 12, grid=(M, M, M), boxes=(3, 2, 2))
    s = ss.ss_cg_setup(A, p, ss.default_opts(precision=ss.SS_FP32_RU, matrix_format=getattr(ss, fmt)))
    x32 = _x32(A.n, 3)
    assert np.array_equal(_apply32(s, x32).view(np.uint32), O.ss_spmv_f32(A, sd, x32).view(np.uint32))


def test_apply_f32_needs_fp32_values():
    A = diffusion3d_lognormal(6, seed=1)
    p = ss.ss_partition(A, ss.SS_PART_BOX, 8, grid=(6, 6, 6), boxes=(2, 2, 2))
    s = ss.ss_cg_setup(A, p)
    with pytest.raises(ss.SSError) as e:
        _apply32(s, _x32(A.n, 0))
    assert e.value.code == ss.SS_EUNSUPPORTED
