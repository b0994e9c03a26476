"""Randomized apply parity through the C-ABI: random SPD matrices (1 to 80k
rows; the large ones couple rows far apart, so their chunks take int32
columns), random partitions given as part arrays (1 to 9 parts, some empty,
scattered or in contiguous blocks), both storage formats, integer and float
data.  The sub-structured product must equal the oracle's on the same
partition bit for bit: both sides round each product, add a local row left to
right in column order and add an interface node's copies in ascending
sub-domain order."""
import numpy as np
import pytest

import oracle as O
import paper_2108_13162_amd as ss
from workloads import random_spd_csr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(40000, 80000)) if seed % 6 == 5 else int(rng.integers(1, 3000))
    A = random_spd_csr(n, float(rng.uniform(0.0, 12.0)), seed=2000 + seed, integer=seed % 3 == 0)
    P = int(rng.integers(1, 10))
    part = rng.integers(0, P, size=n).astype(np.int32)
    if seed % 5 == 4 and P > 1:
        part[part == P // 2] = 0  # an empty part in the middle
    if seed % 2 == 0:
        part = np.sort(part)  # contiguous blocks: few interface nodes
    fmt = ss.SS_MAT_CSR if seed % 4 == 3 else ss.SS_MAT_SELL
    return A, P, part, fmt


@pytest.mark.parametrize("seed", range(30))
def test_random_apply_bitwise(seed):
    A, P, part, fmt = _case(seed)
    p = ss.ss_partition(A, ss.SS_PART_USER, P, user_part=part)
    s = ss.ss_cg_setup(A, p, ss.default_opts(matrix_format=fmt))
    sd = O.split(A.rowptr, A.colidx, part, P)
    rng = np.random.default_rng(seed)
    for x in (rng.standard_normal(A.n), rng.integers(-5, 6, A.n).astype(np.float64)):
        y = ss.ss_cg_apply(s, torch.tensor(x, device=DEV)).cpu().numpy()
        want = O.ss_spmv(A, sd, x)
        assert np.array_equal(y, want), (seed, A.n, P, fmt, float(np.max(np.abs(y - want))))
