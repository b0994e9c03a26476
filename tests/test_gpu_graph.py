"""Sub-structured CG on SS_PART_GRAPH partitions (no coordinates), against
the oracle's sub-structured CG on the same partition, through the C-ABI."""
import numpy as np
import pytest

import oracle as O
import paper_2108_13162_amd as ss
from workloads import config, random_spd_csr, uniform_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _cases():
    w1, w3 = config(1), config(3, size=16)
    R = random_spd_csr(5000, 7.0, seed=8)
    return [("poisson64_graph4", w1.A, w1.b, 4), ("q1hex16_graph8", w3.A, w3.b, 8),
            ("random5000_graph6", R, uniform_rhs(R.n, 5), 6)]


@pytest.mark.parametrize("case", range(3))
def test_apply_and_solve_on_graph_partition(case):
    name, A, b, k = _cases()[case]
    p = ss.ss_partition(A, ss.SS_PART_GRAPH, k)
    part = ss.ss_part_export(p)["part"]
    sd = O.split(A.rowptr, A.colidx, part, k)
    s = ss.ss_cg_setup(A, p)
    # the sub-structured product: bitwise the oracle's
    x = np.random.default_rng(case).standard_normal(A.n)
    assert np.array_equal(ss.ss_cg_apply(s, _t(x)).cpu().numpy(), O.ss_spmv(A, sd, x)), name
    # solve to 1e-10
    xg = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    r = ss.ss_cg_solve(s, _t(b), xg, tol=1e-10, maxit=20000)
    xo, ro = O.ss_cg(A, sd, b, tol=1e-10, maxit=20000)
    assert r.status == ss.SS_OK and ro.status == O.OK, name
    assert abs(r.iterations - ro.iterations) <= 2, (name, r.iterations, ro.iterations)
    assert r.true_relres <= 1e-10
    xs = O.solve_reference(A, b)
    err, erro = (np.linalg.norm(v - xs) / np.linalg.norm(xs) for v in (xg.cpu().numpy(), xo))
    assert err <= max(1e-9, 2 * erro), (name, err, erro)
