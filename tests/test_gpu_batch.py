"""Batched CG (ss_batch_*) against the oracle's CG run pair by pair, against
one-by-one GPU solves, and for invariance under every launch shape the
autotuner may pick.

Each (system, right-hand side) pair is the oracle's plain CG on that system
(the same stopping rule and recomputed-residual restarts).  The SpMV row sums
are evaluated in the oracle's order (bitwise equal); the dot products are
fixed-order sums over 512-row granules, so they differ from the oracle's
sequential sums by rounding only."""
import numpy as np
import pytest

import oracle as O
import paper_2108_13162_amd as ss
from workloads import CSR, batch2d_lognormal, config, diffusion3d_lognormal, uniform_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _systems():
    # uneven sizes: 5x5 .. 45x45 grids, a 3D system and a 1 x 1 system
    S = batch2d_lognormal(6, 5, 45, seed=11)
    S.append(diffusion3d_lognormal(7, seed=12, sigma=0.5))
    S.append(CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([3.0])))
    S += batch2d_lognormal(3, 20, 33, seed=13)
    return S


def _rhs(systems, nrhs, seed):
    rng = np.random.default_rng(seed)
    return [rng.uniform(-1.0, 1.0, size=(A.n, nrhs)) for A in systems]


def _split(bt, flat):
    a = flat.reshape(bt.nrows, bt.nrhs)
    return [a[bt.offsets[s]:bt.offsets[s + 1]] for s in range(len(bt.sizes))]


def _solve(bt, blocks, tol=1e-10, maxit=100000, x0=None):
    b = _t(ss.pack_batch(blocks))
    x = torch.zeros_like(b) if x0 is None else _t(ss.pack_batch(x0))
    res, summ = ss.ss_batch_solve(bt, b, x, tol=tol, maxit=maxit)
    return _split(bt, x.cpu().numpy()), res, summ


@pytest.fixture(scope="module")
def small():
    S = _systems()
    bt = ss.ss_batch_setup(S, nrhs=4)
    B = _rhs(S, 4, 7)
    B[2][:, 1] = 0.0  # one zero right-hand side
    return S, bt, B


def test_pairs_match_oracle_cg(small):
    S, bt, B = small
    X, res, summ = _solve(bt, B)
    assert summ.status == ss.SS_OK
    for s, A in enumerate(S):
        for j in range(4):
            r = res[s * 4 + j]
            b = B[s][:, j]
            xo, ro = O.cg(A, b, tol=1e-10, maxit=100000, hist=False)
            x = X[s][:, j]
            assert r.status == ss.SS_OK
            if not b.any():
                assert r.iterations == 0 and not x.any()
                continue
            assert abs(r.iterations - ro.iterations) <= max(2, 0.05 * ro.iterations), (s, j, r, ro)
            true = np.linalg.norm(b - O.csr_matvec(A, x)) / np.linalg.norm(b)
            assert true <= 1e-10 and abs(r.relres - true) <= 1e-3 * true + 1e-16, (s, j, r.relres, true)
            xr = O.solve_reference(A, b)
            err = np.linalg.norm(x - xr) / np.linalg.norm(xr)
            err_o = np.linalg.norm(xo - xr) / np.linalg.norm(xr)
            assert err <= max(1e-9, 10 * err_o), (s, j, err, err_o)


@pytest.mark.parametrize("k", [1, 6])
def test_fixed_iterations_match_oracle(small, k):
    S, bt, B = small
    X, res, summ = _solve(bt, B, tol=0.0, maxit=k)
    for s, A in enumerate(S):
        for j in range(4):
            r = res[s * 4 + j]
            b = B[s][:, j]
            if not b.any():
                continue
            xo, ro = O.cg(A, b, tol=0.0, maxit=k, hist=False)
            if A.n == 1:  # exact after one step
                assert r.status in (ss.SS_OK, ss.SS_NOT_CONVERGED)
                assert np.allclose(X[s][:, j], xo, rtol=1e-15)
                continue
            assert r.iterations == ro.iterations == k and r.status == ss.SS_NOT_CONVERGED
            # only the dot summation order differs after k steps
            assert np.linalg.norm(X[s][:, j] - xo) <= 1e-12 * np.linalg.norm(xo), (s, j)


CH, PE, GR = ss.SS_BATCH_CHUNKED, ss.SS_BATCH_PERSISTENT, ss.SS_BATCH_GRAPH


def test_results_independent_of_launch_shape(small):
    # both schedules: chunked graphs and the single persistent launch (down to
    # 8 workgroups for all systems' phases), every tile size and unroll
    S, bt, B = small
    ref = None
    for shape in [(2, 0, 8, 32, CH), (1, 0, 4, 32, CH), (8, 0, 8, 2, CH), (1, 8, 5, 32, CH), (4, 1024, 4, 64, CH),
                  (2, 16, 5, 4, CH), (0, 0, 8, 32, CH), (0, 24, 5, 2, CH), (2, 0, 8, 32, PE), (1, 0, 4, 32, PE),
                  (8, 0, 5, 32, PE), (4, 8, 8, 32, PE), (1, 16, 4, 32, PE), (0, 0, 8, 32, PE)]:
        ss.ss_batch_set_tuning(bt, *shape)
        X, res, _ = _solve(bt, B)
        flat = np.concatenate([x.ravel() for x in X])
        its = [r.iterations for r in res]
        if ref is None:
            ref = (flat, its)
        else:
            assert np.array_equal(flat, ref[0]) and its == ref[1], shape
    ss.ss_batch_set_tuning(bt, 2, 0, 8, 32, CH)


def test_autotuner_picks_a_candidate_and_caches_it(small):
    S, bt, B = small
    b = _t(ss.pack_batch(B))
    chosen, trials = ss.ss_batch_tune(bt, b, iters=4, force=True)
    assert len(trials) == 60 and all(ms > 0 for _, ms in trials)
    assert sum(t["schedule"] == PE for t, _ in trials) == 15
    assert sum(t["tile_granules"] == 0 for t, _ in trials) == 12
    shapes = [t for t, _ in trials]
    assert chosen in shapes
    best = min(trials, key=lambda t: t[1])[0]
    assert chosen == best
    again, t2 = ss.ss_batch_tune(bt, b)
    assert again == chosen and t2 == []
    # a new batch of the same structure takes the cached choice at setup
    bt2 = ss.ss_batch_setup(S, nrhs=4)
    assert ss.ss_batch_get_tuning(bt2) == chosen
    X, res, summ = _solve(bt2, B)
    assert summ.status == ss.SS_OK


@pytest.mark.parametrize("nrhs", [1, 2])
def test_fewer_rhs(nrhs):
    S = batch2d_lognormal(4, 6, 30, seed=21)
    bt = ss.ss_batch_setup(S, nrhs=nrhs)
    B = _rhs(S, nrhs, 22)
    X, res, summ = _solve(bt, B)
    assert summ.status == ss.SS_OK
    for s, A in enumerate(S):
        for j in range(nrhs):
            xo, ro = O.cg(A, B[s][:, j], tol=1e-10, hist=False)
            # rounding-order differences shift CG's iteration count on these
            # ill-conditioned systems by a few percent
            assert abs(res[s * nrhs + j].iterations - ro.iterations) <= max(2, 0.05 * ro.iterations)
            xr = O.solve_reference(A, B[s][:, j])
            assert np.linalg.norm(X[s][:, j] - xr) <= 1e-9 * np.linalg.norm(xr)


@pytest.mark.parametrize("schedule", [0, 1, 2])  # SS_BATCH_CHUNKED, SS_BATCH_PERSISTENT, SS_BATCH_GRAPH
def test_initial_guess_and_edge_cases(small, schedule):
    S, bt, B = small
    ss.ss_batch_set_tuning(bt, 2, 0, 8, 32, schedule)
    # starting from the solution: converged after the first residual, 0 iterations
    X, res, _ = _solve(bt, B)
    X2, res2, summ = _solve(bt, B, x0=X)
    assert summ.status == ss.SS_OK and all(r.iterations == 0 for r in res2)
    # maxit = 0
    _, res3, summ3 = _solve(bt, B, maxit=0)
    assert summ3.status == ss.SS_NOT_CONVERGED
    assert all(r.iterations == 0 for r in res3)
    # a NaN in one right-hand side breaks that pair only
    Bn = [b.copy() for b in B]
    Bn[3][5, 2] = np.nan
    Xn, resn, summn = _solve(bt, Bn)
    assert summn.status == ss.SS_EBREAKDOWN
    for i, r in enumerate(resn):
        assert (r.status == ss.SS_EBREAKDOWN) == (i == 3 * 4 + 2), i
    assert np.array_equal(np.concatenate([x.ravel() for s, x in enumerate(Xn) if s != 3]),
                          np.concatenate([x.ravel() for s, x in enumerate(X) if s != 3]))
    # argument errors
    b = _t(ss.pack_batch(B))
    with pytest.raises(ss.SSError):
        ss.ss_batch_solve(bt, b, b)  # b and x overlap
    with pytest.raises(ss.SSError):
        ss.ss_batch_set_tuning(bt, 3, 0, 8, 32)
    with pytest.raises(ss.SSError):
        ss.ss_batch_set_tuning(bt, 2, 12, 8, 32)
    with pytest.raises(ss.SSError):
        ss.ss_batch_set_tuning(bt, 2, 0, 8, 32, 3)  # no such schedule
    with pytest.raises(ss.SSError):
        ss.ss_batch_setup(S, nrhs=3)
    ss.ss_batch_set_tuning(bt, 2, 0, 8, 32, CH)


@pytest.mark.parametrize("shape", [(2, 0, 8, 32), (1, 16, 5, 2), (0, 0, 4, 64)])
def test_whole_solve_graph(shape):
    # SS_BATCH_GRAPH: the first solve runs chunk by chunk and sets the graph's
    # length; the next solves are one graph launch each; a solve that needs
    # more chunks than the graph holds goes on chunk by chunk.  Every result
    # bitwise that of the chunked schedule.
    S = _systems()
    B = _rhs(S, 4, 31)
    bt_ch = ss.ss_batch_setup(S, nrhs=4)
    ss.ss_batch_set_tuning(bt_ch, *shape, CH)
    Xc, rc, _ = _solve(bt_ch, B)
    Xc_short, rc_short, _ = _solve(bt_ch, B, maxit=40)
    flat_c = np.concatenate([x.ravel() for x in Xc])
    its_c = [r.iterations for r in rc]
    bt = ss.ss_batch_setup(S, nrhs=4)
    ss.ss_batch_set_tuning(bt, *shape, GR)
    # a short first solve: the graph gets the chunks of 40 iterations
    Xs, rs, summ = _solve(bt, B, maxit=40)
    assert summ.status == ss.SS_NOT_CONVERGED
    assert bt.launches()["graphs"] == 0 and bt.launches()["chunks"] > 0
    assert np.array_equal(np.concatenate([x.ravel() for x in Xs]), np.concatenate([x.ravel() for x in Xc_short]))
    assert [r.iterations for r in rs] == [r.iterations for r in rc_short]
    # the full solve outgrows it: one graph launch, then chunk by chunk
    X1, r1, summ1 = _solve(bt, B)
    assert summ1.status == ss.SS_OK
    n1 = bt.launches()
    assert n1["graphs"] == 1 and n1["chunks"] > 0 and n1["kernels"] == 0
    assert np.array_equal(np.concatenate([x.ravel() for x in X1]), flat_c) and [r.iterations for r in r1] == its_c
    # the next solve sets the lengths again, chunk by chunk
    X2, r2, summ2 = _solve(bt, B)
    assert summ2.status == ss.SS_OK and bt.launches()["graphs"] == 0
    assert np.array_equal(np.concatenate([x.ravel() for x in X2]), flat_c) and [r.iterations for r in r2] == its_c
    # now the graph holds the whole solve, residual checks included: one launch
    for _ in range(2):
        X3, r3, summ3 = _solve(bt, B)
        n3 = bt.launches()
        assert summ3.status == ss.SS_OK and n3 == {"graphs": 1, "chunks": 0, "kernels": 0}
        assert np.array_equal(np.concatenate([x.ravel() for x in X3]), flat_c) and [r.iterations for r in r3] == its_c
    # other right-hand sides through the same graph (the checks read a copy)
    B2 = _rhs(S, 4, 32)
    Xc2, rc2, _ = _solve(bt_ch, B2)
    X4, r4, _ = _solve(bt, B2)
    assert np.array_equal(np.concatenate([x.ravel() for x in X4]), np.concatenate([x.ravel() for x in Xc2]))
    assert [r.iterations for r in r4] == [r.iterations for r in rc2]


@pytest.mark.parametrize("nrhs", [1, 2])
def test_whole_solve_graph_fewer_rhs_with_restarts(nrhs):
    # SS_BATCH_GRAPH with 1 and 2 right-hand sides, to a tolerance near the
    # attainable floor, so that residual checks restart pairs and the graph's
    # restart segment runs: bitwise the chunked schedule's results, iteration
    # and restart counts
    S = _systems()
    B = _rhs(S, nrhs, 41)
    tol = 1e-13
    bt_ch = ss.ss_batch_setup(S, nrhs=nrhs)
    ss.ss_batch_set_tuning(bt_ch, 2, 0, 8, 32, CH)
    Xc, rc, sc = _solve(bt_ch, B, tol=tol)
    flat_c = np.concatenate([x.ravel() for x in Xc])
    key_c = [(r.status, r.iterations, r.restarts) for r in rc]
    assert any(r.restarts > 0 for r in rc), key_c
    # the graph holds two rounds of chunks (before and after one restart);
    # a solve whose pairs restart again goes on chunk by chunk after it
    fits = max(r.restarts for r in rc) <= 1
    print(f"nrhs {nrhs}: {sum(r.restarts > 0 for r in rc)} pairs restarted, at most {max(r.restarts for r in rc)} times")
    bt = ss.ss_batch_setup(S, nrhs=nrhs)
    ss.ss_batch_set_tuning(bt, 2, 0, 8, 32, GR)
    for k in range(3):
        X, r, summ = _solve(bt, B, tol=tol)
        n = bt.launches()
        if k == 0:
            assert n["graphs"] == 0  # the first solve sets the lengths
        elif fits:
            assert n == {"graphs": 1, "chunks": 0, "kernels": 0}, n
        assert summ.status == sc.status
        assert np.array_equal(np.concatenate([x.ravel() for x in X]), flat_c)
        assert [(q.status, q.iterations, q.restarts) for q in r] == key_c


def test_matches_one_by_one_gpu_solves(small):
    S, bt, B = small
    X, res, _ = _solve(bt, B)
    for s in (0, 4, 6):
        A = S[s]
        part = ss.ss_partition(A, ss.SS_PART_USER, 1, user_part=np.zeros(A.n))
        sol = ss.ss_cg_setup(A, part)
        for j in range(4):
            x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
            r = ss.ss_cg_solve(sol, _t(B[s][:, j]), x, tol=1e-10, maxit=100000)
            assert abs(r.iterations - res[s * 4 + j].iterations) <= max(2, 0.05 * r.iterations)
            xs = x.cpu().numpy()
            assert np.linalg.norm(xs - X[s][:, j]) <= 1e-9 * max(np.linalg.norm(xs), 1e-300)


def test_full_size_batch_256_systems_4_rhs():
    # 256 lognormal 5-point systems on 32^2 .. 256^2 grids, 4 right-hand sides
    w = config(4)
    S, B = w.extra["systems"], w.extra["rhs"]
    bt = ss.ss_batch_setup(S, nrhs=4)
    b = _t(ss.pack_batch(B))
    x = torch.zeros_like(b)
    res, summ = ss.ss_batch_solve(bt, b, x, tol=1e-10, maxit=100000)
    assert summ.status == ss.SS_OK, summ
    X = _split(bt, x.cpu().numpy())
    worst = 0.0
    for s, A in enumerate(S):
        R = B[s] - np.stack([O.csr_matvec(A, X[s][:, j]) for j in range(4)], axis=1)
        rel = np.linalg.norm(R, axis=0) / np.linalg.norm(B[s], axis=0)
        worst = max(worst, rel.max())
    assert worst <= 1e-10, worst
    # smallest and largest systems against the oracle, pair by pair
    sizes = np.array([A.n for A in S])
    for s in (int(np.argmin(sizes)), int(np.argmax(sizes))):
        xo, ro = O.cg(S[s], B[s][:, 0], tol=1e-10, maxit=100000, hist=False)
        assert abs(res[s * 4].iterations - ro.iterations) <= max(2, 0.02 * ro.iterations)
        xr = O.solve_reference(S[s], B[s][:, 0])
        assert np.linalg.norm(X[s][:, 0] - xr) <= max(1e-9, 10 * np.linalg.norm(xo - xr) / np.linalg.norm(xr)) \
            * np.linalg.norm(xr)
    its = np.array([r.iterations for r in res])
    print(f"cfg4 batch: iterations {its.min()}..{its.max()}, worst true relres {worst:.2e}")


@pytest.mark.parametrize("nrhs", [4, 1])
def test_wide_systems_take_the_direct_gather_path(nrhs):
    # a 20^3 7-point system couples rows 400 apart, beyond the LDS window of
    # the staged SpMV for 4 right-hand sides (and a random SPD pattern far
    # beyond it for 1): those launches gather from memory; results must match
    # the oracle pair by pair all the same, next to small staged-size systems
    S = [diffusion3d_lognormal(20, seed=31, sigma=0.5)] + batch2d_lognormal(2, 8, 20, seed=32)
    if nrhs == 1:
        from workloads import random_spd_csr
        S.append(random_spd_csr(5000, 6.0, seed=33))
    bt = ss.ss_batch_setup(S, nrhs=nrhs)
    B = _rhs(S, nrhs, 34)
    X, res, summ = _solve(bt, B)
    assert summ.status == ss.SS_OK
    for s, A in enumerate(S):
        for j in range(nrhs):
            b = B[s][:, j]
            xo, ro = O.cg(A, b, tol=1e-10, hist=False)
            r = res[s * nrhs + j]
            assert abs(r.iterations - ro.iterations) <= max(2, 0.05 * ro.iterations), (s, j, r, ro)
            true = np.linalg.norm(b - O.csr_matvec(A, X[s][:, j])) / np.linalg.norm(b)
            assert true <= 1e-10
    # and the launch shape and schedule still change nothing
    for shape in [(1, 8, 4, 2, CH), (1, 8, 4, 2, PE)]:
        ss.ss_batch_set_tuning(bt, *shape)
        X2, res2, _ = _solve(bt, B)
        assert all(np.array_equal(a, c) for a, c in zip(X, X2)), shape
        assert [r.iterations for r in res] == [r.iterations for r in res2], shape


def test_many_small_systems():
    # 6000 systems of 1x1 .. 12x12 grids, 2 right-hand sides: 12,000 pairs, far
    # more tiles than workgroups, and systems leaving the running list at
    # every polled chunk (chunked, the default) or retiring one by one
    # (persistent); both schedules give the same bits
    S = batch2d_lognormal(6000, 1, 12, seed=41)
    bt = ss.ss_batch_setup(S, nrhs=2)
    B = _rhs(S, 2, 42)
    X, res, summ = _solve(bt, B, maxit=2000)
    assert summ.status == ss.SS_OK
    ss.ss_batch_set_tuning(bt, 2, 0, 8, 32, PE)
    Xc, resc, _ = _solve(bt, B, maxit=2000)
    assert all(np.array_equal(a, c) for a, c in zip(X, Xc))
    assert [r.iterations for r in res] == [r.iterations for r in resc]
    for s, A in enumerate(S):
        for j in range(2):
            r = res[s * 2 + j]
            b = B[s][:, j]
            xo, ro = O.cg(A, b, tol=1e-10, maxit=2000, hist=False)
            assert r.status == ss.SS_OK
            assert abs(r.iterations - ro.iterations) <= max(2, 0.05 * ro.iterations), (s, j, r, ro)
            x = X[s][:, j]
            true = np.linalg.norm(b - O.csr_matvec(A, x)) / np.linalg.norm(b)
            assert true <= 1e-10, (s, j, true)
            xr = O.solve_reference(A, b)
            err = np.linalg.norm(x - xr) / np.linalg.norm(xr)
            err_o = np.linalg.norm(xo - xr) / np.linalg.norm(xr)
            assert err <= max(1e-9, 10 * err_o), (s, j, err, err_o)
