#!/usr/bin/env python3
"""Time to relative residual 1e-10 of the sub-structured CG on one MI355X.

Workload (default): 3D 7-point variable-coefficient diffusion on a 128^3 grid
(2,097,152 unknowns, 14,581,760 stored entries), face coefficients
lognormal(0,1) from seed 2, right-hand side U[-1,1] from seed 102, split into
2 x 2 x 2 box sub-domains; plain (unpreconditioned) FP64 CG from x = 0 until
||b - A x|| <= 1e-10 ||b||.  Inputs are resident in HBM before timing starts.

One step = one complete solve (every CG iteration: local SpMV of all
sub-domains, interface assembly, dots and vector updates, plus the residual
recomputation at convergence).  Prints one JSON line.

The line also carries "variants", each timed on the same GPU after the main
measurement (time to relative residual 1e-10, inputs resident):
  mixed    -- Q1 hexahedral stiffness on 96^3 nodes (884,736 unknowns,
              23.4M entries), 16 weighted-RCB sub-domains: plain FP64 CG vs
              FP32 values/vectors with FP64 iterative refinement (restarted
              inner solves) and with FP64 residual replacement (reliable
              updates, search direction kept);
  batched  -- 256 lognormal 5-point systems on 32^2..256^2 grids, 4
              right-hand sides each: one batched solve (autotuned launch
              shape; also as one whole-solve graph launch and as one
              persistent launch) vs the 1024 (system, rhs) solves one by one;
  adjoint  -- 64^3 smoothed-GRF diffusion, 8 boxes: forward solve and
              forward + adjoint backward through torch.autograd;
  jacobi   -- the main line's system with the Jacobi preconditioner
              (Algorithm 3 with M = diag A) vs plain CG;
  splittings -- the main line's system cut three ways into 8 parts:
              sub-structuring (8 boxes, and 8 parts of the matrix graph
              without coordinates), band-row and band-column (8 bands), with
              the values each would exchange per product across devices.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--config 2]
                  [--variants mixed,batched,adjoint,jacobi,splittings | none]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to rel-res 1e-10 + SpMV HBM GB/s; mixed/batched vs plain FP64 CG"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = [os.path.join(ROOT, "paper_2108_13162_amd", "csrc", f)
              for f in ("kernels.hip", "kernels.h", "device_common.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "spmv_cg_step_traffic.json")


def kernel_sha() -> str:
    """SHA-256 prefix of the sources the single-system kernels are built from."""
    h = hashlib.sha256()
    for fn in KERNEL_SRC:
        with open(fn, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """Counter-measured HBM bytes per SpMV launch, if taken on this kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha() or t.get("workload") != workload:
        return None
    return float(t["hbm_bytes_per_launch"])


def calibrate_copy(torch, nbytes: int = 1 << 30, reps: int = 4) -> None:
    """Plain device copies of known size, for scaling the PMC byte counters."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"# copy calibration: {reps} copies of {nbytes} bytes", file=sys.stderr, flush=True)


def stream_copy_gbps(torch, nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Achievable HBM bandwidth: a plain device-to-device copy (read + write)."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def host_cpu() -> dict:
    """The host the CPU baseline ran on: CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count()
    return {"model": model, "cores_available": avail}


def cpu_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def cpu_baseline(w, sd, tol: float, iters_gpu: int) -> dict:
    """The oracle's sub-structured CG timed to the tolerance on the host: the
    sequential oracle as it stands (one thread), then its all-cores OpenMP
    build (the same CG with a static row partition and thread-ordered
    partial dots) on every core this process may use."""
    import oracle as O

    t0 = time.perf_counter()
    _, r1 = O.ss_cg(w.A, sd, w.b, tol=tol, maxit=100000, hist=False)
    t1 = time.perf_counter() - t0
    nt = cpu_threads()
    t0 = time.perf_counter()
    _, rn = O.ss_cg_omp(w.A, sd, w.b, tol=tol, maxit=100000, threads=nt)
    tn = time.perf_counter() - t0
    print(f"# cpu baseline: 1 thread {t1 * 1e3:.0f} ms ({r1.iterations} iterations), {nt} threads "
          f"{tn * 1e3:.0f} ms ({rn.iterations} iterations)", file=sys.stderr, flush=True)
    return {
        "value": round(t1 * 1e3, 3),
        "unit": "ms",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"the whole solve to relative residual {tol:g} on the bench system (measured, not scaled): "
                   f"sequential FP64 oracle, sub-structured CG, {r1.iterations} iterations "
                   f"({t1 * 1e3 / max(r1.iterations, 1):.2f} ms/iteration; GPU {iters_gpu} iterations)"),
        "status": r1.status,
        "iterations": r1.iterations,
        "true_relres": r1.true_relres,
        "all_cores": {"ms": round(tn * 1e3, 3), "threads": nt, "iterations": rn.iterations,
                      "status": rn.status, "ms_per_iteration": round(tn * 1e3 / max(rn.iterations, 1), 4),
                      "build": "OpenMP, static row partition, per-thread partial dots added in thread order"},
        "host": host_cpu(),
    }


def floor_solution(A, b):
    """The oracle's solution at its attainable floor (global CG to 1e-14 on
    all host cores), the reference of the error figures."""
    import oracle as O

    x, r = O.cg_omp(A, b, tol=1e-14, maxit=200000, threads=cpu_threads())
    return x, r


_REFS: dict = {}
_ORACLE_AT_TOL: dict = {}  # workload -> the oracle's own CG to the bench tolerance, its error vs the floor
_ERRORS = {"on": True, "tol": 1e-10}


def reference_for(w):
    """Floor solution of workload w (cached by name); None when error figures are off."""
    if not _ERRORS["on"]:
        return None
    if w.name not in _REFS:
        t0 = time.perf_counter()
        x, r = floor_solution(w.A, w.b)
        print(f"# oracle floor solution {w.name}: {r.iterations} iterations, true relres {r.true_relres:.1e} "
              f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
        _REFS[w.name] = x
        # the same oracle stopped at the bench tolerance: the error a correct
        # CG run to that residual has on this system
        import oracle as O

        xt, rt = O.cg_omp(w.A, w.b, tol=_ERRORS["tol"], maxit=200000, threads=cpu_threads())
        _ORACLE_AT_TOL[w.name] = {"error_vs_floor": rel_err(xt, x), "iterations": rt.iterations,
                                  "true_relres": rt.true_relres}
    return _REFS[w.name]


def error_vs_oracle(w, x_dev):
    ref = reference_for(w)
    return None if ref is None else rel_err(x_dev.cpu().numpy(), ref)


def rel_err(x, ref) -> float:
    import numpy as np

    return float(np.linalg.norm(np.asarray(x) - ref) / np.linalg.norm(ref))


def _timed(torch, fn, reps: int):
    """Milliseconds per call of fn (one untimed call first); fn's last result."""
    out = fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / max(reps, 1), out


def variant_mixed(ss, torch, reps: int, tol: float) -> dict:
    from workloads import config

    w = config(3)
    A = w.A
    part = ss.partition_workload(w)
    b = torch.tensor(w.b, dtype=torch.float64, device="cuda")
    bn = float(torch.linalg.norm(b))
    out, xs, s64 = {}, {}, None
    for name, prec in (("fp64", ss.SS_FP64), ("fp32_ir", ss.SS_FP32_IR), ("fp32_ru", ss.SS_FP32_RU)):
        s = ss.ss_cg_setup(A, part, ss.default_opts(precision=prec))
        x = torch.zeros_like(b)

        def run():
            x.zero_()
            return ss.ss_cg_solve(s, b, x, tol=tol, maxit=100000)

        ms, r = _timed(torch, run, reps)
        if s64 is None:
            s64 = s
        true = float(torch.linalg.norm(b - ss.ss_cg_apply(s64, x))) / bn
        sp_ms, sp_bytes = ss.ss_cg_time_spmv(s, 30)
        out[name] = {"ms": round(ms, 3), "status": r.status, "iterations": r.iterations,
                     "outer_iterations": r.outer_iterations, "true_relres": true,
                     "step_spmv_us": round(sp_ms * 1e3, 2),
                     "step_spmv_gbps": round(sp_bytes / (sp_ms * 1e-3) / 1e9, 1)}
        if prec == ss.SS_FP32_RU:
            out[name]["residual_replacements"] = out[name].pop("outer_iterations")
        xs[name] = x.clone()
        out[name]["error_vs_oracle"] = error_vs_oracle(w, x)
        print(f"# mixed/{name}: {ms:.3f} ms, {r.iterations} iterations ({r.outer_iterations} outer), "
              f"true relres {true:.2e}", file=sys.stderr, flush=True)
    for v in ("fp32_ir", "fp32_ru"):
        out[f"speedup_{v}_over_fp64"] = round(out["fp64"]["ms"] / out[v]["ms"], 3)
        out[f"{v}_vs_fp64_solution"] = float(torch.linalg.norm(xs[v] - xs["fp64"]) / torch.linalg.norm(xs["fp64"]))
    out["workload"] = w.name
    out["inner_tol"] = ss.default_opts().inner_tol
    out["ru_delta"] = ss.default_opts().ru_delta
    return out


def variant_batched(ss, torch, reps: int, tol: float, one_by_one: bool = True, whole_graph: bool = True) -> dict:
    import numpy as np

    from workloads import config

    w = config(4)
    S, B = w.extra["systems"], w.extra["rhs"]
    nrhs = B[0].shape[1]
    bt = ss.ss_batch_setup(S, nrhs=nrhs)
    b = torch.tensor(ss.pack_batch(B), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    chosen, trials = ss.ss_batch_tune(bt, b, iters=8, force=True)

    def run():
        x.zero_()
        return ss.ss_batch_solve(bt, b, x, tol=tol, maxit=100000)

    ms_b, (res, summ) = _timed(torch, run, reps)
    its = np.array([r.iterations for r in res])
    print(f"# batched: {ms_b:.3f} ms for {len(res)} pairs, iterations {its.min()}..{its.max()}, tuning {chosen}",
          file=sys.stderr, flush=True)
    out = {
        "workload": w.name, "pairs": len(res), "status": summ.status, "batched_ms": round(ms_b, 3),
        "iterations_min": int(its.min()), "iterations_max": int(its.max()),
        "max_relres": summ.relres, "tuning": chosen,
        "tuning_trials_ms_per_iteration": {"best": round(min(t[1] for t in trials), 5),
                                           "worst": round(max(t[1] for t in trials), 5), "count": len(trials)},
    }
    # algorithmic bytes: every iteration of a system while any of its pairs runs
    # reads the matrix once (12 B per entry + 1 B row length) and moves 9
    # vector values of 8 B per row and right-hand side (CG step: r, p, x read
    # once, p, q, x written; update: r, q read, r written)
    per_sys_its = its.reshape(len(S), nrhs).max(axis=1)
    nbytes = sum(int(k) * (12 * A.nnz + A.n + 72 * nrhs * A.n) for k, A in zip(per_sys_its, S))
    out["algorithmic_bytes"] = nbytes
    out["effective_gbps"] = round(nbytes / (ms_b * 1e-3) / 1e9, 1)
    if _ERRORS["on"]:
        # error against the oracle's floor solution for a sample of pairs: the
        # smallest and the largest system, and six seeded random ones
        import oracle as O

        sizes = np.array([A.n for A in S])
        pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)),
                       *np.random.default_rng(4).choice(len(S), 6, replace=False).tolist()})
        xh = x.cpu().numpy()
        offs = np.concatenate([[0], np.cumsum(sizes)])
        errs = []
        for si in pick:
            j = si % nrhs
            xr, _ = O.cg_omp(S[si], np.ascontiguousarray(B[si][:, j]), tol=1e-14, maxit=200000,
                             threads=cpu_threads())
            errs.append(rel_err(xh[offs[si] * nrhs + j: offs[si + 1] * nrhs: nrhs], xr))
        out["error_vs_oracle_sampled"] = {"max": max(errs), "pairs": [[int(si), int(si % nrhs)] for si in pick]}
    # the same solve with every iteration in one launch (persistent schedule,
    # the tuned tiles): same bits, timed for comparison
    x_tuned = x.clone()
    ss.ss_batch_set_tuning(bt, chosen["tile_granules"], 0, chosen["unroll"], chosen["check_every"],
                           ss.SS_BATCH_PERSISTENT)
    ms_p, (res_p, _) = _timed(torch, run, 1)
    out["persistent_one_launch_ms"] = round(ms_p, 3)
    out["persistent_bitwise_equal"] = bool(torch.equal(x, x_tuned)) and \
        [r.iterations for r in res_p] == [r.iterations for r in res]
    print(f"# batched, one persistent launch: {ms_p:.3f} ms, bitwise equal {out['persistent_bitwise_equal']}",
          file=sys.stderr, flush=True)
    if whole_graph:
        # the tuned chunked launches captured as one graph of the whole solve
        # (SS_BATCH_GRAPH): the first solve sets the graph's length, the second
        # builds it, the timed ones are one graph launch each
        ss.ss_batch_set_tuning(bt, chosen["tile_granules"], chosen["grid"], chosen["unroll"], chosen["check_every"],
                               ss.SS_BATCH_GRAPH)
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        out["graph_build_and_solve_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
        t0 = time.perf_counter()
        for _ in range(max(reps, 1)):
            res_g, _ = run()
        torch.cuda.synchronize()
        ms_g = (time.perf_counter() - t0) * 1e3 / max(reps, 1)
        out["graph_one_launch_ms"] = round(ms_g, 3)
        out["graph_launches_per_solve"] = bt.launches()
        out["graph_bitwise_equal"] = bool(torch.equal(x, x_tuned)) and \
            [r.iterations for r in res_g] == [r.iterations for r in res]
        print(f"# batched, one graph launch: {ms_g:.3f} ms (first, with the capture: "
              f"{out['graph_build_and_solve_ms']:.3f} ms), launches {out['graph_launches_per_solve']}, "
              f"bitwise equal {out['graph_bitwise_equal']}", file=sys.stderr, flush=True)
    ss.ss_batch_set_tuning(bt, **chosen)
    if not one_by_one:
        return out
    # one by one: one solver per system (set up outside the timing), every pair solved separately
    solvers = [ss.ss_cg_setup(A, ss.ss_partition(A, ss.SS_PART_USER, 1, user_part=np.zeros(A.n))) for A in S]
    cols = [[torch.tensor(np.ascontiguousarray(Bs[:, j]), device="cuda") for j in range(nrhs)] for Bs in B]
    xs = [torch.zeros(A.n, dtype=torch.float64, device="cuda") for A in S]
    worst = [ss.SS_OK]

    def run_single():
        for s, sol in enumerate(solvers):
            for j in range(nrhs):
                xs[s].zero_()
                r = ss.ss_cg_solve(sol, cols[s][j], xs[s], tol=tol, maxit=100000)
                worst[0] = min(worst[0], r.status) if r.status < 0 else max(worst[0], r.status)

    ms_1, _ = _timed(torch, run_single, 1)
    print(f"# one by one: {ms_1:.3f} ms", file=sys.stderr, flush=True)
    out.update({"status_one_by_one": worst[0], "one_by_one_ms": round(ms_1, 3),
                "speedup_batched_over_one_by_one": round(ms_1 / ms_b, 3)})
    return out


def variant_jacobi(ss, torch, reps: int, tol: float) -> dict:
    """Jacobi-preconditioned CG (Algorithm 3 with M = diag A) vs plain CG on
    the 128^3 lognormal system of the main line."""
    from workloads import config

    w = config(2)
    part = ss.partition_workload(w)
    b = torch.tensor(w.b, dtype=torch.float64, device="cuda")
    out = {"workload": w.name}
    for name, pc in (("cg", ss.SS_PRECOND_NONE), ("pcg_jacobi", ss.SS_PRECOND_JACOBI)):
        s = ss.ss_cg_setup(w.A, part, ss.default_opts(precond=pc))
        x = torch.zeros_like(b)

        def run():
            x.zero_()
            return ss.ss_cg_solve(s, b, x, tol=tol, maxit=100000)

        ms, r = _timed(torch, run, reps)
        out[name] = {"ms": round(ms, 3), "status": r.status, "iterations": r.iterations, "relres": r.relres,
                     "ms_per_iteration": round(ms / max(r.iterations, 1), 5),
                     "error_vs_oracle": error_vs_oracle(w, x)}
        print(f"# jacobi/{name}: {ms:.3f} ms, {r.iterations} iterations", file=sys.stderr, flush=True)
        del s
    out["speedup_pcg_over_cg"] = round(out["cg"]["ms"] / out["pcg_jacobi"]["ms"], 3)
    return out


def exchange_volumes(ss, A, part, nbands: int) -> dict:
    """Values one CG product would move between parts if every part sat on its
    own device (the least each scheme needs), per splitting of A:
    sub-structuring: every copy of an interface node sends its partial sum to
    the other holders; band-row: every band receives the x entries its rows
    reference outside the band; band-column: every band sends the partial y
    entries of rows outside the band."""
    import numpy as np

    n = A.n
    m = n // nbands
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.rowptr))
    cols = A.colidx.astype(np.int64)
    brow = np.minimum(rows // m, nbands - 1)
    bcol = np.minimum(cols // m, nbands - 1)
    off = brow != bcol
    row_x = np.unique(brow[off] * n + cols[off]).size   # (band, x entry) pairs
    col_y = np.unique(bcol[off] * n + rows[off]).size   # (band, y entry) pairs
    e = ss.ss_part_export(part)
    mult = np.diff(e["copy_ptr"]).astype(np.int64)
    return {"sub_structuring": int(np.sum(mult * (mult - 1))), "band_row": int(row_x), "band_col": int(col_y),
            "band_row_allgather": int((nbands - 1) * n), "band_col_allreduce": int(nbands * n)}


def variant_splittings(ss, torch, reps: int, tol: float) -> dict:
    """The paper's three decompositions of the same system into 8 parts
    (Sections 3.1, 3.2, 3.4), all parts on this device: sub-structuring (the
    8 boxes of the main line), band-row and band-column (8 bands): time to the
    tolerance, the CG-step product's bandwidth, and the values each would
    exchange per product across devices."""
    from workloads import config

    import numpy as np

    w = config(2)
    part = ss.partition_workload(w)
    t0 = time.perf_counter()
    gpart = ss.ss_partition(w.A, ss.SS_PART_GRAPH, 8)   # no coordinates: the adjacency graph only
    graph_s = time.perf_counter() - t0
    b = torch.tensor(w.b, dtype=torch.float64, device="cuda")
    out = {"workload": w.name, "parts": 8}
    makers = (("sub_structuring", lambda: ss.ss_cg_setup(w.A, part)),
              ("sub_structuring_graph", lambda: ss.ss_cg_setup(w.A, gpart)),
              ("band_row", lambda: ss.ss_band_setup(w.A, ss.SS_BAND_ROW, 8)),
              ("band_col", lambda: ss.ss_band_setup(w.A, ss.SS_BAND_COL, 8)))
    for name, make in makers:
        s = make()
        x = torch.zeros_like(b)

        def run():
            x.zero_()
            return ss.ss_cg_solve(s, b, x, tol=tol, maxit=100000)

        ms, r = _timed(torch, run, reps)
        spmv_ms, spmv_bytes = ss.ss_cg_time_spmv(s, 50)
        out[name] = {"ms": round(ms, 3), "status": r.status, "iterations": r.iterations,
                     "true_relres": r.true_relres, "ms_per_iteration": round(ms / max(r.iterations, 1), 5),
                     "step_spmv_us": round(spmv_ms * 1e3, 2),
                     "step_spmv_gbps": round(spmv_bytes / (spmv_ms * 1e-3) / 1e9, 1),
                     "error_vs_oracle": error_vs_oracle(w, x)}
        print(f"# splittings/{name}: {ms:.3f} ms, {r.iterations} iterations", file=sys.stderr, flush=True)
        del s
    out["exchange_values_per_product"] = exchange_volumes(ss, w.A, part, 8)
    mult = np.diff(ss.ss_part_export(gpart)["copy_ptr"]).astype(np.int64)
    out["exchange_values_per_product"]["sub_structuring_graph"] = int(np.sum(mult * (mult - 1)))
    out["graph_partition"] = {"host_seconds": round(graph_s, 3), **{k: v for k, v in ss.ss_part_sizes(gpart).items()
                                                                   if k in ("n_loc", "n_gamma", "n_copies")}}
    return out


def variant_adjoint(ss, torch, reps: int, tol: float) -> dict:
    from workloads import config

    w = config(5)
    solver = ss.ss_cg_setup(w.A, ss.partition_workload(w))
    xt = torch.tensor(w.extra["x_target"], dtype=torch.float64, device="cuda")
    v0 = torch.tensor(w.A.val, dtype=torch.float64, device="cuda")
    b0 = torch.tensor(w.b, dtype=torch.float64, device="cuda")

    def fwd():
        with torch.no_grad():
            return ss.sscg_solve(v0, b0, solver, tol=tol)

    def fwd_bwd():
        vals = v0.clone().requires_grad_(True)
        b = b0.clone().requires_grad_(True)
        x = ss.sscg_solve(vals, b, solver, tol=tol, adj_tol=tol)
        loss = 0.5 * torch.sum((x - xt) ** 2)
        loss.backward()
        return vals.grad

    ms_f, xf = _timed(torch, fwd, reps)
    ms_fb, _ = _timed(torch, fwd_bwd, reps)
    print(f"# adjoint: forward {ms_f:.3f} ms, forward+backward {ms_fb:.3f} ms", file=sys.stderr, flush=True)
    return {"workload": w.name, "forward_ms": round(ms_f, 3), "forward_backward_ms": round(ms_fb, 3),
            "backward_over_forward": round((ms_fb - ms_f) / ms_f, 3),
            "forward_error_vs_oracle": error_vs_oracle(w, xf)}


def _solve_line(ss, torch, w, reps: int, tol: float, opts=None) -> dict:
    """Time to tol of one workload (inputs resident), with its iteration
    count, time per iteration, the kernels an iteration launches and the
    error against the oracle's floor solution."""
    A = w.A
    part = ss.partition_workload(w)
    s = ss.ss_cg_setup(A, part, opts)
    b = torch.tensor(w.b, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)

    def run():
        x.zero_()
        return ss.ss_cg_solve(s, b, x, tol=tol, maxit=100000)

    ms, r = _timed(torch, run, reps)
    bn = float(torch.linalg.norm(b))
    true = float(torch.linalg.norm(b - ss.ss_cg_apply(s, x))) / bn
    longest = int(np.max(np.diff(A.rowptr))) if A.n else 0
    info = s.info()
    out = {"workload": w.name, "n": int(A.n), "nnz": int(A.nnz), "n_loc": int(info["n_loc"]),
           "ms": round(ms, 3), "status": r.status, "iterations": r.iterations, "true_relres": true,
           "us_per_iteration": round(ms * 1e3 / max(r.iterations, 1), 2)}
    if s.path() == ss.SS_PATH_SMALL:
        out["path"] = "one launch per solve (one workgroup runs every iteration)"
        out["kernel_launches_per_solve"] = 4   # gather b, gather x, the solve, scatter x
    else:
        out["path"] = "streaming kernels, graph chunks of 32 iterations"
        out["kernels_per_iteration"] = (2 if (info["matrix_format"] == ss.SS_MAT_SELL and longest <= 9) else
                                        (3 if info["matrix_format"] == ss.SS_MAT_SELL else 2))
    out["error_vs_oracle"] = error_vs_oracle(w, x)
    print(f"# {w.name}: {ms:.3f} ms, {r.iterations} iterations, {out['us_per_iteration']} us/iteration",
          file=sys.stderr, flush=True)
    del s
    return out


def variant_configs(ss, torch, reps: int, tol: float) -> dict:
    """Time to tol of the two workloads not timed elsewhere: the 64 x 64
    Poisson system in 2 x 2 boxes (latency bound: 4096 unknowns) and the 64^3
    smoothed-GRF diffusion in 2 x 2 x 2 boxes."""
    from workloads import config

    w1 = config(1)
    # ~1-3 ms solves: enough of them that the device clocks have settled
    return {"poisson2d_64": _solve_line(ss, torch, w1, max(reps, 50), tol),
            "poisson2d_64_streaming": _solve_line(ss, torch, w1, max(reps, 50), tol,
                                                  ss.default_opts(small_solver=ss.SS_SMALL_OFF)),
            "diffusion3d_grf_64": _solve_line(ss, torch, config(5), reps, tol)}


def variant_beyond_mall(ss, torch, reps: int, tol: float) -> dict:
    """The main line's recipe on a 192^3 grid (7.2M unknowns, 51.4M stored
    entries, a ~900 MB working set: several times the 256 MB last-level
    cache), so that the CG step streams from HBM: time to tol and the CG-step
    roofline point."""
    from workloads import config

    w = config(2, size=192)
    A = w.A
    s = ss.ss_cg_setup(A, ss.partition_workload(w))
    b = torch.tensor(w.b, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)

    def run():
        x.zero_()
        return ss.ss_cg_solve(s, b, x, tol=tol, maxit=100000)

    ms, r = _timed(torch, run, reps)
    true = float(torch.linalg.norm(b - ss.ss_cg_apply(s, x))) / float(torch.linalg.norm(b))
    spmv_ms, spmv_bytes = ss.ss_cg_time_spmv(s, 20)
    n_loc = s.info()["n_loc"]
    spmv_only = 12.0 * A.nnz + 20.0 * n_loc
    st_ms, st_bytes = ss.ss_stream_rate(n_loc, 7, 20)
    ceil_gbps = st_bytes / (st_ms * 1e-3) / 1e9
    out = {"workload": w.name, "n": int(A.n), "nnz": int(A.nnz), "n_loc": int(n_loc), "ms": round(ms, 3),
           "status": r.status, "iterations": r.iterations, "true_relres": true,
           "us_per_iteration": round(ms * 1e3 / max(r.iterations, 1), 2),
           "step_spmv_us": round(spmv_ms * 1e3, 2), "step_algorithmic_bytes": int(spmv_bytes),
           "step_gbps": round(spmv_bytes / (spmv_ms * 1e-3) / 1e9, 1),
           "frac": round(spmv_bytes / (spmv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "frac_spmv_only": round(spmv_only / (spmv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "stream_ceiling_gbps": round(ceil_gbps, 1),
           "stream_ceiling_frac": round(ceil_gbps / HBM_PEAK_GBS, 4),
           "step_frac_of_ceiling": round(spmv_bytes / (spmv_ms * 1e-3) / 1e9 / ceil_gbps, 4)}
    print(f"# beyond MALL {w.name}: {ms:.3f} ms, {r.iterations} iterations, step {spmv_ms * 1e3:.1f} us "
          f"({out['frac']:.3f} of 8 TB/s)", file=sys.stderr, flush=True)
    del s
    return out


def main_measurement(args, ss, torch, config):
    """The main line: time to 1e-10 of FP64 sub-structured CG on the chosen workload."""
    w = config(args.config)
    A = w.A
    # setup is timed on its own, outside the solve (a pre-processing step)
    t0 = time.perf_counter()
    part = ss.partition_workload(w)
    t1 = time.perf_counter()
    solver = ss.ss_cg_setup(A, part)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    setup_ms = {"partition": round((t1 - t0) * 1e3, 1), "cg_setup": round((t2 - t1) * 1e3, 1)}
    info = solver.info()
    b = torch.tensor(w.b, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    print(f"# {w.name}: n={A.n} nnz={A.nnz} n_loc={info['n_loc']} format={info['matrix_format']} stored={info['stored']}", file=sys.stderr,
          flush=True)

    for i in range(args.warmup):
        x.zero_()
        r = ss.ss_cg_solve(solver, b, x, tol=args.tol, maxit=100000)
        print(f"# warmup {i}: {r.iterations} iterations, relres {r.relres:.3e}", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results, marks = [], [t0]
    for _ in range(args.steps):
        x.zero_()
        results.append(ss.ss_cg_solve(solver, b, x, tol=args.tol, maxit=100000))
        marks.append(time.perf_counter())  # the solve returns once it is complete
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed * 1e3 / max(args.steps, 1)
    per_step = sorted((b_ - a_) * 1e3 for a_, b_ in zip(marks, marks[1:]))
    ms_median = per_step[len(per_step) // 2] if per_step else ms_step
    r = results[-1] if results else ss.ss_cg_solve(solver, b, x, tol=args.tol, maxit=100000)
    x_solved = x.clone()
    if any(q.status != ss.SS_OK for q in results):
        print(f"bench.py: solve did not converge: {[q.status for q in results]}", file=sys.stderr)
        return None
    print(f"# timed: {args.steps} solves, {ms_step:.3f} ms each, {r.iterations} iterations", file=sys.stderr,
          flush=True)

    # one more solve with b handed over from pinned host memory and x copied
    # back to it: the host-inclusive time, reported beside the value (which
    # starts with the inputs resident in HBM), never as it
    bh = torch.tensor(w.b, dtype=torch.float64).pin_memory()
    xh = torch.empty_like(bh).pin_memory()
    torch.cuda.synchronize()
    th = time.perf_counter()
    b.copy_(bh)
    x.zero_()
    rh = ss.ss_cg_solve(solver, b, x, tol=args.tol, maxit=100000)
    xh.copy_(x)
    torch.cuda.synchronize()
    host_ms = (time.perf_counter() - th) * 1e3
    if rh.status != ss.SS_OK:
        print(f"bench.py: host-inclusive solve did not converge: {rh.status}", file=sys.stderr)
        return None

    # dominant kernel: the CG-step SpMV (p-update + local SpMV + (p, A p) partials)
    spmv_ms, spmv_bytes = ss.ss_cg_time_spmv(solver, 50)
    achieved = spmv_bytes / (spmv_ms * 1e-3) / 1e9
    traffic = load_traffic(w.name)
    n_loc = info["n_loc"]
    # the SpMV-only count: 8 B value + 4 B column per stored entry, 4 B row
    # pointer per row, x read and y written (8 B each) per row
    spmv_only = 12.0 * A.nnz + 4.0 * n_loc + 16.0 * n_loc
    iter_bytes = spmv_bytes + 24.0 * n_loc  # + update kernel: r, q read; r written
    ms_iter = ms_step / max(r.iterations, 1)

    out = {
        "metric": METRIC,
        "value": round(ms_step, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "ms_median": round(ms_median, 3),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "n": int(A.n), "nnz": int(A.nnz), "subdomains": int(w.nparts), "n_loc": int(n_loc),
            "method": "sub-structured CG, M=I, x0=0", "tol": args.tol,
        },
        "iterations": int(r.iterations),
        "relres": r.relres,
        "setup_ms": setup_ms,
        "host_inclusive_ms": {"ms": round(host_ms, 3), "what": "b from pinned host memory, solve, x back to pinned host memory (one run)"},
        "ms_per_iteration": round(ms_iter, 5),
        "iteration_bytes": int(iter_bytes),
        "iteration_gbps": round(iter_bytes / (ms_iter * 1e-3) / 1e9, 1),
        "roofline": {
            "bound": "hbm",
            "kernel": "k_spmv_sell (CG step)" if info["matrix_format"] == ss.SS_MAT_SELL else "k_spmv_csr (CG step)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            # the counter-measured bytes over the same launch time: what the
            # kernel streams (algorithmic bytes shrink with the column encoding)
            "traffic_gbps": round(traffic / (spmv_ms * 1e-3) / 1e9, 1) if traffic else None,
            "launch_ms": round(spmv_ms, 5),
            "algorithmic_bytes": int(spmv_bytes),
            "traffic_what": ("L2-miss bytes (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), served by the "
                             "last-level cache (MALL) or HBM: at this size most of the working set fits the "
                             "256 MB MALL"),
            "frac_spmv_only": round(spmv_only / (spmv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "spmv_only_bytes": int(spmv_only),
            "spmv_only_what": "12 B per stored entry + 4 B row pointer + 16 B (x read, y written) per row",
            "stream_copy_gbps": round(stream_copy_gbps(torch), 1),
        },
    }
    # the same bytes per row streamed without the step's gathers: the ceiling
    # the step is held to on this device
    st_ms, st_bytes = ss.ss_stream_rate(n_loc, 7, 20)
    out["roofline"]["stream_ceiling"] = {
        "gbps": round(st_bytes / (st_ms * 1e-3) / 1e9, 1), "rows": int(n_loc), "slots": 7,
        "what": "gather-free stream of the CG step's pattern (7 values + 3 vector reads + 3 vector writes per row)",
        "step_frac_of_ceiling": round(achieved / (st_bytes / (st_ms * 1e-3) / 1e9), 4)}
    if not args.no_cpu_baseline:
        import oracle as O

        sd = O.split(A.rowptr, A.colidx, O.partition_workload(w), w.nparts)
        out["cpu_baseline"] = cpu_baseline(w, sd, args.tol, r.iterations)
        del sd
        out["error_vs_oracle"] = error_vs_oracle(w, x_solved)
        out["error_what"] = ("||x - x_ref|| / ||x_ref||, x_ref = the oracle's global CG run to 1e-14 "
                             "(its attainable floor) on all host cores")
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 5])
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle legs (timed solves and the floor solutions of the error figures)")
    ap.add_argument("--variants", default="configs,beyond_mall,mixed,batched,adjoint,jacobi,splittings",
                    help="comma list of configs, beyond_mall, mixed, batched, adjoint, jacobi, splittings; "
                         "'none' to skip")
    ap.add_argument("--variant-steps", type=int, default=3)
    ap.add_argument("--no-main", action="store_true",
                    help="profiling aid: skip the main measurement, print only the variants")
    ap.add_argument("--no-one-by-one", action="store_true",
                    help="profiling aid: skip the one-by-one half of the batched comparison")
    ap.add_argument("--no-whole-solve-graph", action="store_true",
                    help="profiling aid: skip the whole-solve graph half of the batched comparison "
                         "(its kernels are the chunked launches')")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run plain 1 GiB device copies first (reference for PMC byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the solver runs on one GPU (all sub-domains resident on one MI355X); "
              f"--gpus {args.gpus} / WORLD_SIZE {world} is not supported", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2108_13162_amd as ss
    from workloads import config

    _ERRORS["on"] = not args.no_cpu_baseline
    _ERRORS["tol"] = args.tol
    if args.copy_calibration:
        calibrate_copy(torch)
    out = {} if args.no_main else main_measurement(args, ss, torch, config)
    if out is None:
        return 1
    chosen = [v for v in args.variants.split(",") if v and v != "none"]
    funcs = {"mixed": variant_mixed, "batched": variant_batched, "adjoint": variant_adjoint, "jacobi": variant_jacobi,
             "splittings": variant_splittings, "configs": variant_configs, "beyond_mall": variant_beyond_mall}
    if chosen:
        out["variants"] = {}
        for v in chosen:
            kw = {"one_by_one": not args.no_one_by_one,
                  "whole_graph": not args.no_whole_solve_graph} if v == "batched" else {}
            out["variants"][v] = funcs[v](ss, torch, args.variant_steps, args.tol, **kw)
            torch.cuda.empty_cache()
    if _ORACLE_AT_TOL:
        out["oracle_cg_at_tol"] = {"what": "the oracle's global CG (all host cores) stopped at the same relative "
                                           "residual: its error against the floor solution, per workload",
                                   **_ORACLE_AT_TOL}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
