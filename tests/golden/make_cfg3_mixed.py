"""Writes tests/golden/cfg3_mixed_counts.json: the oracle's mixed-precision
solves of the 96^3 Q1-hexahedral system (16 weighted-RCB parts) to 1e-10,
for the GPU tests' iteration checks:

  - FP32 CG with FP64 residual replacement (orc_ss_ru, ru_delta 0.1, the
    replacement test every 32 iterations as the device polls it): inner
    iterations and replacements;
  - FP32 inner CG inside FP64 iterative refinement (orc_ss_ir, inner
    tolerance 1e-6): inner iterations and outer corrections.

The FP32 products are rounded exactly as the device rounds them; the FP64
dot products are summed in another order, so the device's counts may differ
by a few iterations.  Calls only oracle/ and the seeded generators.  Run from
the repository root:

    python tests/golden/make_cfg3_mixed.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from workloads import config  # noqa: E402


def main():
    w = config(3)
    sd = O.split(w.A.rowptr, w.A.colidx, O.partition_workload(w), w.nparts)
    out = {"workload": w.name}
    t0 = time.perf_counter()
    _, r = O.ss_ru(w.A, sd, w.b, tol=1e-10, maxit=100000, delta=0.1, check_every=32)
    out["ru"] = {"status": r.status, "iterations": r.iterations, "replacements": r.outer, "true_relres": r.true_relres}
    print("ru", out["ru"], f"{time.perf_counter() - t0:.0f} s", flush=True)
    t0 = time.perf_counter()
    _, r = O.ss_ir(w.A, sd, w.b, tol=1e-10, maxit=100000, inner_tol=1e-6, max_outer=50)
    out["ir"] = {"status": r.status, "iterations": r.iterations, "outer": r.outer, "true_relres": r.true_relres}
    print("ir", out["ir"], f"{time.perf_counter() - t0:.0f} s", flush=True)
    with open(os.path.join(ROOT, "tests", "golden", "cfg3_mixed_counts.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
