"""Writes tests/golden/fullsize_spread.json: the oracle's CG iteration
counts to 1e-10 on the full-size workloads, for two families of dot-product
evaluation.

CG in floating point on an ill-conditioned system is sensitive to the
rounding of its dot products.  Long sequential sums (the plain oracle adds two
million terms left to right) carry errors that cost iterations; tree or
blocked sums, as on a GPU or on several threads, carry far less.  The
reference count is therefore that of the oracle with accurately evaluated dot
products (Dot2, as accurate as twice the working precision): the sub-structured
CG and the CG on the unsplit matrix, whose difference is the spread the GPU
tests allow (at least 2).  The counts of the plain sequential oracle and of its
all-cores build at several thread counts are recorded beside them: they show
how much the summation order alone moves the count.  Calls only oracle/ and the
seeded generators.  Run from the repository root:

    python tests/golden/make_fullsize_spread.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from workloads import config  # noqa: E402

THREADS = (2, 3, 4, 6, 8)


def spread(idx):
    w = config(idx)
    sd = O.split(w.A.rowptr, w.A.colidx, O.partition_workload(w), w.nparts)
    acc = {}
    _, r = O.ss_cg_dot2(w.A, sd, w.b, tol=1e-10, maxit=100000, hist=False)
    acc["ss_cg_dot2"] = r.iterations
    _, r = O.cg_dot2(w.A, w.b, tol=1e-10, maxit=100000, hist=False)
    acc["cg_dot2"] = r.iterations
    seq = {}
    _, rs = O.ss_cg(w.A, sd, w.b, tol=1e-10, maxit=100000, hist=False)
    seq["ss_cg"] = rs.iterations
    _, rg = O.cg(w.A, w.b, tol=1e-10, maxit=100000, hist=False)
    seq["cg_global"] = rg.iterations
    for th in THREADS:
        _, r = O.ss_cg_omp(w.A, sd, w.b, tol=1e-10, maxit=100000, threads=th)
        seq[f"ss_cg_omp_{th}"] = r.iterations
    out = {"workload": w.name, "reference": acc["ss_cg_dot2"], "accurate_dots": acc,
           "spread": max(acc.values()) - min(acc.values()), "sequential_dots": seq,
           "sequential_spread": max(seq.values()) - min(seq.values())}
    print(json.dumps(out), flush=True)
    return out


def main():
    res = {str(i): spread(i) for i in (2, 3, 5)}
    with open(os.path.join(ROOT, "tests", "golden", "fullsize_spread.json"), "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
