"""Write q1hex128_oracle.json: the FP64 oracle's solves of the 128^3 Q1-hex
system (seed 0, tol 1e-10, x0 = 0) in both forms of the iteration.

The GPU parity test at this size compares against these stored values
because the oracle needs minutes per solve here.  Everything stored comes
from `oracle/` alone:

    python tests/golden/make_q1hex128.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

N_SAMPLES = 1024


def main():
    a, b = W.problem(128, 0)
    rows = np.sort(np.random.default_rng(128).choice(a.n, N_SAMPLES, replace=False))
    out = {"workload": "q1hex 128^3 sigma+mass, seed 0, tol 1e-10, x0 = 0, Jacobi",
           "n": int(a.n), "nnz": int(a.rowptr[-1]), "rows": rows.tolist(), "forms": {}}
    for form in ("standard", "single"):
        x, info = oracle.pcg(a, b, tol=1e-10, form=form)
        out["forms"][form] = {"iters": int(info["iters"]), "status": int(info["status"]),
                              "replacements": int(info["replacements"]),
                              "relres_true": float(info["relres_true"]),
                              "x_norm": float(np.linalg.norm(x)), "x_rows": [float(v) for v in x[rows]],
                              # the constant mode dominates x: the mean and the
                              # mean-removed values let a test see the rest
                              "x_mean": float(np.mean(x)),
                              "x_centred_norm": float(np.linalg.norm(x - np.mean(x))),
                              "x_rows_centred": [float(v) for v in x[rows] - np.mean(x)]}
        print(form, info, flush=True)
    with open(os.path.join(HERE, "q1hex128_oracle.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
