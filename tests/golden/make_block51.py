"""Write block51_oracle.json: the block-CG oracle's solve of the 51^3 Q1-hex
system (seed 0) with the 64 right-hand sides B = U[-1, 1] (seed 2), tol
1e-10, X0 = 0, Jacobi.

The GPU parity test at this size compares against these stored values
because the oracle needs minutes here.  Everything stored comes from
`oracle/` alone:

    python tests/golden/make_block51.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle.block_cg as bc  # noqa: E402
import workloads as W  # noqa: E402

N_SAMPLES = 256


def main():
    a, _ = W.problem(51, 0)
    B = W.multi_rhs(a.n, 64)
    rows = np.sort(np.random.default_rng(51).choice(a.n, N_SAMPLES, replace=False))
    X, info = bc.block_pcg(a, B, tol=1e-10)
    mean = X.mean(axis=0)
    out = {"workload": "q1hex 51^3 sigma+mass, seed 0; B = U[-1,1] (seed 2), 64 columns; tol 1e-10, X0 = 0, Jacobi",
           "n": int(a.n), "s": 64, "rows": rows.tolist(), "iters": int(info["iters"]),
           "status": int(info["status"]), "replacements": int(info["replacements"]),
           "min_rank": int(min(info["ranks"])), "relres_true": [float(v) for v in info["relres_true"]],
           "x_norm": [float(v) for v in np.linalg.norm(X, axis=0)],
           "x_mean": [float(v) for v in mean],
           "x_centred_norm": [float(v) for v in np.linalg.norm(X - mean, axis=0)],
           "x_rows": X[rows].tolist()}
    print({k: v for k, v in info.items() if k not in ("ranks", "relres_true")}, flush=True)
    with open(os.path.join(HERE, "block51_oracle.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
