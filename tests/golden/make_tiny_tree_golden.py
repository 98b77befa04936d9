"""Write tests/golden/tiny_tree_vstar.json from the FP64 oracle alone.

Optimal values V* = s0 of plain CP iterations (Sec. 4.1) run from zero to a
relative residual (Sec. 5.3) far below the tolerances the tests use:
  * the tiny tree (N=3, binary, nx=2, nu=1, AV@R_0.95) at its initial state
    x0 and at 0.9 x0 and 0.81 x0 (the request sequence of the served-form
    tests), each at rel_res 1e-10;
  * a ragged tree (random_ragged_problem(1, N=4, nx=3, nu=2, max_children=3))
    at rel_res 1e-7;
and, for each, s0 of the same run when it first reached rel_res 1e-4, so a
test can state how far a 1e-4 solution of the oracle itself lies from V*.

Only `oracle/` does arithmetic here; `paper_2505_12078_amd.workloads` only
draws the seeded inputs.  Run from the repository root:
    python tests/golden/make_tiny_tree_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import spock_oracle as O  # noqa: E402
from paper_2505_12078_amd import workloads as W  # noqa: E402


def run(prob, eps, coarse=1e-4, max_iters=2_000_000):
    D = O.Data(prob)
    F = O.Offline(D)
    a = O.step_size(D)
    Y = D.layout
    z, eta = np.zeros(Y.nz), np.zeros(Y.neta)
    zr, er = O.cp_step(D, F, z, eta, a)
    x1, x2 = O.residuals(D, z, eta, zr, er, a)
    scale = max(1.0, float(np.abs(x1).max()), float(np.abs(x2).max()))
    at_coarse = None
    for k in range(1, max_iters + 1):
        zp, ep = O.cp_step(D, F, z, eta, a)
        x1, x2 = O.residuals(D, z, eta, zp, ep, a)
        z, eta = zp, ep
        rel = max(float(np.abs(x1).max()), float(np.abs(x2).max())) / scale
        if at_coarse is None and rel <= coarse:
            at_coarse = {"iters": k, "s0": float(z[0]), "rel_res": rel}
        if rel <= eps:
            break
    return {"eps": eps, "iters": k, "rel_res": rel, "vstar": float(z[0]), "at_1e-4": at_coarse}


def main(out=os.path.join(ROOT, "tests", "golden", "tiny_tree_vstar.json")):
    t0 = time.time()
    doc = {"_about": "Optimal values V* of the FP64 oracle (plain CP to a tight rel_res); written by "
                     "tests/golden/make_tiny_tree_golden.py, which calls only oracle/ (inputs from workloads.py).",
           "cite": "CP operator T (Sec. 4.1), residuals and relative residual (Sec. 5.3)"}
    tiny = W.config_problem(0)
    doc["tiny"] = []
    for i in range(3):
        p = dict(tiny)
        p["x0"] = tiny["x0"] * (0.9 ** i)
        r = run(p, 1e-10)
        r["x0_scale"] = 0.9 ** i
        doc["tiny"].append(r)
        print("tiny", i, r, "%.0f s" % (time.time() - t0), flush=True)
    r = run(W.random_ragged_problem(1, N=4, nx=3, nu=2, max_children=3), 1e-7)
    doc["ragged_a"] = r
    print("ragged_a", r, "%.0f s" % (time.time() - t0), flush=True)
    doc["oracle_seconds"] = time.time() - t0
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
