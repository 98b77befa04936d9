"""Write tests/golden/medium_tree_cp.json from the FP64 oracle alone.

The medium tree (N=10, branching 3 at stages 0-2 then 1: 229 nodes, nx=20,
nu=10, box and ball constraints, AV@R_0.9, Dirichlet(1) probabilities) is
solved by plain CP iterations (Sec. 4.1) from zero to the relative residual
1e-4 of Sec. 5.3 (rel_res as in the oracle's solve).  The file keeps, at a
few iteration counts K on that trajectory, s0 and every 97th entry of z and
eta (with the indices), so a GPU run of exactly K steps from zero can be
compared entry by entry; and at the stopping iteration the iteration count,
rel_res, V* = s0 and the nested risk objective of the unscaled (x, u) there.

Only `oracle/` does arithmetic here; `paper_2505_12078_amd.workloads` only
draws the seeded inputs.  Run from the repository root:
    python tests/golden/make_medium_tree_golden.py
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

EPS = 1e-4
CHECKPOINTS = (200, 1000, 5000)
STRIDE = 97


def snapshot(k, z, eta):
    iz = list(range(0, len(z), STRIDE))
    ie = list(range(0, len(eta), STRIDE))
    return {"iters": k, "s0": float(z[0]), "z_idx_stride": STRIDE,
            "z": [float(z[i]) for i in iz], "eta": [float(eta[i]) for i in ie],
            "z_inf": float(np.abs(z).max()), "eta_inf": float(np.abs(eta).max())}


def main(out=os.path.join(ROOT, "tests", "golden", "medium_tree_cp.json")):
    prob = W.config_problem(1)
    D = O.Data(prob)
    F = O.Offline(D)
    a = O.step_size(D)
    Y = D.layout
    z = np.zeros(Y.nz)
    eta = np.zeros(Y.neta)
    zr, er = O.cp_step(D, F, z, eta, a)
    x1, x2 = O.residuals(D, z, eta, zr, er, a)
    ref = (float(np.abs(x1).max()), float(np.abs(x2).max()))
    scale = max(1.0, *ref)
    snaps = []
    t0 = time.time()
    k = 0
    rel = np.inf
    r1 = r2 = np.inf
    while True:
        zp, ep = O.cp_step(D, F, z, eta, a)
        x1, x2 = O.residuals(D, z, eta, zp, ep, a)
        z, eta = zp, ep
        k += 1
        r1, r2 = float(np.abs(x1).max()), float(np.abs(x2).max())
        rel = max(r1, r2) / scale
        if k in CHECKPOINTS:
            snaps.append(snapshot(k, z, eta))
        if k % 500 == 0:
            print("step %d rel_res %.3e (%.0f s)" % (k, rel, time.time() - t0), flush=True)
        if rel <= EPS or k >= 200000:
            break
    x = np.array([Y.x(z, i) for i in range(D.tree.n)])
    u = np.array([Y.u(z, i) for i in range(D.tree.n_nl)])
    xs, us = D.unscale(x, u)
    doc = {
        "_about": "FP64 oracle trajectory of plain CP from zero on the medium tree "
                  "(config_problem(1)); written by tests/golden/make_medium_tree_golden.py, "
                  "which calls only oracle/ (inputs from workloads.py).",
        "cite": "CP operator T (Sec. 4.1), residuals and relative residual (Sec. 5.3)",
        "alpha": a, "L_norm": float(O.L_norm(D)), "xi_ref": ref, "eps": EPS,
        "nz": int(Y.nz), "neta": int(Y.neta),
        "stop": {"iters": k, "rel_res": rel, "xi1": r1, "xi2": r2, "s0": float(z[0]),
                 "nested_cost": O.nested_cost(prob, xs, us),
                 "dynamics_violation": O.dynamics_violation(prob, xs, us)},
        "snapshots": snaps,
        "final": snapshot(k, z, eta),
        "oracle_seconds": time.time() - t0,
    }
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", out, doc["stop"])


if __name__ == "__main__":
    main()
