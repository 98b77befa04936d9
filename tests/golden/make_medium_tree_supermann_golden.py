"""Write tests/golden/medium_tree_supermann.json from the FP64 oracle alone.

The medium tree (N=10, branching 3 at stages 0-2 then 1: 229 nodes, nx=20,
nu=10, box and ball constraints, AV@R_0.9) solved to the relative residual
1e-6 of Sec. 5.3 by the SPOCK outer method (SuperMann with Anderson
directions, Sec. 5.2, oracle/supermann_oracle.py), which plain CP iterations
do not reach in 3e5 steps.  Stores V* = s0, the iteration and T counts, and
the nested risk objective and dynamics violation of the unscaled (x, u).

Only `oracle/` does arithmetic here; `paper_2505_12078_amd.workloads` only
draws the seeded inputs.  Run from the repository root:
    python tests/golden/make_medium_tree_supermann_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import spock_oracle as O  # noqa: E402
from oracle import supermann_oracle as SM  # noqa: E402
from paper_2505_12078_amd import workloads as W  # noqa: E402


def main(out=os.path.join(ROOT, "tests", "golden", "medium_tree_supermann.json")):
    prob = W.config_problem(1)
    t0 = time.time()
    r = SM.solve(prob, eps=1e-6, max_iters=100000)
    doc = {"_about": "FP64 SuperMann oracle solve of the medium tree (config_problem(1)) to rel_res 1e-6; "
                     "written by tests/golden/make_medium_tree_supermann_golden.py from oracle/ alone.",
           "cite": "SPOCK algorithm and Anderson's acceleration (Sec. 5.2), termination (Sec. 5.3)",
           "eps": 1e-6, "status": r["status"], "iters": r["iters"], "counts": r["counts"],
           "rel_res": r["rel_res"], "vstar": r["s0"], "alpha": r["alpha"],
           "nested_cost": O.nested_cost(prob, r["x"], r["u"]),
           "dynamics_violation": O.dynamics_violation(prob, r["x"], r["u"]),
           "oracle_seconds": time.time() - t0}
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", out, doc)


if __name__ == "__main__":
    main()
