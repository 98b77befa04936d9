#!/usr/bin/env python3
"""Throughput of the SPOCK Chambolle-Pock step on one MI355X.

Workload: the large scenario tree -- horizon N = 15, branching 2 at stages
0-9 then 1 (1,024 scenarios, 7,167 nodes), nx = 50, nu = 25, box + ball
constraints, AV@R_0.95, seeded synthetic data (no dataset is involved).  A
"step" is one CP iteration T: the backward sweep (L*, S2, Riccati recursion)
and the forward sweep (dynamics, L, S3 projections) over the whole tree.

Reported value: CP iterations per second of the mixed-precision form (float32
steps on float32 copies of the float64 factors), with the plain float64 rate,
time-to-tolerance 1e-4 of both forms, the roofline of the dominant kernel
(HIP events on the library's stream) and the FP64 oracle on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SPOCK iters/s & time-to-tol (1e-4) vs plain FP64; serve p50/p99 latency"
WORKLOAD = ("large tree: N=15, branching 2 at stages 0-9 then 1 (1024 scenarios, 7167 nodes), "
            "nx=50, nu=25, box+ball, AV@R_0.95, Dirichlet probabilities")
HBM_PEAK_GBS = 8000.0


def cpu_baseline(steps):
    """The FP64 oracle (one thread) for `steps` CP steps of the same workload."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--cpu-steps", str(steps)]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def _cpu_baseline_only(steps):
    import numpy as np

    from oracle import spock_oracle as O
    from paper_2505_12078_amd import workloads as W
    prob = W.config_problem(2)
    D = O.Data(prob)
    F = O.Offline(D)
    a = O.step_size(D)
    z, e = np.zeros(D.layout.nz), np.zeros(D.layout.neta)
    t0 = time.perf_counter()
    for _ in range(steps):
        z, e = O.cp_step(D, F, z, e, a)
    dt = time.perf_counter() - t0
    print(json.dumps({"value": steps / dt, "unit": "CP iters/s", "cores": 1, "kind": "oracle",
                      "sample": "%d CP steps from zero on the same 7167-node tree, float64 NumPy, "
                                "one thread; offline factorisation not timed" % steps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tol", action="store_true")
    ap.add_argument("--cpu-baseline-only", action="store_true")
    args = ap.parse_args()
    if args.cpu_baseline_only:
        _cpu_baseline_only(args.cpu_steps)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the CP step of one scenario tree runs on one MI355X "
              "(multi-GPU sharding by subtrees is described in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2505_12078_amd import spock as S
    from paper_2505_12078_amd import workloads as W

    torch.cuda.set_device(0)
    prob = W.config_problem(2)
    t = time.perf_counter()
    P = S.Problem(prob, S.default_settings(eps=1e-4, precision=S.MIXED, check_every=20, max_iters=40000))
    t_setup = time.perf_counter() - t
    P.set_x0(prob["x0"])
    print("setup %.2fs, %s" % (t_setup, P.sizes), file=sys.stderr, flush=True)

    def rate(prec):
        P.run_steps(args.warmup, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.run_steps(args.steps, prec, sync=False)
        torch.cuda.synchronize()
        return args.steps / (time.perf_counter() - t0)

    v32 = rate(S.FP32)
    v64 = rate(S.FP64)
    print("iters/s: f32 %.1f  f64 %.1f" % (v32, v64), file=sys.stderr, flush=True)

    # per-kernel durations on the library's stream (HIP events around every launch)
    kt = {}
    for name, prec in (("f32", S.FP32), ("f64", S.FP64)):
        tot, tb, tf = P.time_steps(args.steps, prec)
        bb, bf = P.step_bytes(prec)
        kt[name] = dict(ms_step=tot, ms_backward=tb, ms_forward=tf, bytes_backward=bb, bytes_forward=bf)
    k = kt["f32"]
    dom = "forward" if k["ms_forward"] >= k["ms_backward"] else "backward"
    ms = k["ms_" + dom]
    by = k["bytes_" + dom]
    achieved = by / (ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_%s<float>" % dom, "avg_ms": round(ms, 4), "bytes_per_launch": by}

    tol = None
    if not args.no_tol:
        tol = {}
        for name, prec in (("mixed", S.MIXED), ("fp64", S.FP64)):
            P.set_settings(precision=prec)
            r = P.solve(prob["x0"])
            tol[name] = {"seconds": round(r["t_solve_s"], 3), "iters": r["iters"], "iters_f32": r["iters_fp32"],
                         "rel_res": r["rel_res"], "converged": r["code"] == S.SPOCK_OK, "s0": r["s0"],
                         "refined_in_f64": bool(r["refined"])}
            print("time-to-tol %s: %s" % (name, tol[name]), file=sys.stderr, flush=True)
        tol["speedup_mixed_vs_fp64"] = round(tol["fp64"]["seconds"] / max(tol["mixed"]["seconds"], 1e-9), 3)

    cpu = None if args.no_cpu else cpu_baseline(args.cpu_steps)
    out = {
        "metric": METRIC, "value": round(v32, 2), "unit": "CP iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1000.0 / v32, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD, "precision": "mixed: f32 steps on f32 copies of f64 factors, "
                   "f64 final check and refinement", "nodes": P.n, "nx": P.nx, "nu": P.nu,
                   "setup_s": round(t_setup, 3)},
        "fp64": {"iters_per_s": round(v64, 2), "ms_per_step": round(1000.0 / v64, 4)},
        "kernels": kt, "roofline": roofline, "time_to_tol": tol, "cpu_baseline": cpu,
    }
    P.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
