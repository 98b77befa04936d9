#!/usr/bin/env python3
"""Throughput of the SPOCK Chambolle-Pock step on one MI355X.

Workload: the large scenario tree -- horizon N = 15, branching 2 at stages
0-9 then 1 (1,024 scenarios, 7,167 nodes), nx = 50, nu = 25, box + ball
constraints, AV@R_0.95, seeded synthetic data (no dataset is involved).  A
"step" is one CP iteration T over the whole tree: four launches -- prep
(node-parallel: L*, S2, the children-independent part of the Riccati-style
recursion), bsweep (leaves -> root recursion), fsweep (root -> leaves
dynamics) and dual (node-parallel: u = K x + d, L, S3 projections, Moreau).

Reported value: CP iterations per second of the mixed-precision form (float32
steps on float32 copies of the float64 factors), with the plain float64 rate,
time-to-tolerance 1e-4 of both forms, the roofline of the dominant kernel
(HIP events on the library's stream) and the FP64 oracle on the host cores.
Beside it: the batched workload (256 uneven trees in the same four launches per
step, aggregate rates, per-launch roofline, time to 1e-4 of the whole batch)
and the served form (continuous batching, p50/p99 latency).

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
KERNELS = ("prep", "bsweep", "fsweep", "dual")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
TRAFFIC_BATCHED_FILE = os.path.join(ROOT, "profiles", "traffic_batched.json")
BATCH_WORKLOAD = ("batched: 256 uneven trees, nx 4..32, nu=nx/2, N 5..20, branching 2..4 for 2..5 "
                  "stages then 1, box+ball, AV@R_0.9, Dirichlet probabilities")


def _kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("spock_kernels.hip", "spock_dev.h"):
        with open(os.path.join(ROOT, "paper_2505_12078_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _measured_traffic(kernel, path=TRAFFIC_FILE):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel sources changed since it was taken."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != _kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def _host_threads():
    """Threads the host gives this job: the OMP setting when there is one
    (the GPU machine sets it to its CPU share), else the visible CPUs."""
    try:
        return max(1, int(os.environ.get("OMP_NUM_THREADS", "")))
    except ValueError:
        return max(1, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count() or 1)


def _cpu_run(steps, threads):
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = str(threads)
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--cpu-steps", str(steps)]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baseline(steps):
    """The FP64 oracle for `steps` CP steps of the same workload, with the BLAS
    and OpenMP thread count set to every host thread the job has and to one."""
    threads = _host_threads()
    allc = _cpu_run(steps, threads)
    one = _cpu_run(steps, 1) if threads > 1 else dict(allc)
    if "error" in allc:
        return allc
    out = dict(allc)
    out["cores"] = threads
    out["sample"] = ("%d CP steps from zero on the same 7167-node tree, float64 NumPy, BLAS/OpenMP threads = %d "
                     "(os.cpu_count() = %s); offline factorisation not timed" % (steps, threads, os.cpu_count()))
    out["os_cpu_count"] = os.cpu_count()
    out["one_thread"] = {"value": one.get("value"), "unit": "CP iters/s", "cores": 1}
    return out


def cpu_baseline_case_study(case_study, instances=3, steps=2):
    """CPU baseline of the case-study leg: the oracle's seconds per CP step on
    the first accepted instances (a bounded sample, float64 NumPy as it
    stands), and that times the GPU's iteration count, the oracle's estimated
    time to the same tolerance."""
    import numpy as np

    from oracle import spock_oracle as O
    from paper_2505_12078_amd import workloads as W
    est = []
    for r in [r for r in case_study["rows"] if "seconds" in r][:instances]:
        prob = W.benchmark_problem(r["k"], nu_max=128)
        D = O.Data(prob)
        F = O.Offline(D)
        alpha = O.step_size(D)
        z, e = np.zeros(D.layout.nz), np.zeros(D.layout.neta)
        t = time.perf_counter()
        for _ in range(steps):
            z, e = O.cp_step(D, F, z, e, alpha)
        sec = (time.perf_counter() - t) / steps
        est.append({"k": r["k"], "oracle_s_per_step": round(sec, 4), "oracle_est_seconds": round(sec * r["iters"], 1),
                    "gpu_seconds": r["seconds"], "ratio": round(sec * r["iters"] / max(r["seconds"], 1e-9), 1)})
    return est


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
    print(json.dumps({"value": steps / dt, "unit": "CP iters/s", "kind": "oracle",
                      "threads_env": os.environ.get("OMP_NUM_THREADS")}))


def _batch_member(k):
    from paper_2505_12078_amd import workloads as W
    return W.batch_problem(k)


def make_batch_inputs(n_problems, workers=None):
    """The batched workload's members, drawn in a process pool (each member is
    seeded by its index, so the pool size does not change them).  Called before
    anything touches the GPU: the pool forks without exec.  Under a profiler
    that sets up the GPU before the program starts, draw in-process
    (workers=1)."""
    import multiprocessing as mp
    t = time.perf_counter()
    workers = max(1, min(workers or 16, os.cpu_count() or 1, n_problems))
    if workers == 1:
        probs = [_batch_member(k) for k in range(n_problems)]
    else:
        with mp.get_context("fork").Pool(workers) as pool:
            probs = pool.map(_batch_member, range(n_problems), chunksize=1)
    return probs, time.perf_counter() - t, workers


def batch_bench(S, probs, gen_s, workers, steps, warmup, solve=True, max_iters=20000, n_compare=64):
    """Batched form on the batched workload: every member advanced by the same
    four launches per step (float32 bulk), node workgroup picked by the
    autotuner on the batch itself; aggregate rates, per-launch roofline and the
    mixed-precision time to rel_res 1e-4 of the whole batch."""
    import numpy as np
    import torch

    from paper_2505_12078_amd import tune
    st = S.default_settings(eps=1e-4, precision=S.MIXED, check_every=20, max_iters=max_iters)
    t = time.perf_counter()
    members = [S.Problem(p, st) for p in probs]
    for P, p in zip(members, probs):
        P.set_x0(p["x0"])
    B = S.Batch(members, st)
    t_setup = time.perf_counter() - t
    nodes = int(sum(P.n for P in members))
    print("batch: %d problems, %d nodes, %d sweep tasks, %.2f GB, setup %.1fs"
          % (len(members), nodes, B.n_tasks, B.device_bytes / 1e9, t_setup), file=sys.stderr, flush=True)
    wg, tune_ms = tune.tune_batch(B, S.FP32)
    B.run_steps(warmup, S.FP32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.run_steps(steps, S.FP32, sync=False)
    torch.cuda.synchronize()
    rate = steps / (time.perf_counter() - t0)
    tot, ms_k = B.time_kernels(steps, S.FP32)
    by_k = B.kernel_bytes(S.FP32)
    kern = {"ms_step_events": round(tot, 5)}
    for kn, ms, by in zip(KERNELS, ms_k, by_k):
        kern[kn] = {"avg_ms": round(ms, 5), "bytes_per_launch": by, "GB_s": round(by / (ms * 1e-3) / 1e9, 1),
                    "frac_hbm": round(by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "traffic": _measured_traffic("k_%s<float>" % kn, TRAFFIC_BATCHED_FILE)}
    step_bytes = float(sum(by_k))
    out = {"workload": BATCH_WORKLOAD,
           "problems": len(members), "nodes": nodes, "batched_steps_per_s": round(rate, 2),
           "problem_iters_per_s": round(rate * len(members), 1), "node_steps_per_s": round(rate * nodes, 1),
           "ms_per_step": round(1000.0 / rate, 4), "bytes_per_step": step_bytes,
           "GB_s": round(step_bytes * rate / 1e9, 1), "frac_hbm": round(step_bytes * rate / 1e9 / HBM_PEAK_GBS, 4),
           "device_bytes": int(B.device_bytes + sum(P.sizes["device_bytes"] for P in members)),
           "kernels_f32": kern, "node_workgroup": wg,
           "tuner_ms_per_step": {str(k): round(v, 4) for k, v in tune_ms.items()},
           "gen_s": round(gen_s, 2), "gen_workers": workers, "setup_s": round(t_setup, 2)}
    print("batch: %.1f batched steps/s (%.3f ms), %.1f GB/s" % (rate, 1000.0 / rate, out["GB_s"]),
          file=sys.stderr, flush=True)
    if solve:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = B.solve([p["x0"] for p in probs])
        t_solve = time.perf_counter() - t0
        it = np.array([i["iters"] for i in infos])
        ok = sum(i["status"] == S.SPOCK_OK for i in infos)
        out["time_to_tol"] = {"eps": 1e-4, "seconds": round(t_solve, 3),
                              "converged": int(ok), "of": len(infos), "max_iters": max_iters,
                              "iters_median": int(np.median(it)), "iters_max": int(it.max()),
                              "refined_in_f64": int(sum(bool(i["refined"]) for i in infos))}
        print("batch time-to-tol: %s" % out["time_to_tol"], file=sys.stderr, flush=True)
        # mixed against plain float64 time-to-tolerance on the same members
        sub = members[:n_compare]
        cmp = {}
        for name, prec in (("mixed", S.MIXED), ("fp64", S.FP64)):
            Bs = S.Batch(sub, S.default_settings(eps=1e-4, precision=prec, check_every=20, max_iters=max_iters))
            Bs.set_launch(wg, S.FP32)
            Bs.set_launch(wg, S.FP64)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos = Bs.solve([p["x0"] for p in probs[:n_compare]])
            dt = time.perf_counter() - t0
            Bs.close()
            cmp[name] = {"seconds": round(dt, 3), "converged": int(sum(i["status"] == S.SPOCK_OK for i in infos)),
                         "iters_median": int(np.median([i["iters"] for i in infos])),
                         "s0": [i["s0"] for i in infos], "ok": [i["status"] == S.SPOCK_OK for i in infos]}
        s_m, s_d = np.array(cmp["mixed"].pop("s0")), np.array(cmp["fp64"].pop("s0"))
        both = np.array(cmp["mixed"].pop("ok")) & np.array(cmp["fp64"].pop("ok"))
        cmp["members"] = n_compare
        cmp["converged_both"] = int(both.sum())
        cmp["max_rel_s0_diff_converged"] = (float(np.max(np.abs(s_m - s_d)[both] / np.maximum(1.0, np.abs(s_d[both]))))
                                            if both.any() else None)
        cmp["speedup_mixed_vs_fp64"] = round(cmp["fp64"]["seconds"] / max(cmp["mixed"]["seconds"], 1e-9), 3)
        out["time_to_tol_mixed_vs_fp64"] = cmp
        print("batch mixed vs fp64 (%d members): %s" % (n_compare, cmp), file=sys.stderr, flush=True)
    B.close()
    for P in members:
        P.close()
    return out


def supermann_time_to_tol(S, prob, eps, max_iters=40000):
    """The SPOCK outer method (SuperMann with Anderson directions, float64)
    from zero to rel_res eps: wall time, SuperMann iterations, applications of
    T and the K0 / K1 / K2 step counts."""
    with S.Problem(prob, S.default_settings(eps=eps, max_iters=max_iters, method=S.SUPERMANN)) as Q:
        r = Q.solve(prob["x0"])
    return {"seconds": round(r["t_solve_s"], 4), "iters": r["iters"], "T_applications": r["n_T"],
            "K0": r["n_K0"], "K1": r["n_K1"], "K2": r["n_K2"], "rel_res": r["rel_res"],
            "converged": r["code"] == S.SPOCK_OK, "s0": r["s0"]}


def small_trees_bench(S, W):
    """Plain float64 CP on the tiny tree (15 nodes) and the medium tree (229
    nodes): steps per second, microseconds per step and per stage level (a
    step walks the N stages twice, backward and forward), and the time to the
    tolerance the configurations state (tiny: rel_res 1e-6; medium: 1e-4,
    which plain CP reaches in about 1.1e4 steps -- 1e-6 takes more than 3e5)."""
    import torch
    out = {}
    for cfg, eps, name in ((0, 1e-6, "tiny"), (1, 1e-4, "medium")):
        prob = W.config_problem(cfg)
        with S.Problem(prob, S.default_settings(eps=eps, max_iters=400000)) as P:
            P.set_x0(prob["x0"])
            P.run_steps(200, S.FP64)
            torch.cuda.synchronize()
            steps = 4000
            t0 = time.perf_counter()
            P.run_steps(steps, S.FP64, sync=False)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            r = P.solve(prob["x0"])
            N = P.sizes["N"]
            out[name] = {"nodes": P.n, "N": N, "nx": P.nx, "nu": P.nu, "steps_per_s": round(1.0 / dt, 1),
                         "us_per_step": round(dt * 1e6, 2), "us_per_stage_level": round(dt * 1e6 / (2 * N), 2),
                         "time_to_tol": {"eps": eps, "seconds": round(r["t_solve_s"], 4), "iters": r["iters"],
                                         "converged": r["code"] == S.SPOCK_OK, "s0": r["s0"]}}
        out[name]["time_to_tol_supermann"] = supermann_time_to_tol(S, prob, eps, max_iters=100000)
        print("%s tree: %s" % (name, out[name]), file=sys.stderr, flush=True)
    return out


def generality_bench(S, W, prob, steps=200):
    """The large tree with the general parts of the formulation in place of
    AV@R and the box-and-ball constraints: a spectral risk and the l2-ball
    ambiguity risk at every non-leaf node (conic data, Sec. 3.3), and the l1
    input penalty of Prop. 2 (slack inputs and general rows; no ball).  Each
    runs the node kernels built with the general products; per variant the
    setup time and the float32 and float64 milliseconds per CP step."""
    import torch
    variants = {"avar": prob, "spectral": W.spectral_risk(prob, weight=0.5, gammas=(0.2, 0.95)),
                "l2_ball": W.l2_ball_risk(prob, r_frac=0.5),
                "l1_penalty": W.l1_input_penalty(dict(prob, x_ball=0.0, xN_ball=0.0), 0.1)}
    out = {}
    for name, p in variants.items():
        t0 = time.perf_counter()
        with S.Problem(p) as P:
            setup = time.perf_counter() - t0
            P.set_x0(p["x0"])
            row = {"setup_s": round(setup, 3), "nu": P.nu,
                   "y_entries": int(P.nz - 1 - P.n * P.nx - P.n_nl * P.nu - 2 * (P.n - 1)),
                   "device_MB": round(P.sizes["device_bytes"] / 1e6, 1)}
            for prec, key in ((S.FP32, "f32"), (S.FP64, "f64")):
                P.run_steps(20, prec)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                P.run_steps(steps, prec, sync=False)
                torch.cuda.synchronize()
                row[key + "_ms_per_step"] = round((time.perf_counter() - t0) / steps * 1e3, 4)
        out[name] = row
        print("generality %s: %s" % (name, row), file=sys.stderr, flush=True)
    return out


def delay_bench(S, W, ns=(2, 4), steps=40):
    """The networked-control case study's parallelization question: CP step
    time of the delay tree's shapes (N = 48, n^2 equiprobable scenarios as
    [n^2, 1, ..., 1] and as [n, n, 1, ..., 1]) at its sizes (state 150 = plant
    100 plus the previous input, nu = 50: products of 150 and 200 outputs),
    float64 and float32, with the algorithmic bytes per step.  The case
    study's own dynamics grow about 150-fold per stage, so over 48 stages the
    offline factorisation leaves float64 (P ~ 150^(2t)); the timed instances
    take random stable dynamics of the same sizes on the same trees (a step's
    work does not depend on the values)."""
    import numpy as np
    import torch
    out = []
    for n in ns:
        for wide in (True, False):
            br = W.delay_branching(n, wide_first=wide)
            parent, _ = W.tree_from_branching(br)
            prob = W.make_problem(parent, 150, 50, np.random.default_rng(1385 + n), x_ball=15.0,
                                  name="delay_shape_n%d" % n)
            t = time.perf_counter()
            with S.Problem(prob, S.default_settings()) as P:
                t_setup = time.perf_counter() - t
                P.set_x0(prob["x0"])
                row = {"n": n, "shape": "[n^2,1,...]" if wide else "[n,n,1,...]", "nodes": P.n,
                       "scenarios": n * n, "setup_s": round(t_setup, 2)}
                for name, prec in (("f64", S.FP64), ("f32", S.FP32)):
                    P.set_iterate(np.zeros(P.nz), np.zeros(P.neta))
                    P.run_steps(4, prec)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    P.run_steps(steps, prec, sync=False)
                    torch.cuda.synchronize()
                    dt = (time.perf_counter() - t0) / steps
                    by = float(sum(P.kernel_bytes(prec)))
                    row[name] = {"ms_per_step": round(dt * 1e3, 4), "steps_per_s": round(1.0 / dt, 1),
                                 "GB_s": round(by / dt / 1e9, 1)}
            out.append(row)
            print("delay tree: %s" % row, file=sys.stderr, flush=True)
    return out


def case_study_bench(S, W, instances=10, eps=1e-3, max_iters=20000):
    """The benchmark case study's random problems (dense event-dependent Q, R;
    n_u capped at 128 so that nx = 2 n_u fits the library): for instances
    0..K-1, setup time, device footprint, and the time, iterations and
    outcome of a mixed-precision solve from zero to rel_res eps (the paper
    recommends float for tolerances around 1e-3).  Its CPU baseline is
    cpu_baseline_case_study."""
    import numpy as np
    import torch
    rows = []
    for k in range(instances):
        prob = W.benchmark_problem(k, nu_max=128)
        row = {"k": k, "name": prob["name"], "n_v": int(prob["n_v"]), "nodes": len(prob["parent"]),
               "nx": int(prob["nx"]), "nu": int(prob["nu"])}
        try:
            row["footprint_bytes"] = S.footprint(prob, S.default_settings(precision=S.MIXED))
            t = time.perf_counter()
            with S.Problem(prob, S.default_settings(eps=eps, precision=S.MIXED, max_iters=max_iters)) as P:
                row["setup_s"] = round(time.perf_counter() - t, 3)
                r = P.solve(prob["x0"])
                torch.cuda.synchronize()
                row.update(seconds=round(r["t_solve_s"], 4), iters=r["iters"], rel_res=r["rel_res"],
                           converged=r["code"] == S.SPOCK_OK, s0=r["s0"])
        except S.SpockError as e:
            row["error"] = str(e)
        rows.append(row)
        print("case study instance: %s" % row, file=sys.stderr, flush=True)
    done = [r for r in rows if "seconds" in r]
    out = {"eps": eps, "precision": "mixed", "max_iters": max_iters, "instances": len(rows),
           "accepted": len(done), "converged": sum(1 for r in done if r["converged"]),
           "median_seconds": float(np.median([r["seconds"] for r in done])) if done else None,
           "max_seconds": max((r["seconds"] for r in done), default=None),
           "median_footprint_MB": float(np.median([r["footprint_bytes"] for r in done]) / 2 ** 20) if done else None,
           "rows": rows}
    return out


def serve_bench(S, W, duration_s=10.0, session_rate=20.0, req_per_session=10, gap_mean=0.5,
                drain_s=40.0, budget=200 << 30, seed=4, precision=None):
    """Poisson sessions (rate session_rate/s), each one tree drawn uniformly from
    {medium tree, large tree, a batched-workload tree} issuing req_per_session
    requests with exponential gaps (mean gap_mean s); request k+1 shifts x0 by
    N(0, 0.1) and re-applies the feasibility guard; warm starts from the
    resident iterate; eps 1e-4, mixed precision unless `precision` says
    otherwise; admission within `budget` bytes of HBM.  Latency = submit ->
    result.  Requests still open when the drain window ends are censored
    there: their latency is at least (window end - submit), and the
    all-request percentiles use that lower bound."""
    import threading
    import numpy as np
    rng = np.random.default_rng(seed)
    pool = {"medium": [W.config_problem(1, i) for i in range(3)],
            "large": [W.config_problem(2, 0)],
            "batched": [W.batch_problem(k, seed=5) for k in range(12)]}
    shapes = ["medium", "large", "batched"]
    # schedule
    sessions = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / session_rate)
        if t > duration_s:
            break
        kind = shapes[int(rng.integers(3))]
        prob = pool[kind][int(rng.integers(len(pool[kind])))]
        times, x0s = [t], [prob["x0"]]
        x = prob["x0"]
        n_nl = prob["gamma"].size
        for _ in range(req_per_session - 1):
            times.append(times[-1] + rng.exponential(gap_mean))
            x = W._guard_x0(x + rng.normal(0.0, np.sqrt(0.1), size=x.size), prob["parent"], prob["A"],
                            prob["x_hi"], prob["x_ball"], prob["xN_hi"], prob["xN_ball"], n_nl)
            x0s.append(x)
        sessions.append((kind, prob, times, x0s))
    settings = S.default_settings(eps=1e-4, precision=S.MIXED if precision is None else precision,
                                  max_iters=200000, check_every=20)
    srv = S.Server(budget, settings)
    ids = [srv.add_tree(sess[1]) for sess in sessions]
    events = sorted((tm, si, k) for si, sess in enumerate(sessions) for k, tm in enumerate(sess[2]))
    results = []
    stop = threading.Event()

    def poller():
        while not stop.is_set():
            results.extend(srv.poll())
            time.sleep(0.01)
        results.extend(srv.poll())

    th = threading.Thread(target=poller)
    th.start()
    t0 = time.perf_counter()
    t_sub = {}
    for tm, si, k in events:
        dt = tm - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        t_sub[si * 1000 + k] = S.now()
        srv.submit(ids[si], sessions[si][3][k], si * 1000 + k)
    t_end = time.perf_counter() + drain_s
    while time.perf_counter() < t_end and len(results) < len(events):
        time.sleep(0.05)
    stop.set()
    th.join()
    t_cut = S.now()
    st = srv.stats()
    srv.close()
    ok = [r for r in results if r["status"] == 0]
    done = {r["req_id"]: r["t_done"] - r["t_submit"] for r in results}
    # every request: finished ones with their latency, open ones censored at the cut
    lat_all = np.array([done.get(q, t_cut - t) for q, t in t_sub.items()])
    lat_ok = np.array([r["t_done"] - r["t_submit"] for r in ok]) if ok else np.array([np.nan])
    span = (max(r["t_done"] for r in results) - min(r["t_submit"] for r in results)) if results else float("nan")
    by_kind = {}
    for q, t in t_sub.items():
        kind = sessions[q // 1000][0]
        by_kind.setdefault(kind, []).append(done.get(q, t_cut - t))
    return {"offered_req_per_s": round(len(events) / duration_s, 2), "requests": len(events),
            "precision": "fp64" if precision == S.FP64 else "mixed", "budget_bytes": int(budget),
            "completed_ok": len(ok), "completed": len(results),
            "completed_fraction": round(len(results) / max(1, len(events)), 4),
            "solves_per_s": round(len(ok) / span, 2) if results else 0.0,
            "p50_latency_s": round(float(np.percentile(lat_all, 50)), 4),
            "p99_latency_s": round(float(np.percentile(lat_all, 99)), 4),
            "latency_note": "over every request; open requests censored at the end of the drain window "
                            "(lower bounds)" if len(results) < len(events) else "over every request",
            "p50_latency_completed_s": round(float(np.percentile(lat_ok, 50)), 4),
            "p99_latency_completed_s": round(float(np.percentile(lat_ok, 99)), 4),
            "p50_by_shape_s": {k: round(float(np.percentile(v, 50)), 4) for k, v in by_kind.items()},
            "warm_fraction": round(float(np.mean([r["warm"] for r in ok])), 3) if ok else 0.0,
            "mean_iters": round(float(np.mean([r["info"]["iters"] for r in ok])), 1) if ok else 0.0,
            "median_iters_warm": (round(float(np.median([r["info"]["iters"] for r in ok if r["warm"]])), 1)
                                  if any(r["warm"] for r in ok) else None),
            "median_iters_cold": (round(float(np.median([r["info"]["iters"] for r in ok if not r["warm"]])), 1)
                                  if any(not r["warm"] for r in ok) else None),
            "sessions": len(sessions), "duration_s": duration_s, "drain_s": drain_s,
            "server": {k: int(v) for k, v in st.items()}}


def _profile_pass(steps):
    """What a profiler should see: `steps` float32 and float64 CP steps of the
    large tree (k_prep / k_bsweep / k_fsweep / k_dual) and one copy of 1 GiB (a
    plain kernel of known traffic for scaling the memory counters)."""
    import torch

    from paper_2505_12078_amd import spock as S
    from paper_2505_12078_amd import workloads as W
    torch.cuda.set_device(0)
    prob = W.config_problem(2)
    P = S.Problem(prob, S.default_settings())
    P.set_x0(prob["x0"])
    for prec in (S.FP32, S.FP64):
        P.run_steps(steps, prec)
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    b32 = P.kernel_bytes(S.FP32)
    b64 = P.kernel_bytes(S.FP64)
    print(json.dumps({"steps": steps, "copy_bytes": 1 << 30, "source_hash": _kernel_source_hash(),
                      "bytes_f32": dict(zip(KERNELS, b32)), "bytes_f64": dict(zip(KERNELS, b64))}))
    P.close()


def _profile_supermann_pass(iters):
    """What a profiler should see for the SuperMann outer method: `iters`
    float64 SuperMann iterations on the large tree (CP step kernels, k_combo,
    k_dots / k_dots_final, k_apply_L)."""
    import torch

    from paper_2505_12078_amd import spock as S
    from paper_2505_12078_amd import workloads as W
    torch.cuda.set_device(0)
    prob = W.config_problem(2)
    with S.Problem(prob, S.default_settings(eps=1e-12, max_iters=iters, method=S.SUPERMANN)) as P:
        r = P.solve(prob["x0"])
    print(json.dumps({"iters": r["iters"], "T": r["n_T"], "K0": r["n_K0"], "K1": r["n_K1"], "K2": r["n_K2"],
                      "seconds": r["t_solve_s"]}))


def _profile_batch_pass(n_problems, steps, node_wg):
    """What a profiler should see for the batched workload: `steps` float32
    batched steps of its 256 members at `node_wg` threads per node workgroup
    (the autotuner's pick on this workload) and one copy of 1 GiB."""
    probs, _, _ = make_batch_inputs(n_problems, workers=1)
    import torch

    from paper_2505_12078_amd import spock as S
    torch.cuda.set_device(0)
    members = [S.Problem(p, S.default_settings()) for p in probs]
    for P, p in zip(members, probs):
        P.set_x0(p["x0"])
    B = S.Batch(members, S.default_settings())
    B.set_launch(node_wg, S.FP32)
    B.run_steps(steps + (steps & 1), S.FP32)
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"steps": steps + (steps & 1), "copy_bytes": 1 << 30, "source_hash": _kernel_source_hash(),
                      "workload": BATCH_WORKLOAD, "node_workgroup": node_wg,
                      "bytes_f32": dict(zip(KERNELS, B.kernel_bytes(S.FP32))), "bytes_f64": None}))
    B.close()
    for P in members:
        P.close()


def summarize_counters(fetch_dir, write_dir, trace_dir, profile_json, out_path=None):
    """Per-launch HBM traffic of the four kernels from two rocprofv3 counter
    runs of `bench.py --profile` (FETCH_SIZE, WRITE_SIZE; KiB per dispatch),
    scaled by what the same counters read for the 1 GiB device copy of that
    run, next to the algorithmic bytes and the kernel-trace durations.  Writes
    profiles/traffic.json (or out_path; the batched workload's counters, from
    `bench.py --profile-batch`, go to TRAFFIC_BATCHED_FILE) and prints
    a markdown table."""
    import csv
    import glob
    import re

    pat = re.compile(r"k_(prep|bsweep|fsweep|dual)(?:_st)?<(float|double), (\d+)(?:, (?:true|false|[012]))?>")

    def rows(d, suffix):
        out = []
        for f in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
            with open(f) as fh:
                out.extend(csv.DictReader(fh))
        return out

    def per_kernel(d, counter):
        vals, names, copy = {}, {}, 0.0
        for r in rows(d, "counter_collection.csv"):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            if "copyBuffer" in r["Kernel_Name"]:
                copy = max(copy, v)
                continue
            m = pat.search(r["Kernel_Name"])
            if m:
                key = "k_%s<%s>" % (m.group(1), m.group(2))
                vals.setdefault(key, []).append(v)
                names[key] = r["Kernel_Name"].split("(")[0].replace("void ", "")
        return {k: sum(v) / len(v) for k, v in vals.items()}, names, copy

    fetch, names, copy_f = per_kernel(fetch_dir, "FETCH_SIZE")
    write, _, copy_w = per_kernel(write_dir, "WRITE_SIZE")
    with open(profile_json) as fh:
        prof = json.loads(fh.read().strip().splitlines()[-1])
    copy_bytes = prof["copy_bytes"]
    ff, wf = copy_bytes / (copy_f * 1024.0), copy_bytes / (copy_w * 1024.0)
    avg_us = {}
    for r in rows(trace_dir, "kernel_stats.csv"):
        m = pat.search(r["Name"])
        if m:
            avg_us["k_%s<%s>" % (m.group(1), m.group(2))] = float(r["AverageNs"]) / 1e3
    out = {"workload": prof.get("workload", WORKLOAD), "source_hash": prof["source_hash"],
           "calibration": {"copy_bytes": copy_bytes, "fetch_factor": round(ff, 4), "write_factor": round(wf, 4)},
           "kernels": {}}
    print("| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM MB (calibrated) | algorithmic MB | ratio | avg us (trace) |")
    print("|---|---|---|---|---|---|---|")
    for prec, tag in (("float", "bytes_f32"), ("double", "bytes_f64")):
        for kn in KERNELS:
            key = "k_%s<%s>" % (kn, prec)
            if key not in fetch or key not in write or not prof.get(tag):
                continue
            fb, wb = fetch[key] * 1024.0 * ff, write[key] * 1024.0 * wf
            alg = prof[tag][kn]
            out["kernels"][key] = {"kernel": names.get(key, key), "fetch_bytes": int(fb), "write_bytes": int(wb),
                                   "bytes_per_launch": int(fb + wb), "algorithmic_bytes": alg,
                                   "ratio_to_algorithmic": round((fb + wb) / alg, 3), "avg_us_trace": avg_us.get(key)}
            print("| %s | %.1f | %.1f | %.1f | %.1f | %.2f | %s |" % (
                names.get(key, key), fetch[key], write[key], (fb + wb) / 1e6, alg / 1e6, (fb + wb) / alg,
                "%.1f" % avg_us[key] if key in avg_us else "-"))
    with open(out_path or TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print("calibration: fetch x%.4f, write x%.4f (1 GiB copy reads FETCH_SIZE %.0f KiB, WRITE_SIZE %.0f KiB)" % (
        ff, wf, copy_f, copy_w))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=24)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tol", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=20.0, help="sessions per second (10 requests each)")
    ap.add_argument("--serve-rate-sustained", type=float, default=0.5,
                    help="a second, lower session rate the device keeps up with (0: skip)")
    ap.add_argument("--serve-drain", type=float, default=20.0,
                    help="seconds the saturated serving runs wait for open requests after the last arrival")
    ap.add_argument("--serve-budget-gb", type=float, default=8.0,
                    help="HBM budget of the capped serving run (0: skip)")
    ap.add_argument("--serve-capped-seconds", type=float, default=5.0)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--no-small", action="store_true", help="skip the tiny and medium trees")
    ap.add_argument("--no-delay", action="store_true", help="skip the networked-control delay trees")
    ap.add_argument("--no-general", action="store_true",
                    help="skip the large tree with general risks and the l1 penalty")
    ap.add_argument("--case-study", type=int, default=6,
                    help="instances of the benchmark case study's random problems to solve (0: skip)")
    ap.add_argument("--case-study-only", action="store_true", help="run only the case-study leg (one JSON line)")
    ap.add_argument("--case-study-iters", type=int, default=1000, help="iteration cap per case-study solve")
    ap.add_argument("--case-study-eps", type=float, default=1e-3)
    ap.add_argument("--batch-problems", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=50)
    ap.add_argument("--no-batch-solve", action="store_true")
    ap.add_argument("--cpu-baseline-only", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: K steps per precision and a 1 GiB device copy")
    ap.add_argument("--profile-batch", action="store_true",
                    help="short run for rocprofv3: K float32 batched steps of the batched workload and a 1 GiB copy")
    ap.add_argument("--profile-supermann", action="store_true",
                    help="short run for rocprofv3: K float64 SuperMann iterations on the large tree")
    ap.add_argument("--batch-node-wg", type=int, default=256)
    ap.add_argument("--traffic-out", default=None, help="output of --summarize-counters (default profiles/traffic.json)")
    ap.add_argument("--summarize-counters", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "TRACE_DIR", "PROFILE_JSON"),
                    help="write profiles/traffic.json from rocprofv3 output of --profile runs (no GPU needed)")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, out_path=args.traffic_out)
        return
    if args.profile_batch:
        _profile_batch_pass(args.batch_problems, args.steps, args.batch_node_wg)
        return
    if args.profile_supermann:
        _profile_supermann_pass(args.steps)
        return
    if args.cpu_baseline_only:
        _cpu_baseline_only(args.cpu_steps)
        return
    if args.profile:
        _profile_pass(args.steps)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the CP step of one scenario tree runs on one MI355X "
              "(sharding a tree by subtrees across GPUs is designed, not built)", file=sys.stderr)
        sys.exit(2)
    if args.case_study_only:
        import torch

        from paper_2505_12078_amd import spock as S
        from paper_2505_12078_amd import workloads as W
        torch.cuda.set_device(0)
        cs = case_study_bench(S, W, instances=args.case_study, eps=args.case_study_eps,
                              max_iters=args.case_study_iters)
        if not args.no_cpu:
            cs["cpu_baseline"] = cpu_baseline_case_study(cs)
        print(json.dumps({"case_study": cs}))
        return

    batch_in = None
    if not args.no_batch:
        batch_in = make_batch_inputs(args.batch_problems)
        print("batch inputs: %d problems in %.1fs (%d workers)" % (len(batch_in[0]), batch_in[1], batch_in[2]),
              file=sys.stderr, flush=True)

    import torch

    from paper_2505_12078_amd import spock as S
    from paper_2505_12078_amd import workloads as W

    torch.cuda.set_device(0)
    prob = W.config_problem(2)
    t = time.perf_counter()
    P = S.Problem(prob, S.default_settings(eps=1e-4, precision=S.MIXED, check_every=20, max_iters=40000))
    t_setup = time.perf_counter() - t
    P.set_x0(prob["x0"])
    nodes = P.n
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
        tot, ms_k = P.time_kernels(args.steps, prec)
        by_k = P.kernel_bytes(prec)
        kt[name] = {"ms_step_events": round(tot, 5)}
        for kn, ms, by in zip(KERNELS, ms_k, by_k):
            kt[name][kn] = {"avg_ms": round(ms, 5), "bytes_per_launch": by,
                            "GB_s": round(by / (ms * 1e-3) / 1e9, 1), "frac_hbm": round(by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    k = kt["f32"]
    dom = max(KERNELS, key=lambda kn: k[kn]["avg_ms"])
    ms, by = k[dom]["avg_ms"], k[dom]["bytes_per_launch"]
    achieved = by / (ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": _measured_traffic("k_%s<float>" % dom),
                "kernel": "k_%s<float>" % dom, "avg_ms": ms, "bytes_per_launch": by}

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
        tol["supermann_fp64"] = supermann_time_to_tol(S, prob, 1e-4)
        print("time-to-tol supermann fp64: %s" % tol["supermann_fp64"], file=sys.stderr, flush=True)

    P.close()
    general = None if args.no_general else generality_bench(S, W, prob)
    small = None if args.no_small else small_trees_bench(S, W)
    delay = None if args.no_delay else delay_bench(S, W)
    case_study = (case_study_bench(S, W, instances=args.case_study, eps=args.case_study_eps,
                                   max_iters=args.case_study_iters) if args.case_study > 0 else None)
    batched = None
    if batch_in is not None:
        batched = batch_bench(S, *batch_in, steps=args.batch_steps + (args.batch_steps & 1), warmup=6,
                              solve=not args.no_batch_solve)
        batch_in = None
    serve = None
    if not args.no_serve:
        serve = serve_bench(S, W, duration_s=args.serve_seconds, session_rate=args.serve_rate,
                            drain_s=args.serve_drain)
        print("serve: %s" % serve, file=sys.stderr, flush=True)
        if args.serve_rate_sustained > 0:
            serve["sustained"] = serve_bench(S, W, duration_s=args.serve_seconds,
                                             session_rate=args.serve_rate_sustained, seed=7)
            print("serve (sustained rate): %s" % serve["sustained"], file=sys.stderr, flush=True)
            # the same request stream served by plain float64 iterations
            serve["sustained_fp64"] = serve_bench(S, W, duration_s=args.serve_seconds,
                                                  session_rate=args.serve_rate_sustained, seed=7,
                                                  precision=S.FP64)
            print("serve (sustained rate, fp64): %s" % serve["sustained_fp64"], file=sys.stderr, flush=True)
        if args.serve_budget_gb > 0:
            # admission under a capped HBM budget: trees are evicted and set up again
            serve["capped"] = serve_bench(S, W, duration_s=args.serve_capped_seconds, session_rate=args.serve_rate,
                                          drain_s=args.serve_drain, budget=int(args.serve_budget_gb * (1 << 30)),
                                          seed=9)
            print("serve (capped budget): %s" % serve["capped"], file=sys.stderr, flush=True)
    cpu = None if args.no_cpu else cpu_baseline(args.cpu_steps)
    if case_study is not None and not args.no_cpu:
        case_study["cpu_baseline"] = cpu_baseline_case_study(case_study)
    out = {
        "metric": METRIC, "value": round(v32, 2), "unit": "CP iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1000.0 / v32, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD, "precision": "mixed: f32 steps on f32 copies of f64 factors, "
                   "f64 final check and refinement", "nodes": nodes, "nx": 50, "nu": 25,
                   "setup_s": round(t_setup, 3)},
        "fp64": {"iters_per_s": round(v64, 2), "ms_per_step": round(1000.0 / v64, 4)},
        "kernels": kt, "roofline": roofline, "time_to_tol": tol, "small_trees": small, "generality": general, "delay_trees": delay,
        "case_study": case_study,
        "batched": batched,
        "serve": serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
