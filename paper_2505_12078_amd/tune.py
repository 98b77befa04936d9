"""Autotuner for the launch shape of the node-parallel kernels.

Two of a CP step's four launches (prep and dual) run one wavefront per tree
node, 1-8 nodes per workgroup (64-512 threads).  The workgroup size trades
the per-problem constants staged once per workgroup against workgroups
resident per CU (LDS and registers); the sweeps always run one wavefront per
workgroup.  The best size depends on nx, nu, the branching profile and the
precision, so it is measured: every candidate runs a few steps on the actual
problem (or batch) and the fastest is kept, with a JSON cache keyed by GPU
architecture, precision, nx, nu and the tree profile.
"""
from __future__ import annotations

import json
import os

from . import spock as S

CANDIDATES = (64, 128, 256, 512)
_DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2505_12078_amd", "tune.json")


def _arch():
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # noqa: BLE001 - no torch or no device: key on the build target
        return "gfx950"


def problem_key(P, precision):
    z = P.sizes
    return "%s|p%d|nx%d|nu%d|n%d|leaves%d|N%d|ch%d" % (_arch(), precision, z["nx"], z["nu"], z["n"],
                                                      z["n_leaf"], z["N"], z["max_children"])


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, cache):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_problem(P, precision=S.FP64, steps=20, cache_path=_DEFAULT_CACHE, use_cache=True):
    """Pick and set the fastest workgroup size for problem P; returns
    (workgroup, {candidate: ms per step}).  P's iterate is restored."""
    key = problem_key(P, precision)
    cache = _load(cache_path) if cache_path else {}
    if use_cache and key in cache:
        P.set_launch(cache[key]["workgroup"], precision)
        return cache[key]["workgroup"], cache[key]["ms"]
    z, e = P.get_iterate()
    times = {}
    for wg in CANDIDATES:
        try:
            P.set_launch(wg, precision)
        except S.SpockError:
            continue
        P.time_steps(4, precision)  # warm-up (graph-free launches)
        times[wg] = P.time_steps(steps, precision)[0]
    best = min(times, key=times.get)
    P.set_launch(best, precision)
    P.set_iterate(z, e)
    if cache_path:
        cache[key] = {"workgroup": best, "ms": {str(k): v for k, v in times.items()}}
        _store(cache_path, cache)
    return best, times


def tune_batch(B, precision=S.FP32, steps=10):
    """Pick and set the fastest workgroup size for a batch (measured on the
    batch itself); returns (workgroup, {candidate: ms per batched step})."""
    times = {}
    for wg in CANDIDATES:
        try:
            B.set_launch(wg, precision)
        except S.SpockError:
            continue
        B.time_steps(2, precision)
        times[wg] = B.time_steps(steps, precision)[0]
    best = min(times, key=times.get)
    B.set_launch(best, precision)
    return best, times
