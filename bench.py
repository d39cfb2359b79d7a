#!/usr/bin/env python3
"""Benchmark of the refined-grid lattice Boltzmann step on one MI355X.

Default workload: flow past a sphere, D3Q27 recursive regularisation with
FP32 populations, 512 x 256 x 256 coarse cells and three octree levels
(~65.8 M cells, 129 M cell updates per coarse step), synthetic seeded input.
A step is one coarse step: 2^(L-1) finest substeps with every level updated
at its own rate (Sec. 4.5).

Prints one JSON line: MLUPS (actual cell updates per second, inputs resident
in HBM), the HBM roofline of the collide-and-stream kernel measured live with
HIP events, and the FP64 CPU oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM peak; surrogate vs Newton equilibrium speedup at rel-L2≤1e-5"
HBM_PEAK_GBS = 8000.0


def workload(name, scale, storage):
    from paper_2504_04465_amd import workloads as W
    if name == "sphere":
        return W.sphere(scale=scale, storage=storage or "fp32")
    if name == "cylinder":
        return W.cylinder(scale=scale, storage=storage or "fp32")
    if name == "cavity":
        return W.cavity(n=64 // scale)
    if name == "sod":
        return W.sod(nx=4096 // scale, storage=storage or "fp32")
    if name == "airfoil":
        return W.airfoil(scale=scale, storage=storage or "fp32")
    raise SystemExit(f"unknown workload {name}")


def describe(w, storage):
    ext = "x".join(str(e) for e in w.ext)
    return f"{w.name}: {w.lattice}-{w.collision}, {ext} coarse cells, {w.n_levels} levels, {storage} populations"


def cpu_baseline(args):
    """time the FP64 oracle on a bounded sample of the same workload, in a
    child process so that OMP_NUM_THREADS takes effect"""
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    threads = max(1, min(16, ncpu))
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", "--workload", args.workload,
           "--cpu-scale", str(args.cpu_scale), "--cpu-steps", str(args.cpu_steps)]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"value": None, "unit": "MLUPS", "cores": threads, "kind": "oracle",
                "sample": "failed: " + r.stderr[-300:]}
    d = json.loads(r.stdout.strip().splitlines()[-1])
    d["cores"] = threads
    return d


def cpu_baseline_child(args):
    from oracle.oracle import Oracle
    w = workload(args.workload, args.cpu_scale, None)
    o = Oracle.from_workload(w)
    o.init_workload(w)
    npl = o.level_counts()
    per_step = sum(int(n) << l for l, n in enumerate(npl))
    t0 = time.perf_counter()
    o.step(args.cpu_steps)
    dt = time.perf_counter() - t0
    print(json.dumps({"value": per_step * args.cpu_steps / dt / 1e6, "unit": "MLUPS", "kind": "oracle",
                      "sample": f"{describe(w, 'fp64')} (1/{args.cpu_scale} scale per axis), "
                                f"{args.cpu_steps} coarse steps, {per_step * args.cpu_steps} updates, "
                                f"{dt:.1f} s"}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sphere")
    ap.add_argument("--storage", default=None)
    ap.add_argument("--scale", type=int, default=1)
    ap.add_argument("--cpu-scale", type=int, default=4)
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-child", action="store_true")
    args = ap.parse_args()
    if args.cpu_baseline_child:
        cpu_baseline_child(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_04465_amd import lbm as B

    w = workload(args.workload, args.scale, args.storage)
    storage = args.storage or w.storage
    t0 = time.perf_counter()
    s = B.LBM.from_workload(w, storage=storage)
    t_build = time.perf_counter() - t0
    s.init_workload(w)
    print(f"[bench] {describe(w, storage)}: {s.n} cells {list(s.n_per_level)}, grid {t_build:.1f} s",
          file=sys.stderr, flush=True)
    step = 0

    def advance(k):
        nonlocal step
        if w.schedule is None:
            s.step(k)
            step += k
            return
        for _ in range(k):
            for face, f in w.schedule(step).items():
                s.set_face(face, f)
            s.step(1)
            step += 1

    advance(args.warmup)
    s.sync()
    torch.cuda.synchronize()
    s.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    advance(args.steps)
    s.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.profile(False)
    st = s.stats()
    L = s.n_levels
    per_step = sum(int(n) << l for l, n in enumerate(s.n_per_level))
    mlups = per_step * args.steps / dt / 1e6
    # roofline of the collide-and-stream kernel, from HIP events around every
    # launch of the timed region: algorithmic bytes / kernel time
    tot_bytes, tot_ms, launches = 0.0, 0.0, 0
    for l in range(L):
        n_l, ms_l, bpu = s.profile_read(l)
        tot_bytes += bpu * int(s.n_per_level[l]) * n_l
        tot_ms += ms_l
        launches += n_l
    achieved = tot_bytes / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
    _, _, bpu_f = s.profile_read(L - 1)
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f16-storage/f32-compute"}[storage],
        "data": "synthetic",
        "config": {"workload": describe(w, storage), "cells": int(s.n),
                   "cells_per_level": [int(x) for x in s.n_per_level],
                   "updates_per_coarse_step": per_step,
                   "equivalent_fine_cells": s.eq_fine},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_collide", "launches": launches,
                     "avg_launch_ms": round(tot_ms / max(launches, 1), 5),
                     "bytes_per_update": bpu_f},
        "modeled_hbm_frac_whole_step": round(per_step * bpu_f * args.steps / dt / 1e9 / HBM_PEAK_GBS, 4),
        "mlups_paper_formula": round(s.n * args.steps * (1 << (L - 1)) / dt / 1e6, 2),
        "newton": {"calls": st["newton_calls"], "iterations": st["newton_iterations"],
                   "failures": st["newton_failures"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
