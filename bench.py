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


# the paper's A100 throughputs (MLUPS) for the same workloads: tree
# (neighbour-list) RR on the uniform L = 2^13 cavity (Table
# perfo_loss_neighbor_list_rr), DDF numerical equilibrium on the uniform
# L = 2^13 Sod tube (Table perfo_fully_gpu_and_speedup, single precision)
PAPER_A100_MLUPS = {
    ("cavity_uniform", "D2Q9", "fp32"): 10541.0, ("cavity_uniform", "D2Q9", "fp64"): 7041.0,
    ("cavity_uniform", "D2Q13", "fp32"): 5634.0, ("cavity_uniform", "D2Q13", "fp64"): 3452.0,
    ("cavity_uniform", "D2Q21", "fp32"): 3405.0, ("cavity_uniform", "D2Q21", "fp64"): 2140.0,
    ("sod_newton", "D2Q13", "fp32"): 1259.1, ("sod_newton", "D2Q21", "fp32"): 618.5,
    ("sod_newton", "D2Q37", "fp32"): 286.9,
}
SOD_T0 = {"D2Q13": 0.35, "D2Q21": 0.9, "D2Q37": 1.0}


def workload(name, scale, storage, lattice=None):
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
    if name == "vortex":
        # convected vortex, refinement patches that follow it (adaptive runs)
        return W.vortex(n=2048 // scale, levels=3, lattice=lattice or "D2Q9", collision="RR",
                        storage=storage or "fp32")
    if name == "cavity_uniform":
        # uniform L = 2^13 lid-driven cavity, RR
        return W.cavity(n=8192 // scale, levels=1, Re=1000.0, lattice=lattice or "D2Q13", collision="RR",
                        storage=storage or "fp32")
    if name == "sod_newton":
        # uniform L x L Sod tube, L = 2^13 (2^12 for D2Q37, as in the
        # paper), DDF numerical equilibrium
        lat = lattice or "D2Q13"
        L = (4096 if lat == "D2Q37" else 8192) // scale
        return W.sod(nx=L, ny=L, band=False, lattice=lat, collision="DDF_NEWTON",
                     theta=SOD_T0[lat], theta_at="right", storage=storage or "fp32")
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
    if args.lattice:
        cmd += ["--lattice", args.lattice]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"value": None, "unit": "MLUPS", "cores": threads, "kind": "oracle",
                "sample": "failed: " + r.stderr[-300:]}
    d = json.loads(r.stdout.strip().splitlines()[-1])
    d["cores"] = threads
    return d


def cpu_baseline_child(args):
    from oracle.oracle import Oracle
    w = workload(args.workload, args.cpu_scale, None, args.lattice)
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


KERNEL_SOURCES = ["kernels.cuh", "k_d3q27.hip", "lattice.h", "ops.h", "layout.h", "layout.cpp",
                  "grid_builder.h", "grid_builder.cpp"]


def counted_traffic(workload_name, storage):
    """HBM bytes per update of the collide kernel per level, measured with
    rocprofv3 counters and stored in the profile of this kernel and workload;
    None when there is no profile or the kernel's sources changed since."""
    import hashlib
    if workload_name != "sphere" or storage not in ("fp32", "fp16"):
        return None
    prof = os.path.join(ROOT, "profiles", f"k_collide_d3q27_rr_{storage}_sphere.md")
    if not os.path.exists(prof):
        return None
    rec = None
    for line in open(prof):
        line = line.strip()
        if line.startswith("traffic {"):
            rec = json.loads(line[len("traffic "):])
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2504_04465_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return {int(k): v for k, v in rec["bytes_per_update"].items()}


def neighbour_list_bytes_per_update(w, storage):
    """algorithmic bytes one cell update moves under the neighbour-list
    formulation of the method (V - 1 int32 neighbour links per cell, Sec. 4.4 data
    layout; the tree-grid performance model of Sec. 6.3): read and write the Q
    populations of every distribution in the storage precision, read the
    Q - 1 int32 pull indices, and read and write the eight multipliers
    where they are kept for the warm start"""
    from paper_2504_04465_amd.lbm import LATTICE_Q
    q = LATTICE_Q[w.lattice]
    s = {"fp64": 8, "fp32": 4, "fp16": 2}[storage]
    dists = 2 if w.collision.startswith("DDF") else 1
    lam = 2 * 8 * (8 if storage == "fp64" else 4) if w.collision in ("DDF_NEWTON", "DDF_MLP_NEWTON") else 0
    return 2 * q * s * dists + 4 * (q - 1) + lam


def rel_l2(a, b, vol):
    """volume-weighted relative L2 of a against b over the cells where both
    are finite (fine ghosts are NaN)"""
    import numpy as np
    vol = np.broadcast_to(vol, a.shape)
    ok = np.isfinite(a) & np.isfinite(b)
    den = np.sqrt(np.sum(vol[ok] * b[ok] ** 2))
    return float(np.sqrt(np.sum(vol[ok] * (a[ok] - b[ok]) ** 2)) / den) if den > 0 else 0.0


def surrogate_leg(args):
    """D2Q21 numerical-equilibrium step (supersonic airfoil) with the Newton
    solve, cold and warm started, against the multiplier surrogate alone and
    with one Newton correction plus Newton fallback.  All variants start from
    the same developed flow; errors are against the FP64-storage Newton path
    from the same state (the GPU path the parity tests tie to the oracle)."""
    import numpy as np
    import torch
    from paper_2504_04465_amd import lbm as B
    from paper_2504_04465_amd import workloads as W
    K, dev = args.sur_steps, args.sur_develop
    w = W.airfoil(scale=args.sur_scale, steps=dev + K + 2)
    t_all = time.perf_counter()

    def ctx(coll, sto, warm):
        c = B.LBM(w.lattice, coll, sto, nu_finest=w.nu_finest, T0=w.T0, gamma=w.gamma, sensor_A=w.sensor_A,
                  sensor_on=w.sensor_on, newton_tol=w.newton_tol, newton_max_it=w.newton_max_it, warm_start=warm)
        c.grid(w.dim, w.ext, w.n_levels, w.refine, w.solid, w.faces)
        return c

    def faces(c, k):
        for face, f in w.schedule(k).items():
            c.set_face(face, f)

    # training set: Newton labels of seeded states from the training box
    lab = ctx("DDF_NEWTON", "fp32", True)
    x = W.mlp_samples(args.sur_samples, seed=5)
    t0 = time.perf_counter()
    lam, ok, _ = lab.mlp_label(x)
    t1 = time.perf_counter()
    hist = lab.mlp_train(x[ok], lam[ok], epochs=args.sur_epochs, batch=1024, lr=1e-2, seed=5)
    t2 = time.perf_counter()
    wts = lab.mlp_get_weights()
    lab.close()
    # developed flow
    d = ctx("DDF_NEWTON", "fp32", True)
    d.init_workload(w)
    for k in range(dev):
        faces(d, k)
        d.step(1)
    d.sync()
    state = d.get_state()
    _, level = d.coords_levels()
    vol = np.ldexp(1.0, -2 * level.astype(np.int64))
    n_cells = d.n
    d.close()

    def run(coll, sto, warm):
        c = ctx(coll, sto, warm)
        if coll != "DDF_NEWTON":
            c.mlp_set_weights(wts)
        c.set_state(*state)
        for k in range(dev, dev + 2):
            faces(c, k)
            c.step(1)
        c.sync()
        s0 = c.stats()
        torch.cuda.synchronize()
        c.profile(True)
        ta = time.perf_counter()
        for k in range(dev + 2, dev + 2 + K):
            faces(c, k)
            c.step(1)
        diverged = None
        try:
            c.sync()
        except B.LbmError as e:  # a numeric failure latched during the timed steps
            if e.code != -6:
                raise
            diverged = str(e)[:160]
        torch.cuda.synchronize()
        wall = (time.perf_counter() - ta) * 1e3
        coll_ms = sum(c.profile_read(l)[1] for l in range(w.n_levels))
        res = {"step_ms": round(wall / K, 3), "collide_ms": round(coll_ms / K, 3)}
        if diverged is not None:
            c.close()
            res["failed"] = diverged
            return res, None
        s1 = c.stats()
        m = c.moments()
        c.close()
        upd = sum(s1["updates"]) - sum(s0["updates"])
        it = s1["newton_iterations"] - s0["newton_iterations"]
        fb = s1["mlp_fallbacks"] - s0["mlp_fallbacks"]
        res.update({"newton_it_per_update": round(it / max(upd, 1), 3),
                    "fallback_rate": round(fb / max(upd, 1), 4)})
        return res, m

    ref_stats, ref = run("DDF_NEWTON", "fp64", True)
    out = {"workload": f"airfoil D2Q21 numerical equilibrium, {w.ext[0]}x{w.ext[1]} coarse, {w.n_levels} levels, "
                       f"{n_cells} cells, fp32 populations, FP64 Newton",
           "developed_coarse_steps": dev, "timed_coarse_steps": K,
           "training": {"samples_drawn": int(len(x)), "accepted": int(ok.sum()), "epochs": args.sur_epochs,
                        "label_s": round(t1 - t0, 3), "train_s": round(t2 - t1, 3),
                        "loss_first_last": [float(hist[0]), float(hist[-1])]},
           "reference": dict(ref_stats, storage="fp64", warm_start=True)}
    def errs(m, r):
        return {"rho": rel_l2(m[0], r[0], vol), "u": rel_l2(m[1:3], r[1:3], vol[None, :]),
                "T": rel_l2(m[3], r[3], vol)}

    cold = None
    for name, coll, warm in [("a_cold", "DDF_NEWTON", False), ("a_warm", "DDF_NEWTON", True),
                             ("b_mlp", "DDF_MLP", True), ("c_mlp_newton", "DDF_MLP_NEWTON", True)]:
        try:
            st, m = run(coll, "fp32", warm)
            if m is not None:
                st["rel_l2_vs_fp64"] = errs(m, ref)
                # against Newton at the same storage precision (cold start):
                # what replacing the solve changes, without the FP32 rounding
                # both share
                if cold is None:
                    cold = m
                else:
                    st["rel_l2_vs_a_cold"] = errs(m, cold)
        except B.LbmError as e:
            st = {"failed": str(e)[:160]}
        out[name] = st
        print(f"[bench] surrogate {name}: {st}", file=sys.stderr, flush=True)
    # the floor of variant (c) from the measured variants: the cost of one
    # Newton step per update (cold minus warm over their step counts), the
    # collide without any Newton step (warm minus its steps), the network
    # (MLP alone minus that base), and (c) at zero fallback = base + one
    # step + network
    ac, aw, bm = out["a_cold"], out["a_warm"], out["b_mlp"]
    if "collide_ms" in ac and "collide_ms" in aw and ac["newton_it_per_update"] > aw["newton_it_per_update"]:
        step = (ac["collide_ms"] - aw["collide_ms"]) / (ac["newton_it_per_update"] - aw["newton_it_per_update"])
        base = aw["collide_ms"] - step * aw["newton_it_per_update"]
        fl = {"newton_step_ms": round(step, 3), "base_ms": round(base, 3)}
        if "collide_ms" in bm:
            mlp = bm["collide_ms"] - base
            floor_c = base + step + mlp
            fl.update({"mlp_ms": round(mlp, 3), "c_at_zero_fallback_ms": round(floor_c, 3),
                       "max_speedup_vs_a_cold": round(ac["collide_ms"] / floor_c, 3),
                       "max_speedup_vs_a_warm": round(aw["collide_ms"] / floor_c, 3)})
        out["floor"] = fl
    c = out["c_mlp_newton"]
    if "step_ms" in c:
        out["speedup_c_vs_a_cold"] = {"step": round(out["a_cold"]["step_ms"] / c["step_ms"], 3),
                                      "collide": round(out["a_cold"]["collide_ms"] / c["collide_ms"], 3)}
        out["speedup_c_vs_a_warm"] = {"step": round(out["a_warm"]["step_ms"] / c["step_ms"], 3),
                                      "collide": round(out["a_warm"]["collide_ms"] / c["collide_ms"], 3)}
    out["seconds"] = round(time.perf_counter() - t_all, 1)
    return out


def fp16_leg(w32, args):
    """The same workload with FP16 populations (f - w_i stored, FP32
    collisions): MLUPS and the collide kernel's algorithmic HBM rate."""
    import torch
    from paper_2504_04465_amd import lbm as B
    from paper_2504_04465_amd import workloads as W
    w = W.sphere(scale=args.scale, storage="fp16")
    s = B.LBM.from_workload(w, storage="fp16")
    s.init_workload(w)
    s.step(args.warmup)
    s.sync()
    torch.cuda.synchronize()
    s.profile(True)
    t0 = time.perf_counter()
    s.step(args.steps)
    s.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    L = s.n_levels
    per_step = sum(int(n) << l for l, n in enumerate(s.n_per_level))
    tb = tm = 0.0
    ups = 0
    counted = counted_traffic(w.name, "fp16")
    ctb = 0.0
    for l in range(L):
        n_l, ms_l, bpu = s.profile_read(l)
        tb += bpu * int(s.n_per_level[l]) * n_l
        tm += ms_l
        ups += int(s.n_per_level[l]) * n_l
        if counted is not None:
            ctb += counted[l] * int(s.n_per_level[l]) * n_l
    s.close()
    traffic = round(ctb / (tm * 1e-3) / 1e9, 1) if counted is not None and tm > 0 else None
    lay = tb / (tm * 1e-3) / 1e9 if tm > 0 else 0.0
    sbpu = neighbour_list_bytes_per_update(w, "fp16")
    ach = sbpu * ups / (tm * 1e-3) / 1e9 if tm > 0 else 0.0
    return {"value": round(per_step * args.steps / dt / 1e6, 2), "unit": "MLUPS",
            "ms_per_step": round(dt / args.steps * 1e3, 4),
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_update": sbpu,
                         "layout_bytes_per_update": round(tb / max(ups, 1), 2),
                         "layout_achieved": round(lay, 1), "layout_frac": round(lay / HBM_PEAK_GBS, 4),
                         "traffic": traffic,
                         "traffic_frac": round(traffic / HBM_PEAK_GBS, 4) if traffic is not None else None,
                         "traffic_bytes_per_update": round(ctb / max(ups, 1), 1) if counted is not None else None}}


def calibrate_copy():
    """A plain copy of exactly 1 GiB (read 1 GiB, write 1 GiB) on the device:
    under rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE it gives the factor between
    the counters and the bytes moved."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)  # device-to-device copy
    torch.cuda.synchronize()
    torch.mul(a, 2.0, out=b)  # elementwise kernel: read 1 GiB, write 1 GiB
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 4 * n, "ok": bool(b[-1].item() == 2.0)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sphere")
    ap.add_argument("--storage", default=None)
    ap.add_argument("--lattice", default=None, help="lattice of the cavity_uniform / sod_newton workloads")
    ap.add_argument("--in-place", action="store_true",
                    help="stream in place on one population buffer (single-level workloads)")
    ap.add_argument("--scale", type=int, default=1)
    ap.add_argument("--cpu-scale", type=int, default=4)
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--no-graphs", action="store_true",
                    help="time kernel launches instead of pairs of coarse steps replayed from a HIP graph "
                         "(the roofline always comes from a profiled, launched run of the same steps)")
    ap.add_argument("--no-fusion", action="store_true",
                    help="launch each level's collide on its own instead of one launch per substep")
    ap.add_argument("--sur-scale", type=int, default=1)
    ap.add_argument("--sur-steps", type=int, default=20)
    ap.add_argument("--sur-develop", type=int, default=260,
                    help="coarse steps before the timed ones: the Mach ramp ends at 200")
    ap.add_argument("--sur-samples", type=int, default=3_300_000)
    ap.add_argument("--sur-epochs", type=int, default=40)
    ap.add_argument("--surrogate-only", action="store_true",
                    help="run only the surrogate leg and print its JSON object")
    ap.add_argument("--cpu-baseline-child", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="one plain 1 GiB device-to-device copy, to scale the HBM byte counters")
    args = ap.parse_args()
    if args.cpu_baseline_child:
        cpu_baseline_child(args)
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.surrogate_only:
        print(json.dumps({"surrogate": surrogate_leg(args)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_04465_amd import lbm as B

    w = workload(args.workload, args.scale, args.storage, args.lattice)
    storage = args.storage or w.storage
    t0 = time.perf_counter()
    torch.cuda.reset_peak_memory_stats()
    s = B.LBM.from_workload(w, storage=storage, in_place=args.in_place)
    # the grid build's temporaries (dense level boxes, sort keys) peak above
    # what the simulation then holds: counted apart
    build_peak_gb = torch.cuda.max_memory_allocated() / 1e9
    torch.cuda.reset_peak_memory_stats()
    if args.no_fusion:
        s.level_fusion(False)
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
    dt_graph = None
    if not args.no_graphs and w.schedule is None:
        s.graphs(True)
        advance(2)
        s.sync()
        t0 = time.perf_counter()
        advance(args.steps)
        s.sync()
        torch.cuda.synchronize()
        dt_graph = time.perf_counter() - t0
        s.graphs(False)
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
    mlups = per_step * args.steps / (dt_graph if dt_graph is not None else dt) / 1e6
    # roofline of the collide-and-stream kernel, from HIP events around every
    # launch of the timed region: algorithmic bytes / kernel time
    tot_bytes, tot_ms, launches = 0.0, 0.0, 0
    for l in range(L):
        n_l, ms_l, bpu = s.profile_read(l)
        tot_bytes += bpu * int(s.n_per_level[l]) * n_l
        tot_ms += ms_l
        launches += n_l
    layout_rate = tot_bytes / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
    n_upd = sum(int(s.n_per_level[l]) * s.profile_read(l)[0] for l in range(L))
    # achieved: the method's algorithmic bytes (neighbour-list formulation)
    # per update x the updates of the timed launches / their summed duration
    sbpu = neighbour_list_bytes_per_update(w, storage)
    achieved = sbpu * n_upd / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
    _, _, bpu_f = s.profile_read(L - 1)
    # counter-measured HBM bytes of the same launches, at the same rate basis
    counted = counted_traffic(w.name, storage)
    traffic = traffic_bpu = None
    if counted is not None and tot_ms > 0:
        tb = sum(counted[l] * int(s.n_per_level[l]) * s.profile_read(l)[0] for l in range(L))
        traffic = round(tb / (tot_ms * 1e-3) / 1e9, 1)
        traffic_bpu = round(tb / sum(int(s.n_per_level[l]) * s.profile_read(l)[0] for l in range(L)), 1)
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round((dt_graph if dt_graph is not None else dt) / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": (round(mlups / PAPER_A100_MLUPS[(args.workload, w.lattice, storage)], 3)
                        if args.scale == 1 and (args.workload, w.lattice, storage) in PAPER_A100_MLUPS else None),
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f16-storage/f32-compute"}[storage],
        "data": "synthetic",
        "config": {"workload": describe(w, storage), "cells": int(s.n),
                   "cells_per_level": [int(x) for x in s.n_per_level],
                   "updates_per_coarse_step": per_step,
                   "equivalent_fine_cells": s.eq_fine},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_frac": round(traffic / HBM_PEAK_GBS, 4) if traffic is not None else None,
                     "kernel": "k_collide", "launches": launches,
                     "avg_launch_ms": round(tot_ms / max(launches, 1), 5),
                     "bytes_per_update": sbpu,
                     "layout_bytes_per_update": round(tot_bytes / max(n_upd, 1), 2),
                     "layout_achieved": round(layout_rate, 1),
                     "layout_frac": round(layout_rate / HBM_PEAK_GBS, 4),
                     "traffic_bytes_per_update": traffic_bpu},
        "modeled_hbm_frac_whole_step": round(per_step * bpu_f * args.steps / dt / 1e9 / HBM_PEAK_GBS, 4),
        "mlups_paper_formula": round(s.n * args.steps * (1 << (L - 1)) / (dt_graph or dt) / 1e6, 2),
        "launch": ("HIP graph per pair of coarse steps" if dt_graph is not None else "kernel launches")
                  + ("" if args.no_fusion else ", concurrent levels in one collide launch per substep"),
        "paper_a100_mlups": PAPER_A100_MLUPS.get((args.workload, w.lattice, storage)) if args.scale == 1 else None,
        "streaming": "in place, one buffer" if args.in_place else "two buffers",
        "device_memory_gb": round(torch.cuda.max_memory_allocated() / 1e9, 2),
        "grid_build_peak_gb": round(build_peak_gb, 2),
        "newton": {"calls": st["newton_calls"], "iterations": st["newton_iterations"],
                   "failures": st["newton_failures"]},
    }
    if args.workload == "vortex":
        # mesh adaptation: patches moved by 1/64 of the box per remesh
        times = []
        for k in range(1, 4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.remesh(w.patch(k * w.ext[0] / 64 / 0.05))
            s.sync()
            times.append((time.perf_counter() - t0) * 1e3)
            s.step(1)
        out["remesh"] = {"ms": [round(t, 1) for t in times], "cells_after": int(s.n),
                         "note": "tree, layout and source lists built on the device, state moved on the device"}
    s.close()
    if args.workload == "sphere" and storage == "fp32" and not args.no_fp16:
        out["fp16_storage"] = fp16_leg(w, args)
    if not args.no_surrogate:
        out["surrogate"] = surrogate_leg(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
