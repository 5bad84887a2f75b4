#!/usr/bin/env python3
"""Throughput of the colour-gradient D2Q9 step on one MI355X.

Default workload: the static-bubble sweep -- nine 512 x 512 periodic lattices
(density ratio gamma in {10, 100, 1000} x dynamic-viscosity ratio M in
{1, 10, 100}, seeded radii 64..128, sigma = 4.444e-4, beta = 0.7, FP32), all
advanced by one batched kernel launch per time step.  A "step" is one time
step of all nine lattices.  Inputs are synthetic and seeded; populations are
resident in HBM before the timed region starts.

Prints ONE JSON line: MLUPS (whole job), the roofline of the step kernel
(algorithmic bytes 144 B per lattice update in FP32 -- 18 populations read and
written -- or 72 B with 16-bit storage, against 8 TB/s), the FP64 CPU oracle
timed on a bounded sample on the host cores, and per-lattice diagnostics.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1903_01168_amd", "csrc", f)
                  for f in ("cg_device.hpp", "cg_kernels.hip")]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def bytes_per_update(storage):
    return 144 if storage == "f32" else 72


def build_cells(args, W):
    if args.workload == "sweep512":
        return W.bubble_sweep(seed=args.seed, n=512, storage=args.storage, collision=args.collision), \
            "static-bubble sweep 512x512 x 9 cells (gamma x M)"
    if args.workload == "bubble64":
        return [W.static_bubble(storage=args.storage, collision=args.collision)], "static bubble 64x64"
    if args.workload == "slug":
        c = W.gravity_slug(seed=args.seed, gamma=10, Re=10, storage=args.storage, collision=args.collision)
        return [c], "gravity slug 4096x256"
    if args.workload == "channel":
        c = W.inlet_outlet(seed=args.seed, storage=args.storage, collision=args.collision)
        return [c], "inlet/outlet channel 8192x512"
    if args.workload == "hbm8192":
        c = W.static_bubble(n=8192, radius=2048.0, storage=args.storage, collision=args.collision)
        return [c], "static bubble 8192x8192"
    raise SystemExit(f"unknown workload {args.workload}")


def laplace(lat, cell):
    """Laplace-law error of a bubble cell from FP64 device reductions."""
    d0 = lat.diag(check=False)
    if d0["n_nonfinite"] > 0:
        return dict(stable=False, n_nonfinite=d0["n_nonfinite"])
    R = math.sqrt(d0["area_r"] / math.pi)
    cx, cy = cell["center"]
    d = lat.diag(circle=(cx, cy, R - 4.0, R + 4.0), check=False)
    p = cell["params"]
    if p["sigma"] > 0:
        sigma = p["sigma"]
    else:
        sigma = 4.0 * p["A"] / (9.0 * (1.0 / p["tau_r"]))
    dp = d["p_in"] - d["p_out"]
    return dict(stable=True, R=R, dp=dp, dp_theory=sigma / R, laplace_err=abs(dp / (sigma / R) - 1.0),
                max_u=d["max_u"], mass_r=d["mass_r"], mass_b=d["mass_b"])


def cpu_baseline(cell, seconds):
    """The FP64 oracle on one lattice of the workload, on the host cores."""
    import oracle
    p = dict(cell["params"])
    s = oracle.Sim(**p).init(cell["rho_r"], cell["rho_b"], cell["ux"], cell["uy"])
    t0 = time.perf_counter()
    s.step(1)
    t1 = time.perf_counter() - t0
    steps = max(1, min(2000, int(seconds / max(t1, 1e-6))))
    t0 = time.perf_counter()
    s.step(steps)
    dt = time.perf_counter() - t0
    nodes = p["nx"] * p["ny"]
    return dict(value=nodes * steps / dt / 1e6, unit="MLUPS", cores=oracle.threads(), kind="oracle",
                sample=f"{p['nx']}x{p['ny']} lattice ({cell['name']}), {steps} steps, FP64, "
                       f"{dt:.1f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="sweep512")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16s", "bf16s"])
    ap.add_argument("--collision", default="bgk", choices=["bgk", "mrt"])
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--strip", type=int, default=0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-only", type=float, default=0.0,
                    help="only time the plain copy kernel over this many GiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1903_01168_amd import capi
    from paper_1903_01168_amd import workloads as W

    capi.load()
    torch.cuda.init()
    stream = torch.cuda.Stream()           # default priority
    sid = stream.cuda_stream

    if args.copy_only > 0:
        n = int(args.copy_only * (1 << 30))
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty(n, dtype=torch.uint8, device="cuda")
        probe = capi.Lattice(W.params(nx=64, ny=64, A=1e-3), stream=sid)
        for _ in range(3):
            probe.bw_copy(b.data_ptr(), a.data_ptr(), n)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record(stream)
        for _ in range(reps):
            probe.bw_copy(b.data_ptr(), a.data_ptr(), n)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps({"copy_bytes": n, "copy_ms": ms, "copy_gbs": 2 * n / ms / 1e6}))
        return

    cells, wname = build_cells(args, W)
    lats = []
    for c in cells:
        lat = capi.Lattice(c["params"], stream=sid)
        if args.strip or args.tile:
            lat.set_launch(args.tile, args.strip)
        lat.init(c["rho_r"], c["rho_b"], c["ux"], c["uy"])
        if "schedule" in c:
            lat.set_inlet_color(np.full(c["params"]["ny"], c["schedule"][0][1], dtype=np.int8))
        lats.append(lat)
    mass0 = [lat.diag(check=False) for lat in lats]
    batch = capi.Batch(lats, tile_x=args.tile, stream=sid)
    nodes = sum(c["params"]["nx"] * c["params"]["ny"] for c in cells)

    batch.step(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    batch.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / max(args.steps, 1)
    mlups = nodes * args.steps / (ms / 1e3) / 1e6

    bpu = bytes_per_update(args.storage)
    achieved = bpu * nodes / (ms_per_step / 1e3) / 1e9   # GB/s of one launch (one step)
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        try:
            tr = json.load(open(TRAFFIC_FILE))
            key = f"{args.workload}/{args.storage}/{args.collision}"
            if tr.get("kernel_hash") == kernel_hash() and key in tr.get("per_launch", {}):
                traffic = tr["per_launch"][key]
        except (OSError, ValueError):
            traffic = None

    cells_out = []
    for lat, c, m0 in zip(lats, cells, mass0):
        info = dict(name=c["name"])
        if "center" in c:
            info.update(laplace(lat, c))
        d = lat.diag(check=False)
        info["mass_drift_r"] = (d["mass_r"] - m0["mass_r"]) / m0["mass_r"] if m0["mass_r"] else 0.0
        info["mass_drift_b"] = (d["mass_b"] - m0["mass_b"]) / m0["mass_b"] if m0["mass_b"] else 0.0
        info["n_nonfinite"] = d["n_nonfinite"]
        cells_out.append(info)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cells[0], args.cpu_seconds)

    p0 = cells[0]["params"]
    out = {
        "metric": "MLUPS & HBM GB/s (% of peak), color-gradient D2Q9; p50/p99 solve latency",
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else f"f32 arithmetic, {args.storage} storage",
        "data": "synthetic (seeded)",
        "config": {"workload": wname, "lattices": len(cells), "nx": p0["nx"], "ny": p0["ny"],
                   "nodes": nodes, "storage": args.storage, "collision": args.collision,
                   "steps_simulated": args.warmup + args.steps, "seed": args.seed,
                   "launch": "one batched k_step launch per step, HIP-graph replay of 32 steps"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_update": bpu, "kernel": "k_step", "kernel_hash": kernel_hash()},
        "cpu_baseline": cpu,
        "wall_s": wall,
        "cells": cells_out,
    }
    print(json.dumps(out))
    batch.close()
    for lat in lats:
        lat.close()


if __name__ == "__main__":
    main()
