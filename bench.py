#!/usr/bin/env python3
"""Throughput of the colour-gradient D2Q9 step on one MI355X.

Default workload: the inlet/outlet channel, 8192 x 512 nodes in FP32 -- the
largest single-GPU configuration and the one whose populations (604 MB, both
buffers) live in HBM rather than in the 256 MB Infinity Cache: a velocity
inlet, a pressure outlet and free-slip walls, heavy liquid below light gas
(density ratio 5, mu_g = mu_l / 2) entering at u = 0.01 with volume fractions
0.8 / 0.2 (the paper's open-channel set-up of Sec. 5.2; its density-ratio-100
alternating-injection recipe goes non-finite in the FP64 oracle within a few
hundred steps, see the design notes).  A "step" is one time step of the
lattice, one kernel launch.  Inputs are synthetic and seeded; populations are
resident in HBM before the timed region starts.

Prints ONE JSON line: MLUPS, the roofline of the step kernel (algorithmic
bytes 144 B per lattice update in FP32 -- 18 populations read and written --
or 80 B with 16-bit storage, where the 16 moving populations take 2 B and the
two rest populations 4 B, against 8 TB/s), the FP64 CPU oracle timed on a
bounded sample on the host cores, the cache-resident nine-lattice sweep as a
secondary figure, a plain copy's rate for context, and the storage-precision
report of a converged bubble against the FP64 oracle.
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
# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction
VALU_PEAK_GIPS = 256 * 4 * 2.4 / 4   # 614.4 G wave64 VALU instructions/s
# the kernels and the host planner that picks their launch shape
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1903_01168_amd", "csrc", f)
                  for f in ("cg_device.hpp", "cg_kernels.hip", "cg_capi.cpp", "cg_schedule.hpp")]


def code_text(src):
    """C++ source with its comments and blank lines removed and each run of
    whitespace in a line made one space: what the compiler sees, so that an
    edit of a comment leaves the kernel's identity (and the traffic measured
    for it) unchanged."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":                                   # string or character literal
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return "\n".join(" ".join(ln.split()) for ln in "".join(out).splitlines() if ln.strip())


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def bytes_per_update(storage):
    return 144 if storage == "f32" else 80


def build_cells(args, W):
    if args.workload == "channel":
        c = W.inlet_outlet(seed=args.seed, storage=args.storage, collision=args.collision)
        return [c], ("inlet/outlet channel 8192x512 (Sec. 5.2 open channel: velocity inlet, pressure outlet, "
                     "free-slip walls, stratified inflow, density ratio 5)")
    if args.workload == "sweep512":
        return W.bubble_sweep(seed=args.seed, n=512, storage=args.storage, collision=args.collision), \
            "static-bubble sweep 512x512 x 9 cells (gamma x M)"
    if args.workload == "bubble64":
        return [W.static_bubble(storage=args.storage, collision=args.collision)], "static bubble 64x64"
    if args.workload == "slug":
        c = W.gravity_slug(seed=args.seed, gamma=10, Re=10, storage=args.storage, collision=args.collision)
        return [c], "gravity slug 4096x256"
    if args.workload == "hbm8192":
        c = W.static_bubble(n=8192, radius=2048.0, storage=args.storage, collision=args.collision)
        return [c], "static bubble 8192x8192"
    raise SystemExit(f"unknown workload {args.workload}")


def measure(capi, torch, stream, cells, steps, warmup, tile, strip):
    """Time `steps` batched steps of the lattices of `cells` after `warmup`
    untimed ones, with HIP events on the batch's stream."""
    import numpy as np
    sid = stream.cuda_stream
    lats = []
    for c in cells:
        lat = capi.Lattice(c["params"], stream=sid)
        if strip or tile:
            lat.set_launch(tile, strip)
        lat.init(c["rho_r"], c["rho_b"], c["ux"], c["uy"])
        if "inlet_color" in c:
            lat.set_inlet_color(c["inlet_color"])
        elif "schedule" in c:
            lat.set_inlet_color(np.full(c["params"]["ny"], c["schedule"][0][1], dtype=np.int8))
        lats.append(lat)
    batch = capi.Batch(lats, tile_x=tile, stream=sid)
    launches = batch.groups
    plans = [batch.group_launch(g) for g in range(launches)]
    nodes = sum(c["params"]["nx"] * c["params"]["ny"] for c in cells)
    nbytes = sum(2 * lat.buffer_bytes for lat in lats)
    batch.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    batch.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    state = []
    for lat in lats:
        d = lat.diag(check=False)
        state.append(dict(n_nonfinite=d["n_nonfinite"], max_u=d["max_u"]))
    batch.close()
    for lat in lats:
        lat.close()
    flav = sorted({"block exchange" if x else "halo lanes" for _, x in plans})
    launch = (f"k_step, {launches} launches per step ({', '.join(flav)}; groups of lattices sized for the Infinity "
              f"Cache, two in flight on two streams), HIP-graph replay of 32 steps" if launches > 1 else
              f"k_step ({flav[0]}, {plans[0][0]} threads per workgroup), one launch per step, HIP-graph replay "
              f"of 32 steps")
    return dict(mlups=nodes * steps / (ms / 1e3) / 1e6, ms_per_step=ms / max(steps, 1), launches=launches,
                nodes=nodes, bytes=nbytes, wall=wall, state=state, flavour=", ".join(flav), launch=launch)


def copy_rate(capi, W, torch, stream, gib):
    """A plain device copy of `gib` GiB (the library's copy kernel): the
    achievable bandwidth beside the 8 TB/s spec, and the calibration of the
    traffic counters."""
    n = int(gib * (1 << 30))
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    probe = capi.Lattice(W.params(nx=64, ny=64, A=1e-3), stream=stream.cuda_stream)
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
    probe.close()
    ms = e0.elapsed_time(e1) / reps
    return {"copy_bytes": n, "copy_ms": ms, "copy_gbs": 2 * n / ms / 1e6}


def stored_counters(args):
    """HBM bytes per launch and VALU instructions per lattice update from the
    rocprofv3 counter runs summarised under profiles/, while the kernel
    sources are the ones those runs measured (else None)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, None
    try:
        tr = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None, None
    if tr.get("kernel_hash") != kernel_hash():
        return None, None
    key = (f"{args.workload}/{args.storage}/{args.collision}" + ("/nsc" if args.ns_correction else "")
           + ("/iso" if args.gradient == "isotropic" else ""))
    return tr.get("per_launch", {}).get(key), tr.get("valu_per_update", {}).get(key)


def cpu_baseline(cell, seconds, steps_cap=2000):
    """The FP64 oracle on one lattice of the workload, on the host cores."""
    import oracle
    p = dict(cell["params"])
    s = oracle.Sim(**p).init(cell["rho_r"], cell["rho_b"], cell["ux"], cell["uy"])
    if "inlet_color" in cell:
        s.set_inlet_color(cell["inlet_color"])
    t0 = time.perf_counter()
    s.step(1)
    t1 = time.perf_counter() - t0
    steps = max(1, min(steps_cap, int(seconds / max(t1, 1e-6))))
    t0 = time.perf_counter()
    s.step(steps)
    dt = time.perf_counter() - t0
    nodes = p["nx"] * p["ny"]
    return dict(value=nodes * steps / dt / 1e6, unit="MLUPS", cores=oracle.threads(), kind="oracle",
                sample=f"{p['nx']}x{p['ny']} lattice ({cell['name']}), {steps} steps, FP64, "
                       f"{dt:.1f} s")


def precision_report(sid, steps=20000):
    """Converged 64 x 64 static bubble (R = 16, A = 1e-3, beta = 0.7): the
    pressure jump and colour-mass drift of each storage format against the FP64
    oracle (run on the host cores here)."""
    import numpy as np
    import oracle
    from paper_1903_01168_amd import capi
    from paper_1903_01168_amd import workloads as W
    c = W.static_bubble(n=64, radius=16)
    p = c["params"]
    s = oracle.Sim(**p).init(c["rho_r"], c["rho_b"], None, None)
    s.step(steps)
    m = s.moments()
    a, b = m["rho_r"] / p["rho0_r"], m["rho_b"] / p["rho0_b"]
    R = math.sqrt((0.5 * (1 + (a - b) / (a + b))).sum() / math.pi)
    y, x = np.mgrid[0:64, 0:64]
    r = np.hypot(x + 0.5 - 32, y + 0.5 - 32)
    dp64 = float(m["p"][r < R - 4].mean() - m["p"][r > R + 4].mean())
    sigma = 4.0 * p["A"] / 9.0
    out = {"case": f"static bubble 64x64 R=16, {steps} steps", "fp64_dp": dp64,
           "fp64_laplace_err": abs(dp64 / (sigma / R) - 1.0)}
    m0 = (c["rho_r"].sum(), c["rho_b"].sum())
    for st in ("f32", "f16s", "bf16s"):
        with capi.Lattice(dict(p, storage=st), stream=sid) as g:
            g.init(c["rho_r"], c["rho_b"])
            g.step(steps)
            d = g.diag(check=False)
            Rg = math.sqrt(d["area_r"] / math.pi)
            d = g.diag(circle=(32.0, 32.0, Rg - 4, Rg + 4), check=False)
        dp = d["p_in"] - d["p_out"]
        out[st] = {"dp_rel_to_fp64": dp / dp64 - 1.0, "laplace_err": abs(dp / (sigma / Rg) - 1.0),
                   "mass_drift_r": d["mass_r"] / m0[0] - 1.0, "mass_drift_b": d["mass_b"] / m0[1] - 1.0,
                   "max_u": d["max_u"]}
    return out


def pct(a, q):
    import numpy as np
    return float(np.percentile(np.asarray(a, dtype=np.float64), q)) if len(a) else None


def serve_init(geo):
    from paper_1903_01168_amd import serve
    if geo["kind"] == "disk":
        return serve.init_disk(geo["cx"], geo["cy"], geo["radius"], geo["rho_r_in"], geo["rho_b_in"],
                               geo["rho_r_out"], geo["rho_b_out"])
    return serve.init_bands(geo["edges"], geo["rho_band_r"], geo["rho_band_b"])


def dp_of(diag, req):
    """Laplace pressure jump of a bubble request and its theoretical value."""
    if req["kind"] != "bubble" or diag["n_nonfinite"] > 0 or diag["n_in"] == 0 or diag["n_out"] == 0:
        return None
    R = math.sqrt(diag["area_r"] / math.pi)
    return diag["p_in"] - diag["p_out"], req["params"]["sigma"] / R


def run_serve(args, log):
    """Serving mix: Poisson arrivals of bubble and slug solves of mixed sizes,
    served by the continuous-batching server in 16-bit shifted storage, then
    the same trace solved one at a time on the plain FP32 single-lattice path
    (FIFO; the queueing of that baseline is replayed from measured solve
    times against the same arrival times)."""
    import threading
    import numpy as np
    import torch
    from paper_1903_01168_amd import capi, serve
    from paper_1903_01168_amd import workloads as W

    capi.load()
    torch.cuda.init()
    trace = W.serve_trace(seed=args.seed, n=args.requests, storage=args.storage)
    lu = np.array([r["nodes"] * r["steps"] for r in trace], dtype=np.float64)
    budget = int(args.hbm_budget_gib * (1 << 30))

    # capacity of the batched path: the first requests of the trace, all
    # enqueued at once with the same step count (a saturated closed batch,
    # admission and retirement included)
    ncal = min(48, len(trace))
    with serve.Server(budget, max_slots=args.max_slots, chunk_steps=args.chunk, storage=args.storage) as s:
        ids = [s.enqueue(r["params"], serve_init(r["geo"]), 2000) for r in trace[:ncal]]
        res = [s.wait(i) for i in ids]
        st = s.stats()
    cal_span = max(r["t_done"] for r in res) - min(r["t_arrive"] for r in res)
    capacity = st["lattice_updates"] / cal_span / 1e6
    lam = args.load * capacity * 1e6 / lu.mean()            # requests per second
    arrive = np.cumsum([r["gap"] for r in trace]) / lam
    log(f"serve: capacity {capacity:.0f} MLUPS ({ncal} requests x 2000 steps at once), lambda {lam:.2f}/s, "
        f"trace span {arrive[-1]:.1f} s, {lu.sum():.3e} LU")

    # served run, arrivals in real time
    srv = serve.Server(budget, max_slots=args.max_slots, chunk_steps=args.chunk, storage=args.storage)
    ids = [None] * len(trace)
    t0 = time.perf_counter()

    def client():
        for i, r in enumerate(trace):
            dt = t0 + arrive[i] - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            ids[i] = srv.enqueue(r["params"], serve_init(r["geo"]), r["steps"])

    th = threading.Thread(target=client)
    th.start()
    served = []
    for i in range(len(trace)):
        while ids[i] is None:
            time.sleep(0.001)
        served.append(srv.wait(ids[i]))
        if (i + 1) % 200 == 0:
            log(f"serve: {i + 1}/{len(trace)} served, t = {time.perf_counter() - t0:.1f} s")
    th.join()
    sst = srv.stats()
    srv.close()
    lat = [r["t_done"] - r["t_arrive"] for r in served]
    span = max(r["t_done"] for r in served) - min(r["t_arrive"] for r in served)
    ok = [r["status"] == capi.LBM_OK for r in served]

    # serial FP32 baseline on the single-lattice path
    stream = torch.cuda.Stream()
    sid = stream.cuda_stream
    service, serial_diag, mass0 = [], [], []
    for i, r in enumerate(trace):
        p = dict(r["params"], storage="f32")
        rr, rb = W.geo_fields(r["geo"], p["nx"], p["ny"])
        mass0.append((float(rr.sum()), float(rb.sum())))
        torch.cuda.synchronize()
        t = time.perf_counter()
        lat32 = capi.Lattice(p, stream=sid)
        lat32.init(rr, rb)
        lat32.step(r["steps"])
        d = lat32.diag(check=False)
        if r["kind"] == "bubble" and d["n_nonfinite"] == 0 and d["area_r"] > 0:
            R = math.sqrt(d["area_r"] / math.pi)
            d = lat32.diag(circle=(r["geo"]["cx"], r["geo"]["cy"], R - 4.0, R + 4.0), check=False)
        lat32.close()
        service.append(time.perf_counter() - t)
        serial_diag.append(d)
        if (i + 1) % 200 == 0:
            log(f"serial fp32: {i + 1}/{len(trace)} solved, {sum(service):.1f} s of solve time")
    done, lat_serial = 0.0, []
    for a, sv in zip(arrive, service):
        done = max(a, done) + sv
        lat_serial.append(done - a)
    serial_span = done - arrive[0]

    # Laplace jump and colour mass of the served 16-bit results against FP32
    dpdiff, dpsettled, mdrift16, mdrift32, unstable16, unstable32 = [], [], [], [], 0, 0
    for r, a, b, (m_r, m_b) in zip(trace, served, serial_diag, mass0):
        da = a["diag"]
        unstable16 += int(a["status"] != capi.LBM_OK)
        unstable32 += int(b["n_nonfinite"] > 0)
        if a["status"] != capi.LBM_OK or b["n_nonfinite"] > 0:
            continue
        for dd, acc in ((da, mdrift16), (b, mdrift32)):
            acc.append(max(abs(dd["mass_r"] / m_r - 1.0) if m_r else 0.0,
                           abs(dd["mass_b"] / m_b - 1.0) if m_b else 0.0))
        x, y = dp_of(da, r), dp_of(b, r)
        if x is not None and y is not None:
            dpdiff.append(abs(x[0] - y[0]) / y[1])
            if abs(y[0] / y[1] - 1.0) < 0.1:      # FP32's jump within 10% of Laplace at the request's step
                dpsettled.append(abs(x[0] - y[0]) / y[1])
    if args.records:
        with open(args.records, "w") as fh:
            for r, a, b, ls, l32 in zip(trace, served, serial_diag, lat, lat_serial):
                x, y = dp_of(a["diag"], r), dp_of(b, r)
                fh.write(json.dumps(dict(i=r["index"], kind=r["kind"], gamma=r["gamma"], nx=r["params"]["nx"],
                                         ny=r["params"]["ny"], steps=r["steps"], status=a["status"],
                                         lat=ls, lat_serial=l32, dp=x[0] if x else None,
                                         dp32=y[0] if y else None, dpth=y[1] if y else None)) + "\n")
    bub = sum(1 for r in trace if r["kind"] == "bubble")
    return dict(
        value=lu.sum() / span / 1e6,
        steps=len(trace),
        ms_per_step=span * 1e3 / len(trace),
        workload=f"serving mix: {len(trace)} Poisson-arriving solves ({bub} static bubbles, "
                 f"{len(trace) - bub} gravity slugs), 64^2..1024^2 nodes, 1000..50000 steps, "
                 f"gamma in {{1,10,100,1000}}",
        serving=dict(
            requests=len(trace), lambda_per_s=lam, load=args.load, capacity_mlups=capacity,
            storage=args.storage, chunk_steps=args.chunk, max_slots=args.max_slots,
            hbm_budget_gib=args.hbm_budget_gib, lattice_updates=float(lu.sum()),
            p50_s=pct(lat, 50), p99_s=pct(lat, 99), mean_s=float(np.mean(lat)), makespan_s=span,
            aggregate_mlups=lu.sum() / span / 1e6,
            busy_mlups=sst["lattice_updates"] / sst["busy_s"] / 1e6 if sst["busy_s"] else None,
            busy_frac=sst["busy_s"] / span, admit_s=sst["admit_s"], retire_s=sst["retire_s"],
            chunks=sst["chunks"], peak_active=sst["peak_active"],
            peak_bytes=sst["peak_bytes"], unstable=unstable16, completed_ok=int(sum(ok)),
            serial_fp32=dict(p50_s=pct(lat_serial, 50), p99_s=pct(lat_serial, 99),
                             mean_s=float(np.mean(lat_serial)), makespan_s=serial_span,
                             aggregate_mlups=lu.sum() / serial_span / 1e6,
                             solve_mlups=lu.sum() / sum(service) / 1e6, unstable=unstable32),
            # |dp(served, 16-bit) - dp(serial FP32)| / (sigma / R) per bubble request: all of
            # them (many still in their pressure transient) and those whose FP32 jump is within
            # 10% of Laplace at the request's step count (a bubble can pass there mid-oscillation;
            # --workload serve-laplace tells settled ones by running FP32 four times longer)
            laplace_dp_vs_fp32=dict(n=len(dpdiff), max=max(dpdiff) if dpdiff else None,
                                    p99=pct(dpdiff, 99), median=pct(dpdiff, 50),
                                    over_1pct=int(sum(d > 0.01 for d in dpdiff)),
                                    near_laplace_n=len(dpsettled),
                                    near_laplace_max=max(dpsettled) if dpsettled else None,
                                    near_laplace_median=pct(dpsettled, 50),
                                    near_laplace_over_1pct=int(sum(d > 0.01 for d in dpsettled)),
                                    note="near_laplace: FP32's jump within 10% of sigma/R at the request's step "
                                         "count, which a bubble can pass mid-oscillation; --workload "
                                         "serve-laplace tells settled bubbles by running FP32 four times "
                                         "longer"),
            mass_drift=dict(served_max=max(mdrift16) if mdrift16 else None,
                            fp32_max=max(mdrift32) if mdrift32 else None),
        ),
        first_bubble=next(r for r in trace if r["kind"] == "bubble"),
        budget_bytes=budget,
    )


def main_serve(args, log):
    from paper_1903_01168_amd import workloads as W
    t0 = time.perf_counter()
    r = run_serve(args, log)
    wall = time.perf_counter() - t0
    sv = r["serving"]
    bpu = bytes_per_update(args.storage)
    cpu = None
    if not args.no_cpu_baseline:
        fb = r["first_bubble"]
        p = dict(fb["params"])
        rr, rb = W.geo_fields(fb["geo"], p["nx"], p["ny"])
        cpu = cpu_baseline(dict(params=p, rho_r=rr, rho_b=rb, ux=None, uy=None,
                                name=f"bubble gamma={fb['gamma']}"), args.cpu_seconds)
    out = {
        "metric": "MLUPS & HBM GB/s (% of peak), color-gradient D2Q9; p50/p99 solve latency",
        "value": r["value"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": 0,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else f"f32 arithmetic, {args.storage} storage",
        "data": "synthetic (seeded)",
        "config": {"workload": r["workload"], "storage": args.storage, "seed": args.seed,
                   "step": "one request solved to completion (value: lattice updates / makespan)",
                   "launch": f"batched k_step over all active lattices, HIP-graph chunks of {args.chunk}"},
        "roofline": {"bound": "hbm", "achieved": sv["busy_mlups"] * bpu / 1e3 if sv["busy_mlups"] else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": sv["busy_mlups"] * bpu / 1e3 / HBM_PEAK_GBS if sv["busy_mlups"] else None,
                     "traffic": None, "bytes_per_update": bpu, "kernel": "k_step",
                     "note": "lattice updates / time spent in chunks (chunk set-up included)"},
        "cpu_baseline": cpu,
        "serving": sv,
        "wall_s": wall,
    }
    print(json.dumps(out), flush=True)


def main_serve_laplace(args, log):
    """The serving mix's bubble requests served twice through the server, in
    16-bit and in FP32 storage (the same groups and chunks: grouping is
    bit-neutral, so the two differ by storage alone), and their Laplace
    pressure jumps compared: |dp(16-bit) - dp(FP32)| / (sigma / R).  Every
    request whose difference exceeds 1% is run again in FP32 on the
    single-lattice path for four times its steps, to tell a storage error from
    a bubble that has not settled (FP32's own jump still moving by more than
    1% of sigma / R)."""
    import numpy as np
    import torch
    from paper_1903_01168_amd import capi, serve
    from paper_1903_01168_amd import workloads as W

    capi.load()
    torch.cuda.init()
    trace = [r for r in W.serve_trace(seed=args.seed, n=args.requests, storage=args.storage)
             if r["kind"] == "bubble"]
    budget = int(args.hbm_budget_gib * (1 << 30))
    res = {}
    for st in (args.storage, "f32"):
        t0 = time.perf_counter()
        with serve.Server(budget, max_slots=args.max_slots, chunk_steps=args.chunk, storage=st) as s:
            ids = [s.enqueue(dict(r["params"], storage=st), serve_init(r["geo"]), r["steps"]) for r in trace]
            res[st] = [s.wait(i) for i in ids]
        log(f"serve-laplace: {len(trace)} bubbles served in {st} in {time.perf_counter() - t0:.1f} s")
    rows, diffs = [], []
    for r, a, b in zip(trace, res[args.storage], res["f32"]):
        x, y = dp_of(a["diag"], r), dp_of(b["diag"], r)
        row = dict(i=r["index"], gamma=r["gamma"], n=r["params"]["nx"], steps=r["steps"],
                   status16=a["status"], status32=b["status"])
        if x is None or y is None or a["status"] != capi.LBM_OK or b["status"] != capi.LBM_OK:
            row["compared"] = False
            rows.append(row)
            continue
        row.update(compared=True, diff=abs(x[0] - y[0]) / y[1], lap32=y[0] / y[1] - 1.0, lap16=x[0] / x[1] - 1.0)
        diffs.append(row["diff"])
        rows.append(row)
    outliers = [row for row in rows if row.get("compared") and row["diff"] > 0.01]
    for row, r in ((row, next(t for t in trace if t["index"] == row["i"])) for row in outliers):
        p = dict(r["params"], storage="f32")
        rr, rb = W.geo_fields(r["geo"], p["nx"], p["ny"])
        with capi.Lattice(p) as g:
            g.init(rr, rb)
            g.step(4 * r["steps"])
            d = g.diag(check=False)
            y = None
            if d["n_nonfinite"] == 0 and d["area_r"] > 0:
                R = math.sqrt(d["area_r"] / math.pi)
                d = g.diag(circle=(r["geo"]["cx"], r["geo"]["cy"], R - 4.0, R + 4.0), check=False)
                y = dp_of(d, r)
        b = dp_of(res["f32"][trace.index(r)]["diag"], r)
        row["lap32_4x"] = y[0] / y[1] - 1.0 if y else None
        row["fp32_moves_4x"] = abs(y[0] - b[0]) / y[1] if y else None
        log(f"serve-laplace outlier {row}")
    settled_out = [row for row in outliers if row["fp32_moves_4x"] is not None and row["fp32_moves_4x"] <= 0.01]
    out = {
        "workload": f"serving mix, bubble requests only: {len(trace)} of {args.requests} "
                    f"(gamma in {{1,10,100,1000}}, 64^2..1024^2, 1000..50000 steps)",
        "storage": args.storage, "compared": len(diffs),
        "not_compared": sum(1 for row in rows if not row.get("compared")),
        "diff_median": pct(diffs, 50), "diff_p99": pct(diffs, 99), "diff_max": max(diffs) if diffs else None,
        "over_1pct": len(outliers),
        "over_1pct_with_fp32_settled": len(settled_out),
        "outliers": outliers,
        "definition": "diff = |dp(16-bit) - dp(FP32)| / (sigma / R), both served through the server; "
                      "fp32_moves_4x = |dp(FP32, 4 x steps) - dp(FP32)| / (sigma / R)",
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="channel",
                    help="channel (default), sweep512, slug, hbm8192, bubble64, serve, or serve-laplace "
                         "(16-bit against FP32 storage on the serving mix's bubbles)")
    ap.add_argument("--storage", default=None, choices=["f32", "f16s", "bf16s"],
                    help="population storage (default f32; f16s for the serving mix)")
    ap.add_argument("--collision", default="bgk", choices=["bgk", "mrt"])
    ap.add_argument("--ns-correction", action="store_true",
                    help="Navier-Stokes correction of Sec. 2.1.3 (needs --collision mrt)")
    ap.add_argument("--gradient", default="nearest", choices=["nearest", "isotropic"],
                    help="colour-gradient stencil: nearest neighbours, or the second-neighbour isotropic one")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--strip", type=int, default=0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the storage-precision report (converged 64x64 bubble vs the FP64 oracle)")
    ap.add_argument("--cpu-steps", type=int, default=2000, help="at most this many oracle steps in cpu_baseline")
    ap.add_argument("--no-secondary", action="store_true", help="channel: skip the cache-resident sweep figure")
    ap.add_argument("--secondary-steps", type=int, default=2000, help="steps of the cache-resident sweep figure")
    ap.add_argument("--no-copy", action="store_true", help="skip the plain-copy bandwidth figure")
    ap.add_argument("--requests", type=int, default=2000, help="serve: number of requests")
    ap.add_argument("--load", type=float, default=0.8, help="serve: offered load / measured capacity")
    ap.add_argument("--chunk", type=int, default=100, help="serve: steps per chunk")
    ap.add_argument("--max-slots", type=int, default=256, help="serve: lattices advanced together")
    ap.add_argument("--hbm-budget-gib", type=float, default=64.0, help="serve: device memory budget")
    ap.add_argument("--records", default="", help="serve: write one JSON line per request to this file")
    ap.add_argument("--copy-only", type=float, default=0.0,
                    help="only time the plain copy kernel over this many GiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the step runs on one GPU: there is no multi-GPU path to measure "
                                   "(how a lattice would be split into slabs is described in the design notes)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.storage is None:
        args.storage = "f16s" if args.workload in ("serve", "serve-laplace") else "f32"

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.workload == "serve":
        main_serve(args, log)
        return
    if args.workload == "serve-laplace":
        main_serve_laplace(args, log)
        return

    import torch
    from paper_1903_01168_amd import capi
    from paper_1903_01168_amd import workloads as W

    capi.load()
    torch.cuda.init()
    stream = torch.cuda.Stream()           # default priority
    sid = stream.cuda_stream

    if args.copy_only > 0:
        print(json.dumps(copy_rate(capi, W, torch, stream, args.copy_only)))
        return

    cells, wname = build_cells(args, W)
    if args.ns_correction:
        if args.collision != "mrt":
            raise SystemExit("--ns-correction needs --collision mrt")
        for c in cells:
            c["params"]["ns_correction"] = True
    for c in cells:
        c["params"]["gradient"] = args.gradient
    m = measure(capi, torch, stream, cells, args.steps, args.warmup, args.tile, args.strip)
    log(f"{wname}: {m['mlups']:.0f} MLUPS, {m['ms_per_step'] * 1e3:.1f} us per step, "
        f"{m['launches']} launch(es) per step")

    bpu = bytes_per_update(args.storage)
    nodes = m["nodes"]
    # algorithmic bytes of one launch over the launch's average duration:
    # with one launch per step (a single lattice) the launches run back to
    # back on one stream and the HIP events around the timed region give their
    # average; with several launches per step (groups of a batch, two in
    # flight on two streams) only the step's time is defined, and the figure
    # is the algorithmic bytes of a step over it
    achieved = bpu * nodes / (m["ms_per_step"] / 1e3) / 1e9
    traffic, valu = stored_counters(args)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "bytes_per_update": bpu,
                "kernel": "k_step", "flavour": m["flavour"], "launches_per_step": m["launches"],
                "launch_us" if m["launches"] == 1 else "step_us": m["ms_per_step"] * 1e3,
                "kernel_hash": kernel_hash(),
                "definition": "achieved = bytes_per_update x lattice nodes of one launch / average launch "
                              "duration (HIP events around the timed launches on their stream)"
                              if m["launches"] == 1 else
                              "achieved = bytes_per_update x nodes of one step / step time (several launches "
                              "per step, two in flight on two streams)"}
    if m["bytes"] <= 256 << 20:
        roofline["note"] = ("working set within MI355X's 256 MB Infinity Cache: a cache rate, not an HBM "
                            "figure")
    if valu is not None:
        v = dict(per_update=valu, achieved=m["mlups"] * 1e6 * valu / 1e9, peak=VALU_PEAK_GIPS,
                 unit="G wave64 VALU instructions/s")
        v["frac"] = v["achieved"] / VALU_PEAK_GIPS
        if args.storage == "f32":
            roofline["valu"] = v
        else:
            # the 16-bit codec makes those kernels VALU-bound
            hbm = {k: roofline[k] for k in ("achieved", "peak", "unit", "frac")}
            roofline.update(bound="alu", achieved=v["achieved"], peak=v["peak"], unit=v["unit"], frac=v["frac"],
                            valu_per_update=valu, hbm=hbm)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cells[0], args.cpu_seconds, steps_cap=args.cpu_steps)
    secondary = None
    if args.workload == "channel" and not args.no_secondary:
        # the cache-resident counterpart: the 9 x 512^2 static-bubble sweep
        # (340 MB in groups sized for the Infinity Cache)
        sw = W.bubble_sweep(seed=args.seed, n=512, storage=args.storage, collision=args.collision)
        ms = measure(capi, torch, stream, sw, args.secondary_steps, 64, 0, 0)
        secondary = {"workload": "static-bubble sweep 9 x 512^2 (gamma in {10,100,1000} x M in {1,10,100})",
                     "value": ms["mlups"], "unit": "MLUPS", "ms_per_step": ms["ms_per_step"],
                     "launches_per_step": ms["launches"], "steps": args.secondary_steps,
                     "alg_gbs": bpu * ms["nodes"] / (ms["ms_per_step"] / 1e3) / 1e9,
                     "note": "mall-resident: lattices stepped in groups that stay in the 256 MB Infinity Cache "
                             "between steps; a cache rate, not an HBM figure"}
        secondary["frac_of_hbm_peak"] = secondary["alg_gbs"] / HBM_PEAK_GBS
    copy = None if args.no_copy else copy_rate(capi, W, torch, stream, 1.0)
    precision = None if args.no_precision else precision_report(sid)

    p0 = cells[0]["params"]
    out = {
        "metric": "MLUPS & HBM GB/s (% of peak), color-gradient D2Q9; p50/p99 solve latency",
        "value": m["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else f"f32 arithmetic, {args.storage} storage",
        "data": "synthetic (seeded)",
        "config": {"workload": wname, "lattices": len(cells), "nx": p0["nx"], "ny": p0["ny"],
                   "nodes": nodes, "storage": args.storage, "collision": args.collision,
                   "ns_correction": bool(args.ns_correction), "gradient": args.gradient,
                   "population_bytes": m["bytes"], "steps_simulated": args.warmup + args.steps,
                   "seed": args.seed, "launch": m["launch"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "mall_resident": secondary,
        "hbm_copy": copy,
        "precision": precision,
        "wall_s": m["wall"],
        "state": m["state"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
