"""How much the paper's observables move between readings of the rules the
paper leaves open (test infrastructure, run by hand: ``python -m oracle.readings``).

Runs the FP64 oracle twice or more per case, once with the reading the
library implements and once per alternative (``Sim(alt=...)``), and prints
the observables the paper judges each case by:

* open channel with two stratified phases (Sec. 2.5 item 3 verification: a
  500 x 50 channel, density ratio 5, heavy inflow six times the light one,
  MRT with the Navier-Stokes correction, 50000 steps): the inflow velocity of
  each phase over its prescribed value (on the inlet column and one node in), the outlet pressure over p_out (the
  paper asks for 2%), the heavy layer's thickness half-way down the channel,
  and the largest change of any node's velocity against the library's
  reading.  Alternatives: Q = 0 on wall ghost nodes (Sec. 2.1.3) and the
  outlet colour taken from the column upstream (Sec. 2.5 item 3);
* a droplet on a wall relaxing to a prescribed contact angle (Sec. 2.4; the
  100 x 100 case, MRT with the correction, 20000 steps), nearest-neighbour and
  second-neighbour gradient: the cap angle and the largest velocity change.
  Alternatives: Q = 0 on wall ghost nodes, and for the second-neighbour
  gradient the outer ghost row linearly extrapolated (Sec. 4 remark).
"""
import math
import multiprocessing as mp
import os
import sys

os.environ.setdefault("OMP_NUM_THREADS", "1")   # one thread per case; the cases run side by side

import numpy as np

import oracle
from paper_1903_01168_amd import workloads as W

CHANNEL_STEPS = 50000
DROPLET_STEPS = 20000


def _channel(alt):
    nx, ny, gamma, ul = 500, 50, 5.0, 0.005
    uh = 6 * ul
    p = W.params(nx=nx, ny=ny, bc_x="open", bc_y="walls", rho0_r=gamma, rho0_b=1.0, tau_r=0.6, tau_b=0.75,
                 A=1e-3, u_in_r=uh, u_in_b=ul, p_out=0.48, collision="mrt", ns_correction=True)
    color = np.where(np.arange(ny) < ny // 2, 1, -1).astype(np.int8)
    rr = np.where(color[:, None] > 0, gamma, 0.0) * np.ones((1, nx))
    rb = np.where(color[:, None] > 0, 0.0, 1.0) * np.ones((1, nx))
    s = oracle.Sim(**dict(p, alt=alt)).init(rr, rb, None, None)
    s.set_inlet_color(color)
    s.step(CHANNEL_STEPS)
    m = s.moments()
    heavy = color > 0
    psi = (m["rho_r"] - m["rho_b"]) / (m["rho_r"] + m["rho_b"])
    return dict(m=m, obs=dict(
        v_heavy=m["ux"][heavy, 0].mean() / uh, v_light=m["ux"][~heavy, 0].mean() / ul,
        v_heavy1=m["ux"][heavy, 1].mean() / uh, v_light1=m["ux"][~heavy, 1].mean() / ul,
        p_out=m["p"][:, -1].mean() / 0.48, p_out1=m["p"][:, -2].mean() / 0.48,
        layer=float((0.5 * (1 + psi[:, nx // 2])).sum()), umax=float(np.hypot(m["ux"], m["uy"]).max())))


def cap_angle(m):
    """Contact angle (degrees) of the circular cap with the red area and the
    red width of the bottom row."""
    psi = (m["rho_r"] - m["rho_b"]) / (m["rho_r"] + m["rho_b"])
    area, base = (0.5 * (1 + psi)).sum(), (0.5 * (1 + psi[0])).sum()
    f = lambda t: (t - math.sin(t) * math.cos(t)) / (4 * math.sin(t) ** 2) - area / base ** 2
    lo, hi = 1e-3, math.pi - 1e-3
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        lo, hi = (lo, mid) if f(lo) * f(mid) <= 0 else (mid, hi)
    return math.degrees(0.5 * (lo + hi))


def _droplet(angle, gradient, alt):
    c = W.wall_droplet(angle, n=100, collision="mrt")
    p = dict(c["params"], ns_correction=True, gradient=gradient, alt=alt)
    s = oracle.Sim(**p).init(c["rho_r"], c["rho_b"], None, None)
    s.step(DROPLET_STEPS)
    m = s.moments()
    return dict(m=m, obs=dict(angle=cap_angle(m), umax=float(np.hypot(m["ux"], m["uy"]).max())))


def _run(job):
    kind, args = job
    out = _channel(*args) if kind == "channel" else _droplet(*args)
    print(f"done {kind} {args}", file=sys.stderr, flush=True)
    return out


def main():
    A = oracle
    jobs = [("channel", (0,)), ("channel", (A.ALT_Q_WALL_ZERO,)), ("channel", (A.ALT_OUTLET_UPSTREAM,))]
    for angle in (60.0, 120.0):
        jobs += [("droplet", (angle, "nearest", 0)), ("droplet", (angle, "nearest", A.ALT_Q_WALL_ZERO)),
                 ("droplet", (angle, "isotropic", 0)), ("droplet", (angle, "isotropic", A.ALT_ISO_EXTRAP))]
    with mp.Pool(min(len(jobs), 8)) as pool:
        res = pool.map(_run, jobs)
    base = {}
    for (kind, args), r in zip(jobs, res):
        key = (kind,) + tuple(a for a in args[:-1])
        if args[-1] == 0:
            base[key] = r["m"]
    for (kind, args), r in zip(jobs, res):
        ref = base[(kind,) + tuple(args[:-1])]
        du = float(max(np.abs(r["m"]["ux"] - ref["ux"]).max(), np.abs(r["m"]["uy"] - ref["uy"]).max()))
        rho, rho0 = r["m"]["rho_r"] + r["m"]["rho_b"], ref["rho_r"] + ref["rho_b"]
        drho = float((np.abs(rho - rho0) / rho0).max())
        obs = " ".join(f"{k} {v:.5f}" for k, v in r["obs"].items())
        print(f"{kind} {args}: {obs} | max |du| {du:.2e} max |drho|/rho {drho:.2e}", flush=True)


if __name__ == "__main__":
    main()
