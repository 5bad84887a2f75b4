"""Writes e1_channel.json: the FP64 oracle's observables of the paper's
inlet/outlet verification channel (Sec. 2.5 item 3: a 500 x 50 channel,
heavy fluid (density ratio 5) in the lower half of the inflow, light above,
the heavy one entering six times faster, MRT with the Navier-Stokes
correction, 50000 steps), for no-slip and free-slip walls: per phase, the
mean velocity over its rows on the inlet column and the two columns after
it, over the prescribed value; the mean pressure on the outlet column and the
one before it, over p_out; at steps 10000, 25000 and 50000.  The same
observables of a second run whose stored populations are rounded to FP32
after every step (the oracle's sensitivity to FP32 storage, for the parity
bound) are kept beside them.  Only the oracle is called.
Run: python tests/golden/make_e1_channel.py"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle                                     # noqa: E402
from paper_1903_01168_amd import workloads as W   # noqa: E402

NX, NY, GAMMA, UL = 500, 50, 5.0, 0.005
UH = 6 * UL
P_OUT = 0.48
CHECKPOINTS = (10000, 25000, 50000)


def case(walls):
    p = W.params(nx=NX, ny=NY, bc_x="open", bc_y=walls, rho0_r=GAMMA, rho0_b=1.0, tau_r=0.6, tau_b=0.75,
                 A=1e-3, u_in_r=UH, u_in_b=UL, p_out=P_OUT, collision="mrt", ns_correction=True)
    color = np.where(np.arange(NY) < NY // 2, 1, -1).astype(np.int8)
    rr = np.where(color[:, None] > 0, GAMMA, 0.0) * np.ones((1, NX))
    rb = np.where(color[:, None] > 0, 0.0, 1.0) * np.ones((1, NX))
    return p, color, rr, rb


def observables(m, color):
    heavy = color > 0
    out = {}
    for x in (0, 1, 2):
        out[f"v_heavy_{x}"] = float(m["ux"][heavy, x].mean() / UH)
        out[f"v_light_{x}"] = float(m["ux"][~heavy, x].mean() / UL)
    out["p_out"] = float(m["p"][:, -1].mean() / P_OUT)
    out["p_out_1"] = float(m["p"][:, -2].mean() / P_OUT)
    return out


def main():
    res, rnd = {}, {}
    for walls in ("walls", "freeslip"):
        p, color, rr, rb = case(walls)
        for out, r32 in ((res, False), (rnd, True)):
            s = oracle.Sim(**p).init(rr, rb, None, None)
            s.set_inlet_color(color)
            out[walls] = {}
            for t in CHECKPOINTS:
                s.step(t - s.steps_done, round_f32=r32)
                out[walls][str(t)] = observables(s.moments(), color)
                print(walls, "rounded" if r32 else "plain", t, out[walls][str(t)], flush=True)
    with open(os.path.join(HERE, "e1_channel.json"), "w") as f:
        json.dump({"case": "inlet/outlet verification channel 500 x 50, density ratio 5, v_heavy = 6 v_light, "
                           "MRT + Navier-Stokes correction (FP64 oracle)", "values": res,
                   "values_fp32_storage": rnd}, f, indent=1)


if __name__ == "__main__":
    main()
