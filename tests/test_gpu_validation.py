"""Validation runs of the paper's own set-ups on the GPU (context for the
parity tests: these compare with the paper's statements, not with the
oracle).

Square-to-droplet (Sec. 4): a light square of side 0.33 n relaxes to a
circle; the pressure jump (means over r < R - 4 and r > R + 4, R from the
red area) against Laplace's sigma / R, sigma = 0.01, beta scaled with the
resolution as in the paper.  The paper reports at most 1% error for density
and viscosity ratios (1, 1) at the bubble's centre and under 2.5% for
(5, 2); measured here after 20 capillary times t_s = sqrt(rho a^3 / sigma):
(1, 1) 1.6% / 0.8-1.0% / 0.1-1.0% at 60^2 / 100^2 / 200^2, (5, 2)
2.7-3.0% / 1.3-1.7% / 0.3-1.3% (BGK-MRT).  Bounds: 2% and 3.5% at 60^2,
1.5% and 2.5% above; (1, 100) within 2.5%; (1000, 1000) within 3% after 40
t_s at 60^2 and 100^2 (the heavy fluid's sound waves decay slowly); the
error at 200^2 below that at 60^2 for (1, 1) and (5, 2).

Inlet/outlet (Sec. 2.5 item 3 verification): a 500 x 50 channel, heavy
(density 5) below light, v_heavy = 6 v_light, 50000 steps, MRT with the
Navier-Stokes correction (without it the plain schemes, in the FP64 oracle
as on the GPU, send a pressure wave through the outlet and blow up within
50000 steps here).  The prescribed inlet velocity of each phase and the
outlet pressure are recovered within 2% (the paper's bound) on the boundary
nodes, where the Zou-He completion makes them exact by construction, and the
outlet pressure one node in (not exact: 0.9996 of p_out).  The inflow does
not stay plug-shaped: one node in, the mean over the heavy phase's rows is
3.2% above its prescribed velocity and the light phase's 11.5% (no-slip
walls; 3.1% and 11.4% with free-slip walls: the 6:1 velocity jump at the
interface reshapes the profile at once), above the paper's 2%; this is the
method's result, not the kernels': the GPU reproduces every one of these
observables of the FP64 oracle (tests/golden/e1_channel.json, written by
make_e1_channel.py) within E1_AGREE = 2e-4, one hundredth of the paper's
2% (measured: up to 1.8e-4, the light phase two nodes in after 50000 steps
with free-slip walls; 3e-5 and less elsewhere).  That is not the per-node
parity rule of tests/bounds.py: over tens of thousands of steps of a nearly
steady open flow, FP32 rounding that falls the same way at every node and
step shifts such row means coherently (the FP64 oracle with FP32-rounded
storage moves them by only 1e-8, its roundings having random signs).  The run
stays finite with max |u| < 0.1."""
import json
import math
import os
import sys

import numpy as np
import pytest

from paper_1903_01168_amd import capi
from paper_1903_01168_amd import workloads as W

pytestmark = pytest.mark.gpu

SIGMA = 0.01
E1_AGREE = 2e-4


def say(*a):
    print("[gpu-validation]", *a, file=sys.stderr, flush=True)


def _laplace_error(c, collision, t_caps):
    p = dict(c["params"], collision=collision)
    ts = math.sqrt(c["side"] ** 3 / SIGMA)
    with capi.Lattice(p) as g:
        g.init(c["rho_r"], c["rho_b"])
        g.step(int(t_caps * ts))
        d0 = g.diag()
        R = math.sqrt(d0["area_r"] / math.pi)
        cx, cy = c["center"]
        d = g.diag(circle=(cx, cy, R - 4, R + 4))
    return (d["p_in"] - d["p_out"]) * R / SIGMA - 1.0


SQUARE = [((1, 1, 1.0), {60: 0.02, 100: 0.015, 200: 0.015}),
          ((5, 2, 1.0), {60: 0.035, 100: 0.025, 200: 0.025}),
          ((1, 100, 0.515), {60: 0.025, 100: 0.025, 200: 0.025})]


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
@pytest.mark.parametrize("case", SQUARE, ids=["rho1_mu1", "rho5_mu2", "rho1_mu100"])
def test_square_to_droplet_laplace(case, collision):
    (gamma, M, tau_l), bounds = case
    errs = {}
    for n, bound in bounds.items():
        c = W.square_droplet(n, gamma, M, sigma=SIGMA, tau_light=tau_l)
        errs[n] = _laplace_error(c, collision, 20)
        say(f"({gamma},{M}) {collision} {n}x{n}: Laplace error {100 * errs[n]:+.2f}%")
        assert abs(errs[n]) <= bound
    if M <= 2:
        assert abs(errs[200]) < abs(errs[60])


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_square_to_droplet_density_ratio_1000(collision):
    for n in (60, 100):
        c = W.square_droplet(n, 1000, 1000, sigma=SIGMA)
        err = _laplace_error(c, collision, 40)
        say(f"(1000,1000) {collision} {n}x{n}: Laplace error {100 * err:+.2f}%")
        assert abs(err) <= 0.03


@pytest.mark.parametrize("walls", ["walls", "freeslip"])
def test_inlet_outlet_recovers_prescribed_values(walls):
    nx, ny, gamma, ul = 500, 50, 5.0, 0.005
    uh = 6 * ul
    p = W.params(nx=nx, ny=ny, bc_x="open", bc_y=walls, rho0_r=gamma, rho0_b=1.0, tau_r=0.6, tau_b=0.75,
                 A=1e-3, u_in_r=uh, u_in_b=ul, p_out=0.48, collision="mrt", ns_correction=True)
    color = np.where(np.arange(ny) < ny // 2, 1, -1).astype(np.int8)
    rr = np.where(color[:, None] > 0, gamma, 0.0) * np.ones((1, nx))
    rb = np.where(color[:, None] > 0, 0.0, 1.0) * np.ones((1, nx))
    heavy = color > 0
    with open(os.path.join(os.path.dirname(__file__), "golden", "e1_channel.json")) as f:
        stored = json.load(f)
    gold, gold32 = stored["values"][walls], stored["values_fp32_storage"][walls]
    with capi.Lattice(p) as g:
        g.init(rr, rb)
        g.set_inlet_color(color)
        for t in (10000, 25000, 50000):
            g.step(t - g.steps_done)
            m = g.moments()
            got = {"p_out": m["p"][:, -1].mean() / 0.48, "p_out_1": m["p"][:, -2].mean() / 0.48}
            for x in (0, 1, 2):
                got[f"v_heavy_{x}"] = m["ux"][heavy, x].mean() / uh
                got[f"v_light_{x}"] = m["ux"][~heavy, x].mean() / ul
            ref, ref32 = gold[str(t)], gold32[str(t)]
            umax = float(np.hypot(m["ux"], m["uy"]).max())
            say(f"{walls} step {t}: " + ", ".join(f"{k} {v:.5f} (FP64 {ref[k]:.5f})" for k, v in got.items())
                + f", max |u| {umax:.3f}")
            assert abs(got["v_heavy_0"] - 1) <= 0.02 and abs(got["v_light_0"] - 1) <= 0.02
            assert abs(got["p_out"] - 1) <= 0.02
            assert abs(got["p_out_1"] - 1) <= 0.02
            for k, v in got.items():
                assert abs(v - ref[k]) <= E1_AGREE, (k, v, ref[k], abs(ref32[k] - ref[k]))
            assert umax < 0.1
