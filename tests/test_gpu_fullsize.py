"""Parity at the full sizes of the benchmark configurations, in the launch
configuration bench.py times (a batch: one k_step launch per group of lattices
and step, two groups in flight on two streams, automatic tile width and strip
height, HIP-graph replay): the nine 512 x 512 lattices of
the bubble sweep, the 4096 x 256 gravity slug and the 8192 x 512 inlet/outlet
channel, each against the FP64 oracle after STEPS steps (one graph replay of
32 steps plus single launches).

Bounds.  The FP32-against-FP64 bound of the static bubble, max |d rho| / rho
<= 1e-5 and max |d u| <= 1e-6, or, where the flow amplifies rounding (sharp
density-ratio interfaces in their first steps), 20 times the change that
storage rounding alone causes in the FP64 oracle (50 times for FP32 storage,
whose GPU error is mostly arithmetic): its populations rounded to FP32 or
passed through a model of the 16-bit format (tests/storage16.py) after every
step.  The GPU rounds each population ten to thirty times per step where
storage rounds it once; measured ratios of GPU error to storage-only
sensitivity run from 4 to 28.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1903_01168_amd import capi
from paper_1903_01168_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 40


def say(*a):
    print("[gpu-fullsize]", *a, file=sys.stderr, flush=True)


def _errors(om, gm):
    rho_o = om["rho_r"] + om["rho_b"]
    rho_g = gm["rho_r"] + gm["rho_b"]
    drho = float(np.max(np.abs(rho_g - rho_o) / rho_o))
    du = float(max(np.max(np.abs(gm["ux"] - om["ux"])), np.max(np.abs(gm["uy"] - om["uy"]))))
    return drho, du


def _oracle(c, steps, color=None, storage=None):
    """The oracle's moments after `steps`; with `storage`, its stored
    populations are rounded to that format after every step."""
    s = oracle.Sim(**c["params"]).init(c["rho_r"], c["rho_b"], c["ux"], c["uy"])
    if color is not None:
        s.set_inlet_color(color)
    if storage is None:
        s.step(steps)
    else:
        from storage16 import quantise
        for _ in range(steps):
            s.step(1)
            pops = s.get_pops()
            s.set_pops(pops.astype(np.float32).astype(np.float64) if storage == "f32"
                       else quantise(pops, c["params"], storage))
    return s.moments()


def _check(name, storage, om, gm, c, color=None, sens=None):
    """sens: (oracle moments, case) on which to measure the storage
    sensitivity instead of (om, c)."""
    drho, du = _errors(om, gm)
    if drho <= 1e-5 and du <= 1e-6:
        say(f"{storage} {name}: drho/rho {drho:.2e}, du {du:.2e} (fixed bounds)")
        return
    so, sc = sens if sens is not None else (om, c)
    s_rho, s_u = _errors(so, _oracle(sc, STEPS, color, storage))
    f = 50 if storage == "f32" else 20
    tol_rho, tol_u = max(1e-5, f * s_rho), max(1e-6, f * s_u)
    say(f"{storage} {name}: drho/rho {drho:.2e}, du {du:.2e}; storage sensitivity of the oracle "
        f"{s_rho:.2e}, {s_u:.2e} -> bounds {tol_rho:.2e}, {tol_u:.2e}")
    assert drho <= tol_rho and du <= tol_u, name


@pytest.fixture(scope="module")
def sweep_fp64():
    cells = W.bubble_sweep(seed=0, n=512)
    say(f"oracle: 9 x 512^2, {STEPS} steps")
    return cells, [_oracle(c, STEPS) for c in cells]


# Sweep cells beyond the method's stable range: with density ratio 1000 the
# FP64 oracle goes non-finite within 500 steps at viscosity ratios 1 and 10
# (tau_light = 100.5 and 10.5 against tau_heavy = 0.6) and reaches |u| = 0.17
# by step 4000 at ratio 100; all three blow up within the benchmark's 20200
# steps.  Their first steps amplify rounding by two orders of magnitude or
# more, so they are checked for finite values only.
UNSTABLE = {(1000, 1), (1000, 10), (1000, 100)}


@pytest.mark.parametrize("storage", ["f32", "f16s", "bf16s"])
def test_sweep512_batched(sweep_fp64, storage):
    cells, ref = sweep_fp64
    if storage != "f32":      # the three density ratios at viscosity ratio 10
        keep = [k for k, c in enumerate(cells) if c["M"] == 10]
        cells, ref = [cells[k] for k in keep], [ref[k] for k in keep]
    lats = []
    for c in cells:
        g = capi.Lattice(dict(c["params"], storage=storage))
        g.init(c["rho_r"], c["rho_b"])
        lats.append(g)
    with capi.Batch(lats) as b:
        b.step(STEPS)
    try:
        for c, g, om in zip(cells, lats, ref):
            gm = g.moments(check=False)
            if (c["gamma"], c["M"]) in UNSTABLE:
                assert all(np.all(np.isfinite(gm[k])) for k in ("rho_r", "rho_b", "ux", "uy")), c["name"]
                say(f"{storage} {c['name']}: finite (unstable configuration, not compared)")
                continue
            _check(c["name"], storage, om, gm, c)
    finally:
        for g in lats:
            g.close()


@pytest.mark.parametrize("variant", ["isotropic", "mrt_nsc"])
def test_sweep512_variants(variant):
    """The three density ratios at viscosity ratio 10 of the sweep, batched
    at full size, with the second-neighbour gradient (its own tile width)
    and with MRT and the Navier-Stokes correction, against the oracle run
    with the same variant (density ratio 1000, beyond the stable range:
    only whether the run is still finite is compared)."""
    cells = [c for c in W.bubble_sweep(seed=0, n=512) if c["M"] == 10]
    extra = dict(gradient="isotropic") if variant == "isotropic" else dict(collision="mrt", ns_correction=True)
    cells = [dict(c, params=dict(c["params"], **extra)) for c in cells]
    lats = []
    for c in cells:
        g = capi.Lattice(c["params"])
        g.init(c["rho_r"], c["rho_b"])
        lats.append(g)
    with capi.Batch(lats) as b:
        b.step(STEPS)
    try:
        for c, g in zip(cells, lats):
            gm = g.moments(check=False)
            om = _oracle(c, STEPS)
            if (c["gamma"], c["M"]) in UNSTABLE:
                # beyond the stable range: with the correction (heavy-fluid sound speed
                # 0.022) the oracle itself is non-finite by step 20; the GPU agrees on
                # whether the run is still finite
                fin = [all(np.all(np.isfinite(m[k])) for k in ("rho_r", "rho_b", "ux", "uy")) for m in (gm, om)]
                say(f"{c['name']} {variant}: finite on the GPU {fin[0]}, in the oracle {fin[1]}")
                assert fin[0] == fin[1], c["name"]
                continue
            _check(f"{c['name']} {variant}", "f32", om, gm, c)
    finally:
        for g in lats:
            g.close()


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_slug_4096x256(storage):
    c = W.gravity_slug(seed=0, gamma=10, Re=10)
    om = _oracle(c, STEPS)
    with capi.Lattice(dict(c["params"], storage=storage)) as g:
        g.init(c["rho_r"], c["rho_b"])
        g.step(STEPS)
        _check("slug 4096x256", storage, om, g.moments(check=False), c)


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_channel_8192x512(storage):
    """The paper's open-channel set-up (stratified inflow, density ratio 5).
    The storage sensitivity is measured on the same channel cut to 1024
    columns: in STEPS steps nothing travels further than STEPS nodes, so the
    shorter channel holds every neighbourhood the long one has (inlet, outlet,
    interface rows, uniform bulk)."""
    c = W.inlet_outlet(seed=0)
    color = c["inlet_color"]
    om = _oracle(c, STEPS, color)
    with capi.Lattice(dict(c["params"], storage=storage)) as g:
        g.init(c["rho_r"], c["rho_b"])
        g.set_inlet_color(color)
        g.step(STEPS)
        gm = g.moments(check=False)
    short = W.inlet_outlet(seed=0, nx=1024)
    _check("channel 8192x512", storage, om, gm, c, color, sens=(_oracle(short, STEPS, color), short))
