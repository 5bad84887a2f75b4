"""Parity at the full sizes of the benchmark configurations, in the launch
configurations that bench.py times, over LONG = 1000 steps in FP32 against the
FP64 oracle: the 8192 x 512 inlet/outlet channel as one lattice with the
planned flavour (block exchange: its two buffers exceed 256 MiB), and the
six stable cells of the 9 x 512^2 bubble sweep as a batch (one k_step launch
per group of lattices and step, two groups in flight on two streams, planned
tile width and strip height, HIP-graph replay); the sweep's cells at viscosity
ratio 10 with the second-neighbour gradient and with MRT and the
Navier-Stokes correction; the 4096 x 256 gravity slug.

The oracle's side is stored (tests/golden/fullsize_<case>.npz, written by
tests/golden/make_fullsize.py, which calls only the oracle): its moments on
a grid of sampled nodes and the edge columns, and its sensitivity to FP32
storage rounding over the whole lattice.  Bounds (tests/bounds.py): the
fixed FP32 bound on every sample, or FACTOR times that sensitivity; the
ratio of the GPU error to it is printed for every case.  The three cells at
density ratio 1000 lie beyond the method's stable range (the FP64 oracle
goes non-finite within 500 steps at viscosity ratios 1 and 10 and reaches
|u| = 0.17 by step 4000 at 100); they run SHORT steps in the batch, where
only finiteness is compared.

16-bit storage at these sizes: colour mass to 1e-7 and finite values after
LONG steps (the bubble sweep, the slug) and 3 LONG steps (the channel); its
accuracy against FP64 is measured on converged observables by the precision
tests.
"""
import os
import sys

import numpy as np
import pytest

from bounds import Bound, oracle_run
from paper_1903_01168_amd import capi
from paper_1903_01168_amd import workloads as W

pytestmark = pytest.mark.gpu

LONG = 1000
SHORT = 40
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

UNSTABLE = {(1000, 1), (1000, 10), (1000, 100)}


def say(*a):
    print("[gpu-fullsize]", *a, file=sys.stderr, flush=True)


def _stored(name):
    """The oracle's sampled moments after LONG steps and a Bound whose
    sensitivity is the stored one."""
    z = np.load(os.path.join(GOLDEN, f"fullsize_{name}.npz"))
    assert int(z["steps"]) == LONG
    om = {k: z[k] for k in ("rho_r", "rho_b", "ux", "uy")}
    bound = Bound(om, None, tag="gpu-fullsize")
    bound.s = (float(z["s_rho"]), float(z["s_u"]))
    return (z["ys"], z["xs"]), bound


def _check(name, gm):
    (ys, xs), bound = _stored(name)
    bound.check(name, {k: gm[k][ys, xs] for k in ("rho_r", "rho_b", "ux", "uy")}, always_ratio=True)


def _finite(m):
    return all(np.all(np.isfinite(m[k])) for k in ("rho_r", "rho_b", "ux", "uy"))


def _batch(cells, steps, storage="f32"):
    lats = []
    for c in cells:
        g = capi.Lattice(dict(c["params"], storage=storage))
        g.init(c["rho_r"], c["rho_b"])
        lats.append(g)
    with capi.Batch(lats) as b:
        b.step(steps)
    return lats


def _close(lats):
    for g in lats:
        g.close()


def _name(c, variant=""):
    return f"sweep_g{c['gamma']}_M{c['M']}" + (f"_{variant}" if variant else "")


def test_channel_8192x512():
    """The paper's open-channel set-up (stratified inflow, density ratio 5),
    one lattice, planned launch, as the benchmark steps it."""
    c = W.inlet_outlet(seed=0)
    with capi.Lattice(c["params"]) as g:
        g.init(c["rho_r"], c["rho_b"])
        g.set_inlet_color(c["inlet_color"])
        g.step(LONG)
        _check("channel", g.moments(check=False))


def test_sweep512_batched():
    cells = [c for c in W.bubble_sweep(seed=0, n=512) if (c["gamma"], c["M"]) not in UNSTABLE]
    lats = _batch(cells, LONG)
    try:
        for c, g in zip(cells, lats):
            _check(_name(c), g.moments(check=False))
    finally:
        _close(lats)


def test_sweep512_unstable_cells_finite():
    """The density-ratio-1000 cells, batched with the rest: the GPU agrees
    with the oracle on whether each run is still finite after SHORT steps."""
    cells = W.bubble_sweep(seed=0, n=512)
    lats = _batch(cells, SHORT)
    try:
        for c, g in zip(cells, lats):
            if (c["gamma"], c["M"]) not in UNSTABLE:
                continue
            om = oracle_run(c["params"], c["rho_r"], c["rho_b"], steps=SHORT)
            fin = (_finite(g.moments(check=False)), _finite(om))
            say(f"{c['name']}: finite on the GPU {fin[0]}, in the oracle {fin[1]}")
            assert fin[0] == fin[1], c["name"]
    finally:
        _close(lats)


@pytest.mark.parametrize("variant", ["iso", "mrt_nsc"])
def test_sweep512_variants(variant):
    """The stable cells at viscosity ratio 10, batched, with the
    second-neighbour gradient and with MRT and the correction."""
    extra = dict(gradient="isotropic") if variant == "iso" else dict(collision="mrt", ns_correction=True)
    cells = [c for c in W.bubble_sweep(seed=0, n=512) if c["M"] == 10 and (c["gamma"], c["M"]) not in UNSTABLE]
    lats = _batch([dict(c, params=dict(c["params"], **extra)) for c in cells], LONG)
    try:
        for c, g in zip(cells, lats):
            _check(_name(c, variant), g.moments(check=False))
    finally:
        _close(lats)


def test_slug_4096x256():
    c = W.gravity_slug(seed=0, gamma=10, Re=10)
    with capi.Lattice(c["params"]) as g:
        g.init(c["rho_r"], c["rho_b"])
        g.step(LONG)
        _check("slug", g.moments(check=False))


@pytest.mark.parametrize("storage", ["f16s", "bf16s"])
def test_16bit_full_size_conserves(storage):
    """16-bit storage at the benchmark sizes over LONG steps (the channel
    3 LONG): finite, and
    each colour's mass within 1e-7 of its initial value where it is
    conserved.  The channel's open faces exchange mass, so there only
    finiteness is asserted (a trace colour pushed below zero at the outlet
    once grew without bound in 16-bit storage) and the mass against the FP32
    run is reported."""
    cases = [("slug 4096x256", W.gravity_slug(seed=0, gamma=10, Re=10), None, LONG)]
    ch = W.inlet_outlet(seed=0)
    # long enough to pass the step (about 1600) at which the outlet's trace
    # colour first went negative in 16-bit storage
    cases.append(("channel 8192x512", ch, ch["inlet_color"], 3 * LONG))
    for name, c, color, steps in cases:
        out = {}
        for st in ("f32", storage):
            with capi.Lattice(dict(c["params"], storage=st)) as g:
                g.init(c["rho_r"], c["rho_b"])
                if color is not None:
                    g.set_inlet_color(color)
                g.step(steps)
                out[st] = g.diag(check=False)
        a, b = out["f32"], out[storage]
        ref = (a["mass_r"], a["mass_b"]) if color is not None else (c["rho_r"].sum(), c["rho_b"].sum())
        dr, db = b["mass_r"] / ref[0] - 1, b["mass_b"] / ref[1] - 1
        say(f"{storage} {name}, {steps} steps: {b['n_nonfinite']} non-finite, colour mass {dr:+.1e} {db:+.1e} "
            f"(against {'FP32' if color is not None else 'the initial mass'}), max|u| {b['max_u']:.3e} "
            f"(FP32 {a['max_u']:.3e})")
        assert b["n_nonfinite"] == 0 and a["n_nonfinite"] == 0
        if color is None:
            assert abs(dr) <= 1e-7 and abs(db) <= 1e-7
    cells = [c for c in W.bubble_sweep(seed=0, n=512) if (c["gamma"], c["M"]) not in UNSTABLE]
    lats = _batch(cells, LONG, storage=storage)
    try:
        for c, g in zip(cells, lats):
            d = g.diag(check=False)
            dr, db = d["mass_r"] / c["rho_r"].sum() - 1, d["mass_b"] / c["rho_b"].sum() - 1
            say(f"{storage} {c['name']}: {d['n_nonfinite']} non-finite, colour mass {dr:+.1e} {db:+.1e}")
            assert d["n_nonfinite"] == 0
            assert abs(dr) <= 1e-7 and abs(db) <= 1e-7
    finally:
        _close(lats)
