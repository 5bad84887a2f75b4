"""Edge cases of the GPU step against the FP64 oracle: degenerate lattice
sizes (one node, one row, one column), widths around the 64-column
wavefront block and the workgroup span, walls on one- and two-row channels,
open channels from two columns wide to widths around a block (the outlet
column then one of the halo nodes of the block next to it), one fluid
only, no surface tension, recolouring
strength beta at both ends of its range, zero steps, and the largest lattices the
ABI accepts.  Bounds (tests/bounds.py):
the FP32 bound of the static bubble (max |d rho| / rho <= 1e-5, max |d u| <= 1e-6);
the rough random fields of the size cases are compared population by
population over one step from a developed oracle state (2e-6 rho0_max: one
step injects about 24 ulps, 1.4e-6 relative) and over their first 20 steps
to the fixed bound or, where it is exceeded, FACTOR times the oracle's own
sensitivity to FP32 storage rounding."""
import sys

import numpy as np
import pytest

import oracle
from bounds import Bound, oracle_run
from paper_1903_01168_amd import capi
from paper_1903_01168_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 60
SHORT = 20


def say(*a):
    print("[gpu-edges]", *a, file=sys.stderr, flush=True)


def _run(p, rr, rb, ux=None, uy=None, steps=STEPS, color=None, launch=None):
    s = oracle.Sim(**p).init(rr, rb, ux, uy)
    if color is not None:
        s.set_inlet_color(color)
    s.step(steps)
    om = s.moments()
    with capi.Lattice(p) as g:
        if launch:
            g.set_launch(*launch)
        g.init(rr, rb, ux, uy)
        if color is not None:
            g.set_inlet_color(color)
        g.step(steps)
        gm = g.moments()
    return om, gm


def _errors(om, gm):
    rho_o = om["rho_r"] + om["rho_b"]
    drho = float(np.max(np.abs(gm["rho_r"] + gm["rho_b"] - rho_o) / rho_o))
    du = float(max(np.max(np.abs(gm["ux"] - om["ux"])), np.max(np.abs(gm["uy"] - om["uy"]))))
    return drho, du


SIZES = [(1, 1, "periodic"), (1, 9, "periodic"), (9, 1, "periodic"), (2, 2, "periodic"), (5, 1, "walls"),
         (5, 2, "walls"), (1, 6, "walls"), (59, 7, "periodic"), (60, 7, "periodic"), (61, 7, "walls"),
         (119, 5, "periodic"), (121, 5, "walls"), (241, 3, "periodic"), (300, 1, "walls"),
         (1, 4, "freeslip"), (7, 1, "freeslip"), (61, 2, "slip_top"), (125, 6, "freeslip"),
         (63, 5, "walls"), (64, 5, "periodic"), (65, 4, "freeslip"), (127, 3, "periodic"), (128, 3, "walls"),
         (129, 4, "slip_top"), (130, 2, "walls"), (257, 3, "periodic")]


@pytest.mark.parametrize("nx,ny,bcy", SIZES)
def test_degenerate_and_ragged_sizes(nx, ny, bcy):
    """Every population after one GPU step from the oracle's state at step
    STEPS - 1 within 2e-6 rho0_max (a wrong neighbour, wrap or wall would
    show at O(1)); and the fields after SHORT steps from the initial rough
    field within the parity bound (Bound).  (Over STEPS steps some of these
    rough fields amplify any rounding difference by two orders of magnitude
    at once, e.g. 241 x 3: 4e-7 at step 20, 2.5e-5 at step 40, with every
    single step at FP32 level, so the multi-step comparison stops earlier.)"""
    p = W.params(nx=nx, ny=ny, bc_y=bcy, rho0_r=1.0, rho0_b=3.0, tau_r=0.7, tau_b=0.9, A=1e-3,
                 gx=1e-5 if bcy != "periodic" else 0.0)
    rr, rb, ux, uy = W.random_fields(nx, ny, seed=nx * 31 + ny, rho0_r=1.0, rho0_b=3.0)
    o = oracle.Sim(**p).init(rr, rb, ux, uy)
    o.step(STEPS - 1)
    state = o.get_pops()
    o.step(1)
    ref = o.get_pops()
    om = oracle_run(p, rr, rb, ux, uy, steps=SHORT)
    bound = Bound(om, lambda: oracle_run(p, rr, rb, ux, uy, steps=SHORT, round_f32=True), tag="gpu-edges")
    for launch in ((64, 0), (256, 1), (1024, 2)):
        with capi.Lattice(p) as g:
            g.set_launch(*launch)
            g.set_pops(state)
            g.step(1)
            err = float(np.abs(g.get_pops() - ref).max())
        _, gm = _run(p, rr, rb, ux, uy, steps=SHORT, launch=launch)
        say(f"{nx}x{ny} {bcy} tile {launch[0]}: one step max |dN| {err:.2e}")
        assert err <= 2e-6 * 3.0
        bound.check(f"{nx}x{ny} {bcy} tile {launch[0]}, {SHORT} steps", gm)


@pytest.mark.parametrize("nx", [2, 63, 64, 65, 66, 129])
def test_narrow_open_channel(nx):
    p = W.params(nx=nx, ny=6, bc_x="open", bc_y="walls", rho0_r=1.0, rho0_b=2.0, tau_r=0.8, tau_b=0.9, A=1e-3,
                 u_in_r=0.01, u_in_b=0.01, p_out=0.48)
    color = np.array([1, 1, 1, -1, -1, -1], dtype=np.int8)
    rr = np.where(color[:, None] > 0, 1.0, 0.0) * np.ones((1, nx))
    rb = np.where(color[:, None] > 0, 0.0, 2.0) * np.ones((1, nx))
    for launch in ((64, 0), (1024, 1)):
        drho, du = _errors(*_run(p, rr, rb, color=color, launch=launch))
        say(f"open {nx}x6 tile {launch[0]}: drho/rho {drho:.2e} du {du:.2e}")
        assert drho <= 1e-5 and du <= 1e-6


@pytest.mark.parametrize("storage", ["f32", "f16s", "bf16s"])
def test_one_fluid_only(storage):
    """Blue absent everywhere: it stays exactly zero in every storage, and the
    red fluid follows the single-phase oracle."""
    p = W.params(nx=100, ny=20, bc_y="walls", tau_r=0.8, tau_b=0.8, A=1e-3, gx=1e-5, storage=storage)
    rr = np.ones((20, 100))
    rb = np.zeros((20, 100))
    om, gm = _run(p, rr, rb)
    assert np.all(gm["rho_b"] == 0.0)
    if storage == "f32":
        drho, du = _errors(om, gm)
        assert drho <= 1e-5 and du <= 1e-6


@pytest.mark.parametrize("A,beta", [(0.0, 0.7), (1e-3, 0.0), (1e-3, 1.0)])
def test_surface_tension_and_recolouring_limits(A, beta):
    c = W.static_bubble(n=48, radius=12)
    p = dict(c["params"], A=A, beta=beta)
    drho, du = _errors(*_run(p, c["rho_r"], c["rho_b"], steps=300))
    say(f"A={A} beta={beta}: drho/rho {drho:.2e} du {du:.2e}")
    assert drho <= 1e-5 and du <= 1e-6


def test_zero_steps():
    """lbm_step(0) changes nothing; the moments at step 0 (of the pulled
    initial populations) agree with the oracle's."""
    c = W.static_bubble(n=40, radius=10)
    with capi.Lattice(c["params"]) as g:
        g.init(c["rho_r"], c["rho_b"])
        before = g.get_pops()
        g.step(0)
        assert g.steps_done == 0 and np.array_equal(g.get_pops(), before)
        gm = g.moments()
    om = oracle.Sim(**c["params"]).init(c["rho_r"], c["rho_b"], None, None).moments()
    drho, du = _errors(om, gm)
    assert drho <= 1e-6 and du <= 1e-7


def test_maximum_size_fp32():
    """The largest FP32 lattice the ABI accepts at 65536 columns (65536 x 1820:
    a colour half of a buffer just below 4 GiB, so the last rows use the
    largest 32-bit offsets; the planned block-exchange launch): a stratified
    state uniform in x under a body force stays uniform in x bit for bit over
    20 steps, and its columns match the oracle on a 64-column lattice."""
    nx, ny, steps = 65536, 1820, 20
    kw = dict(bc_y="walls", rho0_r=1.0, rho0_b=3.0, tau_r=0.8, tau_b=0.9, A=1e-3, gx=1e-5)
    band = ((np.arange(ny) // 91) % 2 == 0)[:, None]          # 20 bands, 19 interfaces
    col_r, col_b = np.where(band, 1.0, 0.0), np.where(band, 0.0, 3.0)
    with capi.Lattice(W.params(nx=nx, ny=ny, **kw)) as g:
        g.init(np.ascontiguousarray(np.broadcast_to(col_r, (ny, nx))),
               np.ascontiguousarray(np.broadcast_to(col_b, (ny, nx))))
        g.step(steps)
        gm = g.moments()
    for k in ("rho_r", "rho_b", "ux", "uy"):
        assert np.array_equal(gm[k], np.broadcast_to(gm[k][:, :1], gm[k].shape)), k
    o = oracle.Sim(**W.params(nx=64, ny=ny, **kw)).init(np.repeat(col_r, 64, axis=1), np.repeat(col_b, 64, axis=1),
                                                        None, None)
    o.step(steps)
    om = o.moments()
    keys = ("rho_r", "rho_b", "ux", "uy")
    drho, du = _errors({k: om[k][:, :1] for k in keys}, {k: gm[k][:, :1] for k in keys})
    say(f"{nx}x{ny} FP32: x-uniform bit for bit; column against the oracle drho/rho {drho:.2e} du {du:.2e}")
    assert drho <= 1e-5 and du <= 1e-6


@pytest.mark.parametrize("storage", ["f16s", "bf16s"])
def test_maximum_size_16bit(storage):
    """The largest 16-bit lattice the ABI accepts at 65536 columns (65536 x
    3276): finite after 20 steps, and each colour's mass within 1e-7 (the
    dither depends on the node's position, so the state is not x-uniform)."""
    nx, ny, steps = 65536, 3276, 20
    band = ((np.arange(ny) // 91) % 2 == 0)[:, None]
    rr = np.ascontiguousarray(np.broadcast_to(np.where(band, 1.0, 0.0), (ny, nx)))
    rb = np.ascontiguousarray(np.broadcast_to(np.where(band, 0.0, 3.0), (ny, nx)))
    m0 = (rr.sum(), rb.sum())
    p = W.params(nx=nx, ny=ny, bc_y="walls", rho0_r=1.0, rho0_b=3.0, tau_r=0.8, tau_b=0.9, A=1e-3, gx=1e-5,
                 storage=storage)
    with capi.Lattice(p) as g:
        g.init(rr, rb)
        del rr, rb
        g.step(steps)
        d = g.diag(check=False)
    dr, db = d["mass_r"] / m0[0] - 1, d["mass_b"] / m0[1] - 1
    say(f"{nx}x{ny} {storage}: {d['n_nonfinite']} non-finite, colour mass {dr:+.1e} {db:+.1e}")
    assert d["n_nonfinite"] == 0
    assert abs(dr) <= 1e-7 and abs(db) <= 1e-7
