"""GPU parity: the HIP step (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances (FP32 arithmetic against FP64, tests/bounds.py): after 1000 steps
of the static bubble, max |d rho| / rho <= 1e-5 and max |d u| <= 1e-6
(lattice units).  The other configurations use the same bound, or, where the
flow amplifies rounding (rough random fields, moving interfaces) and that
bound is exceeded, FACTOR times the change that rounding the oracle's stored
populations to FP32 after every step causes.
Exact cases (pure streaming, bounce-back, launch-shape independence,
checkpoint resume) are compared bit for bit.
"""
import sys

import numpy as np
import pytest

from bounds import Bound, oracle_run
from paper_1903_01168_amd import capi
from paper_1903_01168_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-parity]", *a, file=sys.stderr, flush=True)


def _pair(params, rr, rb, ux=None, uy=None, steps=100, orc=None, schedule=None, launch=None):
    """Run the oracle and the GPU on the same inputs; return both moment sets."""
    import oracle
    say(f"pair nx={params['nx']} ny={params['ny']} steps={steps} bc=({params['bc_x']},{params['bc_y']}) "
        f"coll={params['collision']} store={params['storage']}")
    o = oracle.Sim(**params).init(rr, rb, ux, uy)
    with capi.Lattice(params) as g:
        if launch:
            g.set_launch(*launch)
        g.init(rr, rb, ux, uy)
        if schedule:
            done = 0
            for k, (start, col) in enumerate(schedule):
                end = schedule[k + 1][0] if k + 1 < len(schedule) else steps
                end = min(end, steps)
                if end <= start:
                    continue
                cy = np.full(params["ny"], col, dtype=np.int8) if np.isscalar(col) else np.asarray(col, np.int8)
                o.set_inlet_color(cy)
                g.set_inlet_color(cy)
                o.step(end - start)
                g.step(end - start)
                done = end
            assert done == steps
        else:
            o.step(steps)
            g.step(steps)
        gm = g.moments()
    return o.moments(), gm


def _errors(om, gm):
    rho_o = om["rho_r"] + om["rho_b"]
    rho_g = gm["rho_r"] + gm["rho_b"]
    drho = np.max(np.abs(rho_g - rho_o) / rho_o)
    dr = max(np.max(np.abs(gm["rho_r"] - om["rho_r"])), np.max(np.abs(gm["rho_b"] - om["rho_b"])))
    du = max(np.max(np.abs(gm["ux"] - om["ux"])), np.max(np.abs(gm["uy"] - om["uy"])))
    return drho, dr, du


def test_pure_streaming_bit_exact():
    """One colour, no relaxation and no surface tension: k steps are an exact shift."""
    nx, ny = 300, 37
    p = W.params(nx=nx, ny=ny, tau_r=1e30, tau_b=1e30, A=0.0)
    rng = np.random.default_rng(0)
    pops = np.zeros((2, 9, ny, nx))
    pops[0] = rng.uniform(0.05, 0.3, (9, ny, nx)).astype(np.float32)
    with capi.Lattice(p) as g:
        g.set_pops(pops)
        g.step(3)
        got = g.get_pops()
    cx = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    cy = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    for i in range(9):
        ref = np.roll(np.roll(pops[0, i], 3 * cy[i], 0), 3 * cx[i], 1)
        assert np.array_equal(got[0, i], ref), f"direction {i}"
    assert np.all(got[1] == 0)


def test_bounce_back_bit_exact():
    nx, ny = 130, 6
    p = W.params(nx=nx, ny=ny, bc_y="walls", tau_r=1e30, tau_b=1e30, A=0.0)
    rng = np.random.default_rng(1)
    pops = np.zeros((2, 9, ny, nx))
    pops[0] = rng.uniform(0.05, 0.3, (9, ny, nx)).astype(np.float32)
    with capi.Lattice(p) as g:
        g.set_pops(pops)
        g.step(1)
        got = g.get_pops()[0]
    for i, o in ((2, 4), (5, 7), (6, 8)):
        assert np.array_equal(got[i, 0], pops[0, o, 0])
    for i, o in ((4, 2), (7, 5), (8, 6)):
        assert np.array_equal(got[i, ny - 1], pops[0, o, ny - 1])


def test_static_bubble_1000_steps():
    """64 x 64 bubble, density and viscosity ratio 1, A = 1e-3, beta = 0.7."""
    c = W.static_bubble()
    om, gm = _pair(c["params"], c["rho_r"], c["rho_b"], steps=1000)
    drho, dr, du = _errors(om, gm)
    say(f"static bubble 1000 steps: max drho/rho={drho:.3e} max du={du:.3e}")
    assert drho <= 1e-5
    assert du <= 1e-6


CASES = {
    "periodic_ratio5": dict(nx=300, ny=40, rho0_r=1.0, rho0_b=5.0, tau_r=0.7, tau_b=1.1, A=1e-3),
    "walls_force": dict(nx=200, ny=33, bc_y="walls", rho0_r=1.0, rho0_b=3.0, tau_r=0.8, tau_b=0.6, A=1e-3,
                        gx=1e-5, gy=-2e-6),
    "mrt_walls": dict(nx=130, ny=29, bc_y="walls", collision="mrt", rho0_r=1.0, rho0_b=10.0, tau_r=0.9,
                      tau_b=0.6, A=1e-3, gx=1e-5),
    "sigma_mode": dict(nx=256, ny=48, rho0_r=1.0, rho0_b=2.0, tau_r=0.6, tau_b=1.5, sigma=4e-4),
    "narrow_periodic": dict(nx=70, ny=5, rho0_r=1.0, rho0_b=1.0, tau_r=1.0, tau_b=0.75, A=2e-3, beta=0.99),
    # free-slip walls (Sec. 2.5 item 1), both sides, and no-slip bottom with free-slip top
    "freeslip_force": dict(nx=150, ny=21, bc_y="freeslip", rho0_r=1.0, rho0_b=3.0, tau_r=0.8, tau_b=0.6,
                           A=1e-3, gx=1e-5, gy=-2e-6),
    "slip_top_mrt": dict(nx=110, ny=17, bc_y="slip_top", collision="mrt", rho0_r=1.0, rho0_b=4.0, tau_r=0.9,
                         tau_b=0.7, A=1e-3, gx=1e-5),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_parity_cases(name):
    kw = dict(CASES[name])
    p = W.params(**kw)
    rr, rb, ux, uy = W.random_fields(p["nx"], p["ny"], seed=7, rho0_r=p["rho0_r"], rho0_b=p["rho0_b"],
                                     umax=0.01)
    om, gm = _pair(p, rr, rb, ux, uy, steps=200)
    _, dr, _ = _errors(om, gm)
    say(f"{name}: drho_k={dr:.3e}")
    Bound(om, lambda: oracle_run(p, rr, rb, ux, uy, steps=200, round_f32=True), tag="gpu-parity").check(name, gm)


SHAPES = {
    # bubble sweep cell (density ratio 10, viscosity ratio 10), 128 x 128, sigma-mode
    "bubble_g10": lambda: W.bubble_cell(10, 10, 40, n=128),
    "bubble_g100_mrt": lambda: W.bubble_cell(100, 10, 30, n=96, collision="mrt"),
    # gravity slug: walls, body force, density ratio 10
    "slug_g10": lambda: W.gravity_slug(nx=512, ny=64, gamma=10, Re=100, g=1e-6, band_lo=60, band_hi=150),
}


@pytest.mark.parametrize("name", sorted(SHAPES))
def test_parity_shapes(name):
    """1000 steps of bubble and slug shapes.  Bound: the fixed FP32 bound, or,
    where the flow itself amplifies rounding (moving interfaces), FACTOR times
    the change that FP32 storage rounding alone causes in the oracle; the
    ratio of the GPU error to that change is printed for every shape."""
    c = SHAPES[name]()
    steps = 1000
    om, gm = _pair(c["params"], c["rho_r"], c["rho_b"], steps=steps)
    _, dr, _ = _errors(om, gm)
    say(f"{name}: drho_k={dr:.3e}")
    Bound(om, lambda: oracle_run(c["params"], c["rho_r"], c["rho_b"], steps=steps, round_f32=True),
          tag="gpu-parity").check(name, gm, always_ratio=True)


def _stratified_channel(nx, ny, gamma, heavy_frac=0.8, u_heavy=0.03, u_light=0.005):
    """The paper's inlet/outlet set-up: heavy fluid (red) in the lower rows of
    the inlet, light (blue) above, the heavy one injected faster."""
    p = W.params(nx=nx, ny=ny, bc_x="open", bc_y="walls", rho0_r=float(gamma), rho0_b=1.0, tau_r=0.6,
                 tau_b=0.8, A=1e-3, u_in_r=u_heavy, u_in_b=u_light, p_out=0.48)
    hrows = int(round(heavy_frac * ny))
    color = np.where(np.arange(ny) < hrows, 1, -1).astype(np.int8)
    rr = np.zeros((ny, nx))
    rb = np.ones((ny, nx))
    rr[:hrows] = gamma
    rb[:hrows] = 0.0
    return p, rr, rb, color


def test_parity_open_channel_stratified():
    """Velocity inlet / pressure outlet / walls, density ratio 5 (Sec. 5.2 set-up)."""
    p, rr, rb, color = _stratified_channel(160, 24, 5.0)
    om, gm = _pair(p, rr, rb, steps=400, schedule=[(0, color)])
    drho, dr, du = _errors(om, gm)
    say(f"open channel stratified: drho/rho={drho:.3e} drho_k={dr:.3e} du={du:.3e}")
    assert drho <= 1e-5
    assert du <= 1e-6


def test_parity_open_channel_switching():
    """Inlet colour switching between red and blue (density ratio 1)."""
    p = W.params(nx=160, ny=24, bc_x="open", bc_y="walls", tau_r=0.7, tau_b=1.0, A=1e-3, u_in_r=0.01,
                 u_in_b=0.01, p_out=0.48)
    rr = np.zeros((24, 160))
    rb = np.ones((24, 160))
    sched = [(0, 1), (80, -1), (150, 1)]
    om, gm = _pair(p, rr, rb, steps=300, schedule=sched)
    drho, dr, du = _errors(om, gm)
    say(f"open channel switching: drho/rho={drho:.3e} drho_k={dr:.3e} du={du:.3e}")
    assert drho <= 1e-5
    assert du <= 1e-6


# (threads per workgroup, strip rows, step flavour: True block exchange,
# False halo lanes, None planned)
LAUNCH_SHAPES = ((256, 0, None), (64, 1, False), (128, 7, False), (64, 45, False), (256, 3, False),
                 (64, 1, True), (128, 7, True), (256, 3, True), (512, 5, True), (1024, 2, True), (1024, 16, True))


def _launch_shapes_agree(p, rr, rb, ux, uy, steps=50, color=None):
    ref = None
    for tx, strip, xch in LAUNCH_SHAPES:
        with capi.Lattice(p) as g:
            g.set_launch(tx, strip, exchange=xch)
            g.init(rr, rb, ux, uy)
            if color is not None:
                g.set_inlet_color(color)
            g.step(steps)
            pops = g.get_pops()
        if ref is None:
            ref = pops
        else:
            assert np.array_equal(pops, ref), (tx, strip, xch)


@pytest.mark.parametrize("storage", ["f32", "f16s", "bf16s"])
def test_launch_shape_independence(storage):
    """Workgroup width, strip height and step flavour change only who computes
    a node, not what: halo lanes, or whole blocks per wavefront with one
    wavefront gathering its own halo nodes or several exchanging their edge
    columns through LDS; strips of one row to the whole height."""
    p = W.params(nx=300, ny=45, bc_y="walls", rho0_r=1.0, rho0_b=4.0, tau_r=0.7, tau_b=0.9, A=1e-3,
                 gx=1e-6, storage=storage)
    rr, rb, ux, uy = W.random_fields(300, 45, seed=3, rho0_r=1.0, rho0_b=4.0)
    _launch_shapes_agree(p, rr, rb, ux, uy)


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_launch_shape_independence_corrected_open(storage):
    """The same with MRT and the Navier-Stokes correction (Q exchanged beside
    the colour field) on an open channel with free-slip walls, whose outlet
    column is a halo node of the block before it (130 = 2 x 64 + 2)."""
    p = W.params(nx=130, ny=37, bc_x="open", bc_y="freeslip", collision="mrt", ns_correction=True,
                 rho0_r=5.0, rho0_b=1.0, tau_r=0.7, tau_b=0.9, A=1e-3, u_in_r=0.01, u_in_b=0.01, p_out=0.48,
                 storage=storage)
    rr, rb, _, _ = W.random_fields(130, 37, seed=8, rho0_r=5.0, rho0_b=1.0)
    color = np.where(np.arange(37) < 20, 1, -1).astype(np.int8)
    _launch_shapes_agree(p, rr, rb, None, None, color=color)


def test_graph_replay_matches_launches():
    """lbm_step(n) with graph replays equals n single-step calls bit for bit."""
    c = W.static_bubble(n=96, radius=20)
    with capi.Lattice(c["params"]) as a, capi.Lattice(c["params"]) as b:
        a.init(c["rho_r"], c["rho_b"])
        b.init(c["rho_r"], c["rho_b"])
        a.step(203)
        for _ in range(203):
            b.step(1)
        assert np.array_equal(a.get_pops(), b.get_pops())


def test_checkpoint_resume_bit_exact():
    c = W.static_bubble()
    with capi.Lattice(c["params"]) as a:
        a.init(c["rho_r"], c["rho_b"])
        a.step(37)
        blob = a.save_state()
        a.step(100)
        ref = a.get_pops()
    with capi.Lattice(c["params"]) as b:
        b.load_state(blob)
        assert b.steps_done == 37
        b.step(100)
        assert np.array_equal(b.get_pops(), ref)


def test_diag_consistency():
    c = W.static_bubble()
    with capi.Lattice(c["params"]) as g:
        g.init(c["rho_r"], c["rho_b"])
        g.step(10)
        m = g.moments()
        d = g.diag(circle=(32.0, 32.0, 12.0, 20.0))
    assert d["mass_r"] == pytest.approx(m["rho_r"].sum(), rel=1e-6)
    assert d["mass_b"] == pytest.approx(m["rho_b"].sum(), rel=1e-6)
    assert d["max_u"] == pytest.approx(np.hypot(m["ux"], m["uy"]).max(), rel=1e-5)
    y, x = np.mgrid[0:64, 0:64]
    r = np.hypot(x + 0.5 - 32, y + 0.5 - 32)
    assert d["n_in"] == int((r < 12).sum()) and d["n_out"] == int((r > 20).sum())
    assert d["p_in"] == pytest.approx(m["p"][r < 12].mean(), rel=1e-6)
    assert d["n_nonfinite"] == 0 and d["step"] == 10


def test_unstable_reported():
    """A run driven far beyond the stable range reports LBM_E_UNSTABLE."""
    p = W.params(nx=64, ny=16, bc_y="walls", tau_r=0.5001, tau_b=0.5001, A=1e-3, gx=5e-2)
    rr, rb, ux, uy = W.random_fields(64, 16, seed=2, umax=0.2)
    with capi.Lattice(p) as g:
        g.init(rr, rb, ux, uy)
        g.step(3000)
        d = g.diag(check=False)
        assert d["n_nonfinite"] > 0
        with pytest.raises(capi.LbmError) as e:
            g.moments()
        assert e.value.code == capi.LBM_E_UNSTABLE


@pytest.mark.parametrize("storage", ["f32", "bf16s"])
def test_batch_bit_identical_to_single(storage):
    """One batched launch per step over different lattices gives each lattice
    exactly the result of stepping it alone."""
    cases = []
    c = W.static_bubble(n=96, radius=20, storage=storage)
    cases.append((c["params"], c["rho_r"], c["rho_b"], None, None))
    c = W.gravity_slug(nx=300, ny=40, gamma=10, Re=100, band_lo=40, band_hi=80, g=1e-5, storage=storage)
    cases.append((c["params"], c["rho_r"], c["rho_b"], None, None))
    p = W.params(nx=130, ny=20, bc_x="open", bc_y="walls", rho0_r=5.0, rho0_b=1.0, tau_r=0.7, tau_b=0.9,
                 A=1e-3, u_in_r=0.01, u_in_b=0.01, p_out=0.48, collision="mrt", storage=storage)
    cases.append((p, np.zeros((20, 130)), np.ones((20, 130)), None, None))
    alone = []
    for prm, rr, rb, ux, uy in cases:
        say(f"alone {prm['nx']}x{prm['ny']} {storage}")
        with capi.Lattice(prm) as g:
            g.init(rr, rb, ux, uy)
            g.step(150)
            alone.append(g.get_pops())
    lats = [capi.Lattice(prm) for prm, *_ in cases]
    for lat, (prm, rr, rb, ux, uy) in zip(lats, cases):
        lat.init(rr, rb, ux, uy)
    say(f"batch of {len(lats)} {storage}")
    with capi.Batch(lats) as b:
        b.step(150)
        got = [lat.get_pops() for lat in lats]
    for a, g in zip(alone, got):
        assert np.array_equal(a, g)
    for lat in lats:
        lat.close()


def _open_case(bc_y="walls"):
    p, rr, rb, color = _stratified_channel(96, 20, 5.0)
    return dict(params=dict(p, bc_y=bc_y), rho_r=rr, rho_b=rb, color=color)


ONE_STEP = {
    "open_g5": _open_case,
    "open_g5_freeslip": lambda: _open_case("freeslip"),
    "bubble_g10": lambda: W.bubble_cell(10, 10, 20, n=64),
    "bubble_g10_mrt": lambda: W.bubble_cell(10, 1, 20, n=64, collision="mrt"),
    "slug_g10": lambda: W.gravity_slug(nx=256, ny=32, gamma=10, Re=100, g=1e-5, band_lo=40, band_hi=90),
    "bubble_g1": lambda: W.static_bubble(n=64, radius=16),
    "droplet_wet120": lambda: W.wall_droplet(120.0, n=64),
}


@pytest.mark.parametrize("name", sorted(ONE_STEP))
def test_one_step_from_oracle_state(name):
    """One GPU step from a developed oracle state equals one oracle step up to
    FP32 rounding: |dN| <= 2e-6 rho0_max for every population."""
    import oracle
    c = ONE_STEP[name]()
    p = c["params"]
    o = oracle.Sim(**p).init(c["rho_r"], c["rho_b"])
    if "color" in c:
        o.set_inlet_color(c["color"])
    o.step(300)
    state = o.get_pops()
    o.step(1)
    ref = o.get_pops()
    with capi.Lattice(p) as g:
        if "color" in c:
            g.set_inlet_color(c["color"])
        g.set_pops(state)
        g.step(1)
        got = g.get_pops()
    err = np.abs(got - ref)
    k, i, y, x = np.unravel_index(np.argmax(err), err.shape)
    scale = max(p["rho0_r"], p["rho0_b"])
    say(f"one step {name}: max |dN| = {err.max():.3e} at colour {k} dir {i} (x={x}, y={y}); "
        f"ref {ref[k, i, y, x]:.6e} got {got[k, i, y, x]:.6e}; state rho_r={state[0, :, y, x].sum():.4e} "
        f"rho_b={state[1, :, y, x].sum():.4e}")
    d = got - ref
    say(f"   mass bias per step: red {d[0].sum():.3e} blue {d[1].sum():.3e} (of {ref[0].sum():.4e}, "
        f"{ref[1].sum():.4e}); state mass red {state[0].sum():.4e} blue {state[1].sum():.4e}")
    for kk in range(2):
        for ii in range(9):
            say(f"   colour {kk} dir {ii}: max {err[kk, ii].max():.3e} mean {d[kk, ii].mean():+.3e}")
    assert err.max() <= 2e-6 * scale


def test_batch_cache_groups_bit_identical():
    """Lattices whose buffers exceed the cache budget are stepped in groups
    that take turns (256 steps each); every lattice still gets exactly the
    result of stepping it alone."""
    cases = [W.bubble_cell(g, g, 256, n=1024) for g in (1, 10, 100)]
    alone = []
    for c in cases:
        with capi.Lattice(c["params"]) as g:
            g.init(c["rho_r"], c["rho_b"])
            g.step(300)
            alone.append(g.get_pops())
    lats = [capi.Lattice(c["params"]) for c in cases]
    for lat, c in zip(lats, cases):
        lat.init(c["rho_r"], c["rho_b"])
    with capi.Batch(lats) as b:
        assert b.groups >= 2
        say(f"batch of 3 x 1024^2 FP32 in {b.groups} cache groups")
        b.step(300)
    try:
        for lat, ref in zip(lats, alone):
            assert lat.steps_done == 300
            assert np.array_equal(lat.get_pops(), ref)
    finally:
        for lat in lats:
            lat.close()


def test_batch_lanes_bit_identical():
    """Groups of unequal size stepped two at a time on two streams, in calls
    of uneven length (partial rounds; the group that straddles the two
    streams' halves split between them), with the contexts' own streams used
    right after each call (moments) and before the next (setting an inlet
    colour is not needed: a population write instead): every lattice equals
    itself stepped alone, bit for bit."""
    cases = [W.bubble_cell(g, m, 40, n=n) for g, m, n in ((1, 1, 192), (10, 1, 256), (100, 10, 128), (5, 2, 320),
                                                          (2, 20, 160))]
    kicks = {1: 0.999}                       # after the second call, lattice 1's populations are scaled
    calls = (1, 63, 300, 7, 256)
    alone = []
    for i, c in enumerate(cases):
        with capi.Lattice(c["params"]) as g:
            g.init(c["rho_r"], c["rho_b"])
            for j, n in enumerate(calls):
                g.step(n)
                if j == 1 and i in kicks:
                    g.set_pops(g.get_pops() * kicks[i])
            alone.append(g.get_pops())
    lats = [capi.Lattice(c["params"]) for c in cases]
    for lat, c in zip(lats, cases):
        lat.init(c["rho_r"], c["rho_b"])
    try:
        with capi.Batch(lats) as b:
            assert b.groups >= 2
            say(f"batch of {len(cases)} lattices in {b.groups} groups on two streams")
            for j, n in enumerate(calls):
                b.step(n)
                m = [lat.moments() for lat in lats]      # on the contexts' streams
                assert all(np.isfinite(x["rho_r"]).all() for x in m)
                if j == 1:
                    for i, f in kicks.items():
                        lats[i].set_pops(lats[i].get_pops() * f)
            for lat, ref in zip(lats, alone):
                assert lat.steps_done == sum(calls)
                assert np.array_equal(lat.get_pops(), ref)
    finally:
        for lat in lats:
            lat.close()
