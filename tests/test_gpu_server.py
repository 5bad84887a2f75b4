"""The solve server on the GPU: each request's result equals the same
lattice stepped alone with lbm_step, bit for bit, whatever else ran in the
same launches; a blowing-up request is isolated."""
import math
import sys

import numpy as np
import pytest

from paper_1903_01168_amd import capi
from paper_1903_01168_amd import serve
from paper_1903_01168_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-server]", *a, file=sys.stderr, flush=True)


def _cases(storage):
    cases = []
    for n, gamma, steps in ((64, 1.0, 37), (128, 10.0, 250), (192, 100.0, 101), (64, 5.0, 400)):
        c = W.bubble_cell(gamma, 10, n // 4, n=n, storage=storage)
        init = serve.init_disk(n / 2, n / 2, n // 4, 1.0, 0.0, 0.0, gamma)
        cases.append((c["params"], init, steps, c["rho_r"], c["rho_b"], None))
    s = W.gravity_slug(nx=320, ny=48, gamma=10, Re=100, g=1e-5, band_lo=40, band_hi=90, storage=storage)
    heavy = s["rho_r"][0] > 0
    edges = [0] + [x for x in range(1, 320) if heavy[x] != heavy[x - 1]]
    cases.append((s["params"], serve.init_bands(edges, 10.0, 1.0), 333, s["rho_r"], s["rho_b"], None))
    p = W.params(nx=130, ny=20, bc_x="open", bc_y="walls", rho0_r=5.0, rho0_b=1.0, tau_r=0.7, tau_b=0.9, A=1e-3,
                 u_in_r=0.01, u_in_b=0.01, p_out=0.48, collision="mrt", storage=storage)
    color = np.where(np.arange(20) < 10, 1, -1).astype(np.int8)
    rr, rb = np.zeros((20, 130)), np.ones((20, 130))
    cases.append((p, serve.init_fields(rr, rb, inlet_color=color), 150, rr, rb, color))
    # requests with the Navier-Stokes correction (stepped by the other kernel
    # variant, in a group of their own) and with a contact angle at the walls
    c = W.bubble_cell(5.0, 2, 24, n=96, collision="mrt", storage=storage)
    c["params"]["ns_correction"] = True
    cases.insert(2, (c["params"], serve.init_disk(48, 48, 24, 1.0, 0.0, 0.0, 5.0), 180, c["rho_r"], c["rho_b"],
                     None))
    d = W.wall_droplet(120.0, n=64, storage=storage)
    cases.append((d["params"], serve.init_fields(d["rho_r"], d["rho_b"]), 222, d["rho_r"], d["rho_b"], None))
    # and one with the second-neighbour gradient (another kernel variant and tile width)
    c = W.bubble_cell(10.0, 10, 20, n=80, storage=storage)
    c["params"]["gradient"] = "isotropic"
    cases.insert(1, (c["params"], serve.init_disk(40, 40, 20, 1.0, 0.0, 0.0, 10.0), 130, c["rho_r"], c["rho_b"],
                     None))
    return cases


def _alone(p, steps, rr, rb, color, init=None):
    with capi.Lattice(p) as g:
        g.init(rr, rb)
        if color is not None:
            g.set_inlet_color(color)
        g.step(steps)
        m = g.moments(check=False)
        if init is not None and init["kind"] == serve.LBM_INIT_DISK:
            R = math.sqrt(g.diag(check=False)["area_r"] / math.pi)
            m["laplace"] = g.diag(circle=(init["cx"], init["cy"], R - 4.0, R + 4.0), check=False)
        return m


@pytest.mark.parametrize("storage,budget_lattices", [("f32", 100), ("f32", 2), ("f16s", 100)])
def test_served_equals_alone(storage, budget_lattices):
    cases = _cases(storage)
    import ctypes as C
    L = capi.load()
    sizes = [L.lbm_bytes_required(C.byref(capi.make_params(c[0]))) for c in cases]
    budget = max(sizes) * budget_lattices
    say(f"serving {len(cases)} requests, storage {storage}, budget {budget} B")
    with serve.Server(budget, max_slots=16, chunk_steps=64, storage=storage) as s:
        ids = [s.enqueue(p, init, steps, keep_fields=True) for p, init, steps, *_ in cases]
        res = [s.wait(i, fields=True) for i in ids]
        st = s.stats()
    assert st["peak_bytes"] <= budget
    for (p, init, steps, rr, rb, color), r in zip(cases, res):
        assert r["status"] == capi.LBM_OK and r["steps_done"] == steps
        ref = _alone(p, steps, rr, rb, color, init)
        for k in ("rho_r", "rho_b", "ux", "uy"):
            assert np.array_equal(r[k], ref[k]), (p["nx"], p["ny"], k)
        if "laplace" in ref:    # Laplace sampling of a bubble request
            for k in ("p_in", "p_out", "n_in", "n_out", "mass_r", "mass_b", "area_r"):
                assert r["diag"][k] == ref["laplace"][k], (p["nx"], k)
            assert r["diag"]["n_in"] > 0 and r["diag"]["n_out"] > 0


def test_unstable_request_is_isolated():
    good = W.static_bubble(n=96, radius=24)
    bad = W.params(nx=64, ny=16, bc_y="walls", tau_r=0.5001, tau_b=0.5001, A=1e-3, gx=5e-2)
    rr, rb, ux, uy = W.random_fields(64, 16, seed=2, umax=0.2)
    with serve.Server(1 << 30, max_slots=8, chunk_steps=64) as s:
        a = s.enqueue(good["params"], serve.init_disk(48, 48, 24, 1.0, 0.0, 0.0, 1.0), 500, keep_fields=True)
        b = s.enqueue(bad, serve.init_fields(rr, rb, ux, uy), 3000)
        ra, rb_ = s.wait(a, fields=True), s.wait(b)
    assert rb_["status"] == capi.LBM_E_UNSTABLE and rb_["diag"]["n_nonfinite"] > 0
    assert ra["status"] == capi.LBM_OK
    ref = _alone(good["params"], 500, good["rho_r"], good["rho_b"], None)
    assert np.array_equal(ra["rho_r"], ref["rho_r"]) and np.array_equal(ra["ux"], ref["ux"])


def test_served_in_cache_groups_equals_alone():
    """Active lattices beyond the cache budget run in groups within a chunk."""
    cases = [W.bubble_cell(g, g, 256, n=1024) for g in (1, 10, 100)]
    with serve.Server(4 << 30, max_slots=8, chunk_steps=64, storage="f32") as s:
        ids = [s.enqueue(c["params"], serve.init_disk(512, 512, 256, 1.0, 0.0, 0.0, float(g)), 150, keep_fields=True)
               for c, g in zip(cases, (1, 10, 100))]
        res = [s.wait(i, fields=True) for i in ids]
    for c, r in zip(cases, res):
        assert r["status"] == capi.LBM_OK and r["steps_done"] == 150
        ref = _alone(c["params"], 150, c["rho_r"], c["rho_b"], None)
        for k in ("rho_r", "rho_b", "ux", "uy"):
            assert np.array_equal(r[k], ref[k]), k
