"""Pins of the seeded workload recipes (host logic, no GPU)."""
import math
import os

import numpy as np
import pytest

from paper_1903_01168_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_periodic_slug_tau_table():
    """Re -> (tau_g, tau_l) of the paper's periodic slug case is reproduced by
    the recipe used for the gravity-slug workload (nu_g = nu_l * gamma / 2)."""
    rows = np.loadtxt(os.path.join(GOLD, "periodic_slug_tau.txt"))
    g, H, gamma = 5.0e-7, 91, 5.0
    for Re, tau_g, tau_l in rows:
        nu_l = math.sqrt(g * H ** 3 / (8.0 * Re))
        assert W.tau_from_nu(nu_l) == pytest.approx(tau_l, abs=6e-4)
        assert W.tau_from_nu(nu_l * gamma / 2.0) == pytest.approx(tau_g, abs=1.1e-3)
        case = W.gravity_slug(nx=64, ny=H, gamma=gamma, Re=Re, g=g, band_lo=10, band_hi=20)
        assert case["params"]["tau_r"] == pytest.approx(tau_l, abs=6e-4)
        assert case["params"]["tau_b"] == pytest.approx(tau_g, abs=1.1e-3)


def test_static_bubble_geometry():
    c = W.static_bubble()
    rr, rb = c["rho_r"], c["rho_b"]
    assert rr.shape == (64, 64)
    assert np.all((rr == 1) ^ (rb == 1)) and np.all(rr + rb == 1)
    # cell-centred disk: symmetric under transposition and mirrors
    assert np.array_equal(rr, rr.T) and np.array_equal(rr, rr[::-1]) and np.array_equal(rr, rr[:, ::-1])
    assert abs(rr.sum() - math.pi * 256) < 40


def test_bubble_sweep_seeded():
    a = W.bubble_sweep(seed=0, n=64)
    b = W.bubble_sweep(seed=0, n=64)
    c = W.bubble_sweep(seed=1, n=64)
    assert [x["radius"] for x in a] == [x["radius"] for x in b]
    assert [x["radius"] for x in a] != [x["radius"] for x in c]
    assert len(a) == 9
    for cell in a:
        p = cell["params"]
        assert 64 <= cell["radius"] <= 128
        assert min(p["tau_r"], p["tau_b"]) == pytest.approx(0.6)
        nu_l, nu_h = (p["tau_r"] - 0.5) / 3, (p["tau_b"] - 0.5) / 3
        assert nu_h / nu_l == pytest.approx(cell["M"] / cell["gamma"])
        assert p["rho0_b"] == cell["gamma"] and p["rho0_r"] == 1.0


def test_slug_bands_and_schedule():
    rng = np.random.default_rng(0)
    heavy = W.slug_bands(4096, rng)
    edges = np.flatnonzero(np.diff(heavy.astype(int))) + 1
    bands = np.diff(np.concatenate([[0], edges, [4096]]))
    assert len(bands) % 2 == 0 and len(bands) >= 2
    assert np.all(bands[:-1] >= 200) and np.all(bands[:-1] <= 600)
    sched = W.inlet_schedule(20000, seed=3)
    starts = [s for s, _ in sched]
    assert starts[0] == 0 and all(300 <= b - a <= 800 for a, b in zip(starts, starts[1:]))
    assert all(c1 == -c2 for (_, c1), (_, c2) in zip(sched, sched[1:]))


def test_serve_trace_recipe():
    a = W.serve_trace(seed=3, n=300)
    b = W.serve_trace(seed=3, n=300)
    assert [(r["kind"], r["nodes"], r["steps"], r["gamma"]) for r in a] == \
        [(r["kind"], r["nodes"], r["steps"], r["gamma"]) for r in b]
    kinds = {r["kind"] for r in a}
    assert kinds == {"bubble", "slug"}
    for r in a:
        p = r["params"]
        assert 64 * 64 // 4 <= r["nodes"] <= 1024 * 1024 and r["nodes"] == p["nx"] * p["ny"]
        assert 1000 <= r["steps"] <= 50000 and r["gap"] > 0
        assert r["gamma"] in (W.SERVE_GAMMAS if r["kind"] == "bubble" else W.SERVE_SLUG_GAMMAS)
        assert p["storage"] == "f16s"
        if r["kind"] == "bubble":
            assert p["nx"] == p["ny"] and p["nx"] % 64 == 0 and p["bc_y"] == "periodic"
            assert r["geo"]["radius"] == p["nx"] / 4 and p["rho0_b"] == r["gamma"]
        else:
            assert p["nx"] == 16 * p["ny"] and p["ny"] % 16 == 0 and p["bc_y"] == "walls"
            e = r["geo"]["edges"]
            assert e[0] == 0 and len(e) % 2 == 0 and all(x < y for x, y in zip(e, e[1:])) and e[-1] < p["nx"]


def test_geo_fields_match_generators():
    c = W.bubble_cell(100, 10, 30, n=128)
    geo = dict(kind="disk", cx=64.0, cy=64.0, radius=30.0, rho_r_in=1.0, rho_b_in=0.0, rho_r_out=0.0,
               rho_b_out=100.0)
    rr, rb = W.geo_fields(geo, 128, 128)
    assert np.array_equal(rr, c["rho_r"]) and np.array_equal(rb, c["rho_b"])
    s = W.gravity_slug(seed=5, nx=1024, ny=32, gamma=10)
    edges = W.slug_edges(1024, np.random.default_rng(5))
    rr, rb = W.geo_fields(dict(kind="bands", edges=edges, rho_band_r=10.0, rho_band_b=1.0), 1024, 32)
    assert np.array_equal(rr, s["rho_r"]) and np.array_equal(rb, s["rho_b"])
