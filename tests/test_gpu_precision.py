"""16-bit population storage against FP32 storage and the FP64 oracle:
colour-mass conservation, spurious currents and the Laplace pressure jump of
converged static bubbles (Sec. 4 static bubble tests; the 16-bit formats are
this implementation's storage, not the paper's)."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1903_01168_amd import capi
from paper_1903_01168_amd import workloads as W

pytestmark = pytest.mark.gpu


# FP32 populations keep colour mass only up to rounding: the FP64 oracle whose
# populations are rounded to FP32 after every step drifts by 1.1e-6 (nearest
# gradient) and 3.3e-6 (isotropic gradient) in 20000 steps of this bubble; the
# GPU's FP32 step drifts less (measured up to 1.6e-7), and this bound keeps it
# below both.
FP32_MASS = 1e-6


def say(*a):
    print("[gpu-precision]", *a, file=sys.stderr, flush=True)


def _psi(rr, rb, p):
    a, b = rr / p["rho0_r"], rb / p["rho0_b"]
    return (a - b) / (a + b)


def _laplace_fields(m, p, n):
    """Pressure jump sampled at r < R - 4 and r > R + 4 around the lattice
    centre, R the radius of a disk of the red area."""
    R = math.sqrt((0.5 * (1 + _psi(m["rho_r"], m["rho_b"], p))).sum() / math.pi)
    y, x = np.mgrid[0:n, 0:n]
    r = np.hypot(x + 0.5 - n / 2, y + 0.5 - n / 2)
    return m["p"][r < R - 4].mean() - m["p"][r > R + 4].mean(), R


def _gpu(p, c, steps, storage):
    q = dict(p, storage=storage)
    with capi.Lattice(q) as g:
        g.init(c["rho_r"], c["rho_b"])
        g.step(steps)
        d = g.diag(check=False)
        R = math.sqrt(d["area_r"] / math.pi)
        d = g.diag(circle=(p["nx"] / 2, p["ny"] / 2, R - 4, R + 4), check=False)
    return d


@pytest.fixture(scope="module")
def c1_fp64():
    c = W.static_bubble(n=64, radius=16)
    s = oracle.Sim(**c["params"]).init(c["rho_r"], c["rho_b"], None, None)
    s.step(20000)
    dp, R = _laplace_fields(s.moments(), c["params"], 64)
    say(f"C1 FP64 oracle: dp = {dp:.6e}, R = {R:.3f}, dp / (sigma/R) = {dp / (4e-3 / 9 / R):.5f}")
    return c, dp


@pytest.mark.parametrize("storage", ["f32", "f16s", "bf16s"])
def test_c1_laplace_against_fp64(c1_fp64, storage):
    """Converged 64 x 64 static bubble (R = 16, A = 1e-3, 20000 steps): the
    pressure jump of every storage format is within 1% of the FP64 oracle's."""
    c, dp64 = c1_fp64
    d = _gpu(c["params"], c, 20000, storage)
    dp = d["p_in"] - d["p_out"]
    mr, mb = c["rho_r"].sum(), c["rho_b"].sum()
    say(f"C1 {storage}: dp rel. to FP64 {dp / dp64 - 1:+.2e}, mass drift {d['mass_r'] / mr - 1:+.1e} "
        f"{d['mass_b'] / mb - 1:+.1e}, max|u| {d['max_u']:.2e}")
    assert abs(dp / dp64 - 1) <= 0.01
    bound = FP32_MASS if storage == "f32" else 1e-7
    assert abs(d["mass_r"] / mr - 1) <= bound and abs(d["mass_b"] / mb - 1) <= bound
    assert d["max_u"] <= 2e-5          # FP64: 5e-6


@pytest.mark.parametrize("storage", ["f16s", "bf16s"])
def test_16bit_against_fp32(storage):
    """Density-ratio bubbles and gravity slugs: 16-bit storage keeps colour
    mass to FP32's level and spurious currents near FP32's."""
    cases = []
    for g in (10, 100):
        cases.append((f"bubble 256 gamma={g}", W.bubble_cell(g, g, 64, n=256), 3000))
    cases.append(("slug 512x32 gamma=10", W.gravity_slug(nx=512, ny=32, gamma=10, band_lo=60, band_hi=150), 3000))
    for name, c, steps in cases:
        p = c["params"]
        out = {}
        for st in ("f32", storage):
            with capi.Lattice(dict(p, storage=st)) as g:
                g.init(c["rho_r"], c["rho_b"])
                g.step(steps)
                out[st] = g.diag(check=False)
        mr, mb = c["rho_r"].sum(), c["rho_b"].sum()
        a, b = out["f32"], out[storage]
        say(f"{name} {storage}: mass drift {b['mass_r'] / mr - 1:+.1e} {b['mass_b'] / mb - 1:+.1e} "
            f"(f32 {a['mass_r'] / mr - 1:+.1e} {a['mass_b'] / mb - 1:+.1e}), max|u| {b['max_u']:.2e} (f32 {a['max_u']:.2e})")
        assert b["n_nonfinite"] == 0
        assert abs(b["mass_r"] / mr - 1) <= 1e-7 and abs(b["mass_b"] / mb - 1) <= 1e-7
        assert b["max_u"] <= 1.5 * a["max_u"] + 1e-5


@pytest.mark.parametrize("variant", ["isotropic", "mrt_nsc"])
def test_c1_laplace_variants(variant):
    """The converged 64 x 64 bubble with the second-neighbour gradient, and
    with MRT and the Navier-Stokes correction: every storage's pressure jump
    within 1% of the FP64 oracle's for the same variant, colour mass within
    1e-7 for the 16-bit storages (exact colour-mass bookkeeping) and within
    FP32_MASS for FP32."""
    c = W.static_bubble(n=64, radius=16)
    p = dict(c["params"], gradient="isotropic") if variant == "isotropic" else \
        dict(c["params"], collision="mrt", ns_correction=True)
    s = oracle.Sim(**p).init(c["rho_r"], c["rho_b"], None, None)
    s.step(20000)
    dp64, R = _laplace_fields(s.moments(), p, 64)
    mr, mb = c["rho_r"].sum(), c["rho_b"].sum()
    for storage in ("f32", "f16s", "bf16s"):
        d = _gpu(p, c, 20000, storage)
        dp = d["p_in"] - d["p_out"]
        say(f"C1 {variant} {storage}: dp rel. to FP64 {dp / dp64 - 1:+.2e} (FP64 dp / (sigma/R) = "
            f"{dp64 / (4e-3 / 9 / R):.4f}), mass drift {d['mass_r'] / mr - 1:+.1e} {d['mass_b'] / mb - 1:+.1e}")
        assert abs(dp / dp64 - 1) <= 0.01
        bound = FP32_MASS if storage == "f32" else 1e-7
        assert abs(d["mass_r"] / mr - 1) <= bound and abs(d["mass_b"] / mb - 1) <= bound


@pytest.mark.parametrize("gamma", [10, 100])
def test_density_ratio_laplace_against_fp64(gamma):
    """Converged 128 x 128 bubbles at density ratios 10 and 100 (light
    bubble of radius 32, the same kinematic viscosity in both fluids, tau = 1,
    as in the serving mix; sigma = 0.01), 16000 steps: the FP64 pressure jump
    is then within 0.2% of Laplace's law and unchanged to 1e-4 from step 12000
    to 40000.  The pressure jump of every storage within 1% of the FP64
    oracle's, colour mass within 1e-7 for the 16-bit storages and within
    FP32_MASS for FP32.  (With a ten times smaller sigma and unequal
    viscosities the jump at density ratio 100 is 3e-5 of the pressure and
    still creeping after 60000 steps: FP32 itself then resolves it only to a
    few percent.)"""
    c = W.bubble_cell(gamma, gamma, 32, n=128, tau_min=1.0, sigma=0.01)
    p = c["params"]
    steps = 16000
    s = oracle.Sim(**p).init(c["rho_r"], c["rho_b"], None, None)
    s.step(steps)
    dp64, R = _laplace_fields(s.moments(), p, 128)
    say(f"gamma={gamma} FP64 oracle: dp = {dp64:.6e}, R = {R:.3f}, dp / (sigma/R) = {dp64 / (p['sigma'] / R):.4f}")
    mr, mb = c["rho_r"].sum(), c["rho_b"].sum()
    for storage in ("f32", "f16s", "bf16s"):
        d = _gpu(p, c, steps, storage)
        dp = d["p_in"] - d["p_out"]
        say(f"gamma={gamma} {storage}: dp rel. to FP64 {dp / dp64 - 1:+.2e}, mass drift {d['mass_r'] / mr - 1:+.1e} "
            f"{d['mass_b'] / mb - 1:+.1e}, max|u| {d['max_u']:.2e}")
        assert d["n_nonfinite"] == 0
        assert abs(dp / dp64 - 1) <= 0.01
        bound = FP32_MASS if storage == "f32" else 1e-7
        assert abs(d["mass_r"] / mr - 1) <= bound and abs(d["mass_b"] / mb - 1) <= bound
