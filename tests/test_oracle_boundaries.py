"""Pins of the oracle's boundary readings that the full-step invariants do not
fix: the ghost values of the colour field next to walls and open faces
(Sec. 2.4 extrapolation, R6), the outer ghost rows of the second-neighbour
gradient (R15) and the ghost values of Q of the Navier-Stokes correction
(Sec. 2.1.3, R14).  Each is checked on a field that varies along the
boundary as a single Fourier mode (or a line), whose gradient at the
boundary rows follows in closed form from the rule; the plausible
alternatives give different values (stated per test), and the oracle's
switchable alternative readings are checked against their own closed forms.

The state is put in the rest populations only: pull streaming leaves those
in place whatever the boundary, so the colour densities the gradients see
are exactly the ones set."""
import math

import numpy as np
import pytest

from paper_1903_01168_amd import workloads as W

NX, NY = 24, 7
K = 2 * math.pi * 3 / NX          # three periods across the lattice
AMP = 0.6


def _rest_state(rr, rb):
    ny, nx = rr.shape
    pops = np.zeros((2, 9, ny, nx))
    pops[0, 0] = rr
    pops[1, 0] = rb
    return pops


def _colour_sim(orc, f, **kw):
    """A lattice whose colour field is exactly f (rho0 = 1, 3)."""
    p = dict(W.params(nx=f.shape[1], ny=f.shape[0], rho0_r=1.0, rho0_b=3.0, tau_r=0.8, tau_b=0.9, A=1e-3), **kw)
    s = orc.Sim(**p)
    s.set_pops(_rest_state(1.0 * (1 + f) / 2, 3.0 * (1 - f) / 2))
    return s


def _mode(amp=AMP):
    x = np.arange(NX)
    return amp * np.cos(K * x)


@pytest.mark.parametrize("bc_y", ["walls", "freeslip"])
def test_wall_ghost_rows_of_the_colour_field(orc, bc_y):
    """Sec. 2.4: a wall node takes the W-weighted mean of its fluid
    neighbours; for a flat wall and f = a cos(kx) along it that is
    G f with G = (4 W_1 + 2 W_2 cos k)/(W_1 + 2 W_2) = (2 + cos k)/3, and the
    S2I4 gradient (xi = 1/3, 1/12) of the wall row is
        F_x = D (5 + G)/12,  F_y = +-(1 - G)(2 + cos k) f / 6,
    D = f(x+1) - f(x-1); the interior rows have F_x = D/2, F_y = 0.
    Equal weights (1:1:1) would give G = (1 + 2 cos k)/3 and twice the F_y;
    the axis neighbour alone, G = 1 and F_y = 0."""
    f1 = _mode()
    f = np.tile(f1, (NY, 1))
    s = _colour_sim(orc, f, bc_y=bc_y)
    g = s.gradients()
    G = (2 + math.cos(K)) / 3
    D = np.roll(f1, -1) - np.roll(f1, 1)
    Fy_wall = (1 - G) * (2 + math.cos(K)) * f1 / 6
    assert np.allclose(g["Fx"][0], D * (5 + G) / 12, atol=1e-14, rtol=0)
    assert np.allclose(g["Fx"][NY - 1], D * (5 + G) / 12, atol=1e-14, rtol=0)
    assert np.allclose(g["Fy"][0], Fy_wall, atol=1e-14, rtol=0)
    assert np.allclose(g["Fy"][NY - 1], -Fy_wall, atol=1e-14, rtol=0)
    assert np.allclose(g["Fx"][1:NY - 1], D / 2, atol=1e-14, rtol=0)
    assert np.allclose(g["Fy"][1:NY - 1], 0.0, atol=1e-14, rtol=0)
    assert np.abs(Fy_wall).max() > 1e-2        # the case is not degenerate


def test_open_face_ghost_column_of_the_colour_field(orc):
    """Beyond the pressure outlet the ghost column repeats the outlet column
    (R6), so for a colour field linear in x with slope b the outlet column's
    gradient is F_x = b/2 (linear extrapolation would give b), the next
    column's b; with p_out the common reference pressure the outlet keeps
    the colour field it is given."""
    nx, ny, b = 16, 5, 0.05
    f = np.tile(b * (np.arange(nx) - nx / 2), (ny, 1))
    s = _colour_sim(orc, f, bc_x="open", p_out=1.0 * 0.48, u_in_r=0.0, u_in_b=0.0)
    s.set_inlet_color(np.ones(ny, dtype=np.int8))
    g = s.gradients()
    assert np.allclose(g["Fx"][:, nx - 1], b / 2, atol=1e-14, rtol=0)
    assert np.allclose(g["Fx"][:, 2:nx - 1], b, atol=1e-14, rtol=0)
    assert np.allclose(g["Fy"][:, 2:], 0.0, atol=1e-14, rtol=0)


# second-neighbour stencil (R15): weights by |c|^2
ISO_W = {1: 4 / 21, 2: 4 / 45, 4: 1 / 60, 5: 2 / 315, 8: 1 / 5040}


def _iso_gradient(rows):
    """The 25-point gradient of a field given as rows -2 .. ny+1 (periodic x)."""
    ny = rows.shape[0] - 4
    Fx = np.zeros((ny, rows.shape[1]))
    Fy = np.zeros_like(Fx)
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            c2 = dx * dx + dy * dy
            if c2 == 0:
                continue
            sh = np.roll(rows[2 + dy:2 + dy + ny], -dx, axis=1)
            Fx += ISO_W[c2] * dx * sh
            Fy += ISO_W[c2] * dy * sh
    return Fx, Fy


@pytest.mark.parametrize("alt", [False, True])
def test_outer_ghost_rows_of_the_isotropic_gradient(orc, alt):
    """Second-neighbour gradient next to a wall: the ghost row next to the wall
    holds G f (Sec. 2.4, as above); the row beyond it, which no fluid node
    neighbours, repeats it (R15) -- or, with the alternative reading, is the
    linear extrapolation (2G - 1) f.  The two rows next to each wall match the
    stencil applied to those rows, and the second row does not depend on the
    reading (it reaches only the inner ghost row)."""
    f1 = _mode()
    f = np.tile(f1, (NY, 1))
    s = _colour_sim(orc, f, bc_y="walls", gradient="isotropic", alt=orc.ALT_ISO_EXTRAP if alt else 0)
    g = s.gradients()
    G = (2 + math.cos(K)) / 3
    outer = (2 * G - 1) if alt else G
    rows = np.vstack([outer * f1, G * f1, f, G * f1, outer * f1])
    Fx, Fy = _iso_gradient(rows)
    assert np.allclose(g["Fx"], Fx, atol=1e-14, rtol=0)
    assert np.allclose(g["Fy"], Fy, atol=1e-14, rtol=0)
    if alt:
        ref = _colour_sim(orc, f, bc_y="walls", gradient="isotropic").gradients()
        assert np.array_equal(g["Fy"][1:NY - 1], ref["Fy"][1:NY - 1])
        assert np.abs(g["Fy"][0] - ref["Fy"][0]).max() > 1e-3


@pytest.mark.parametrize("alt", [False, True])
def test_ghost_rows_of_q(orc, alt):
    """Navier-Stokes correction (Sec. 2.1.3): Q = (1.8 alpha - 0.8) rho u.  One
    fluid at rest density with u_x = u0 cos(kx): Q_x is a single mode along
    the walls, its ghost rows take the colour field's rule (R14), so dQx/dx
    on the wall rows is D_Q (5 + G)/12 and D_Q/2 inside, D_Q = Q_x(x+1) -
    Q_x(x-1); with the alternative reading (Q = 0 beyond a wall, the wall
    being at rest) the wall rows give 5 D_Q / 12.  dQy/dy = 0 throughout."""
    u0 = 0.02
    x = np.arange(NX)
    U = u0 * np.cos(K * x)
    rho = np.ones((NY, NX))
    # rest and x-moving populations only (no wall interaction), set so that
    # after pull streaming each node holds N_1 - N_3 = rho U, sum rho
    n1 = np.tile(U / 2 + 0.2, (NY, 1))
    n3 = np.tile(-U / 2 + 0.2, (NY, 1))
    pops = np.zeros((2, 9, NY, NX))
    pops[0, 0] = rho - 0.4
    pops[0, 1] = np.roll(n1, -1, axis=1)     # streamed from x-1
    pops[0, 3] = np.roll(n3, 1, axis=1)      # streamed from x+1
    p = W.params(nx=NX, ny=NY, bc_y="walls", collision="mrt", ns_correction=True, tau_r=0.8, tau_b=0.8, A=0.0)
    s = orc.Sim(**dict(p, alt=orc.ALT_Q_WALL_ZERO if alt else 0))
    s.set_pops(pops)
    m = s.moments()
    assert np.allclose(m["ux"], np.tile(U, (NY, 1)), atol=1e-15, rtol=0)
    s.set_pops(pops)
    g = s.gradients()
    kap = 1.8 * 0.2 - 0.8
    Q = kap * U
    DQ = np.roll(Q, -1) - np.roll(Q, 1)
    G = (2 + math.cos(K)) / 3
    wall = DQ * 5 / 12 if alt else DQ * (5 + G) / 12
    dqx = g["dqxdx"][0]                      # red: the only colour
    assert np.allclose(dqx[0], wall, atol=1e-16, rtol=0)
    assert np.allclose(dqx[NY - 1], wall, atol=1e-16, rtol=0)
    assert np.allclose(dqx[1:NY - 1], DQ / 2, atol=1e-16, rtol=0)
    assert np.allclose(g["dqydy"], 0.0, atol=1e-17, rtol=0)
    assert np.allclose(g["dqxdx"][1], 0.0, atol=0, rtol=0)


def test_fp32_storage_model_rounds_each_population_once(orc):
    """The parity bounds' storage model: a step with round_f32 is the plain
    step followed by rounding every stored population to the nearest FP32
    number (and nothing else)."""
    p = W.params(nx=40, ny=20, rho0_r=1.0, rho0_b=3.0, tau_r=0.7, tau_b=0.9, A=1e-3)
    rr, rb, ux, uy = W.random_fields(40, 20, seed=3, rho0_r=1.0, rho0_b=3.0)
    a = orc.Sim(**p).init(rr, rb, ux, uy)
    b = orc.Sim(**p).init(rr, rb, ux, uy)
    for _ in range(5):
        a.step(1)
        a.set_pops(a.get_pops().astype(np.float32).astype(np.float64))
    b.step(5, round_f32=True)
    assert np.array_equal(a.get_pops(), b.get_pops())
    c = orc.Sim(**p).init(rr, rb, ux, uy).step(5)
    assert not np.array_equal(c.get_pops(), b.get_pops())
