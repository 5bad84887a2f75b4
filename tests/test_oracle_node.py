"""Pins of the oracle's node-level operators against closed forms.

Each test checks a property that the paper's equations fix exactly (moment
identities, conservation, isotropy, exactness on polynomials, algebraic
identities of the boundary completion), not a retyped formula.
"""
import itertools
import math

import numpy as np
import pytest

RNG = np.random.default_rng(1234)


def test_lattice_isotropy(orc):
    cx, cy, opp, W = orc.lattice()
    c = np.stack([cx, cy], 1).astype(float)
    assert W.sum() == pytest.approx(1.0, abs=1e-15)
    # second moment: I/3 ; odd moments vanish
    assert np.allclose(np.einsum("i,ia,ib->ab", W, c, c), np.eye(2) / 3, atol=1e-15)
    assert np.allclose(np.einsum("i,ia->a", W, c), 0, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", W, c, c, c), 0, atol=1e-15)
    # fourth-order isotropy: (d_ab d_cd + d_ac d_bd + d_ad d_bc) / 9
    d = np.eye(2)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", W, c, c, c, c), iso, atol=1e-15)
    # opposite directions and weights by speed class
    for i in range(9):
        assert cx[opp[i]] == -cx[i] and cy[opp[i]] == -cy[i]
    assert W[0] == pytest.approx(4 / 9) and np.allclose(W[1:5], 1 / 9) and np.allclose(W[5:], 1 / 36)
    assert sorted(zip(cx, cy)) == sorted(itertools.product((-1, 0, 1), repeat=2))


def test_mrt_matrices(orc):
    cx, cy, _, _ = orc.lattice()
    M, Mi = orc.mrt_matrices()
    # rows 3 and 5 of M are the momentum rows: they fix the velocity numbering
    assert np.array_equal(M[3], cx) and np.array_equal(M[5], cy)
    assert np.array_equal(M[0], np.ones(9))
    # printed inverse is the inverse; rows are orthogonal
    assert np.allclose(M @ Mi, np.eye(9), atol=1e-14)
    G = M @ M.T
    assert np.allclose(G, np.diag(np.diag(G)))
    # the inverse is M^T diag(1/|row|^2)
    assert np.allclose(Mi, M.T @ np.diag(1 / np.diag(G)), atol=1e-15)


def test_tables(orc):
    for alpha in (0.2, 0.5, 0.9992):
        phi, B, xi = orc.tables(alpha)
        assert phi.sum() == pytest.approx(1.0, abs=1e-15)
        assert phi[0] == alpha
    _, _, _, W = orc.lattice()
    phi, B, xi = orc.tables(0.2)
    cx, cy, _, _ = orc.lattice()
    # xi = 3 W on moving directions, so sum xi c c = I (gradient normalisation)
    assert np.allclose(xi[1:], 3 * W[1:])
    c = np.stack([cx, cy], 1)
    assert np.allclose(np.einsum("i,ia,ib->ab", xi, c, c), np.eye(2))
    assert B.sum() == pytest.approx(1 / 3, abs=1e-15)


@pytest.mark.parametrize("rho0", [(1.0, 1.0), (1.0, 10.0), (1000.0, 1.0), (5.0, 1.0)])
def test_alphas_pressure_balance(orc, rho0):
    ar, ab = orc.alphas(*rho0, 0.2)
    cs2 = lambda a: 3 * (1 - a) / 5
    assert rho0[0] * cs2(ar) == pytest.approx(rho0[1] * cs2(ab), rel=1e-14)
    light, heavy = (ar, ab) if rho0[0] <= rho0[1] else (ab, ar)
    assert light == 0.2 and 0 < light <= heavy + 1e-15 and heavy < 1


@pytest.mark.parametrize("alpha", [0.2, 4 / 9, 0.9])
def test_equilibrium_moments(orc, alpha):
    cx, cy, _, W = orc.lattice()
    c = np.stack([cx, cy], 1).astype(float)
    for _ in range(20):
        rho = RNG.uniform(0.1, 10)
        u = RNG.uniform(-0.1, 0.1, 2)
        E = orc.equilibrium(rho, u[0], u[1], alpha)
        assert E.sum() == pytest.approx(rho, rel=1e-14)
        assert np.allclose(E @ c, rho * u, atol=1e-14 * rho)
        cs2 = 3 * (1 - alpha) / 5
        P = np.einsum("i,ia,ib->ab", E, c, c)
        assert np.allclose(P, rho * cs2 * np.eye(2) + rho * np.outer(u, u), atol=1e-14 * rho)


def test_equilibrium_textbook_limit(orc):
    """alpha = 4/9 turns the density-ratio equilibrium into the textbook D2Q9 one."""
    cx, cy, _, W = orc.lattice()
    for _ in range(10):
        rho = RNG.uniform(0.5, 2)
        u = RNG.uniform(-0.1, 0.1, 2)
        cu = cx * u[0] + cy * u[1]
        ref = W * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (u @ u))
        assert np.allclose(orc.equilibrium(rho, u[0], u[1], 4 / 9), ref, atol=1e-15)


@pytest.mark.parametrize("wr,wb", [(1.0, 1.0), (1 / 0.6, 1 / 1.5), (0.3, 1.8), (1 / 100.5, 1 / 0.6)])
def test_omega_eff(orc, wr, wb):
    d = 0.1
    f = lambda s: orc.omega_eff(s, wr, wb, d)
    chi = 2 * wr * wb / (wr + wb)
    assert f(0.0) == pytest.approx(chi, rel=1e-14)
    assert f(0.5) == wr and f(-0.5) == wb and f(1.0) == wr and f(-1.0) == wb
    # continuity at +-delta and at 0, zero slope at +-delta
    h = 1e-7
    assert f(d) == pytest.approx(wr, rel=1e-13)
    assert f(-d) == pytest.approx(wb, rel=1e-13)
    assert f(1e-12) == pytest.approx(chi, rel=1e-9)
    scale = abs(wr - wb) + 1e-30
    assert abs((f(d) - f(d - h)) / h) < 1e-5 * scale / d + 1e-12
    assert abs((f(-d + h) - f(-d)) / h) < 1e-5 * scale / d + 1e-12
    # monotone between the two pure values
    s = np.linspace(-0.2, 0.2, 401)
    v = np.array([f(x) for x in s])
    dv = np.diff(v)
    assert np.all(dv >= -1e-15) or np.all(dv <= 1e-15)
    if wr == wb:
        assert np.allclose(v, wr, rtol=1e-14)


def test_gradient_exact_on_quadratics(orc):
    for _ in range(20):
        a, b, cc, d, e, f = RNG.normal(size=6)
        q = lambda x, y: a + b * x + cc * y + d * x * x + e * x * y + f * y * y
        patch = [[q(dx, dy) for dx in (-1, 0, 1)] for dy in (-1, 0, 1)]
        F = orc.gradient3x3(patch)
        assert np.allclose(F, [b, cc], atol=1e-14)


def test_perturbation_moments(orc):
    cx, cy, _, _ = orc.lattice()
    c = np.stack([cx, cy], 1).astype(float)
    for _ in range(20):
        F = RNG.normal(size=2) * RNG.uniform(1e-6, 1)
        A = RNG.uniform(1e-4, 1e-2)
        P = orc.perturbation(F, A)
        Fm = np.linalg.norm(F)
        n = F / Fm
        assert abs(P.sum()) < 1e-17 + 1e-15 * A * Fm
        assert np.allclose(P @ c, 0, atol=1e-15 * A * Fm + 1e-18)
        second = np.einsum("i,ia,ib->ab", P, c, c)
        assert np.allclose(second, 2 * A / 9 * Fm * (np.outer(n, n) - np.eye(2)),
                           atol=1e-14 * A * Fm)
    assert np.all(orc.perturbation([0.0, 0.0], 1e-3) == 0)


def test_recolor_conservation_and_shift(orc):
    cx, cy, _, _ = orc.lattice()
    c = np.stack([cx, cy], 1).astype(float)
    for _ in range(20):
        rr, rb = RNG.uniform(0.01, 5, 2)
        ar, ab = orc.alphas(1.0, RNG.uniform(1, 100))
        Nss = RNG.uniform(0.01, 0.5, 9) * (rr + rb)
        Nss *= (rr + rb) / Nss.sum()
        F = RNG.normal(size=2)
        beta = RNG.uniform(0.3, 1.0)
        Nr, Nb = orc.recolor(Nss, rr, rb, F, beta, ar, ab)
        rho = rr + rb
        assert Nr.sum() == pytest.approx(rr, rel=1e-13)
        assert Nb.sum() == pytest.approx(rb, rel=1e-13)
        assert np.allclose(Nr + Nb, Nss, atol=1e-15 * rho)
        n = F / np.linalg.norm(F)
        shift = Nr @ c - rr / rho * (Nss @ c)
        expect = beta * rr * rb / rho ** 2 * (0.4 + math.sqrt(2) / 10) * (rr * (1 - ar) + rb * (1 - ab)) * n
        assert np.allclose(shift, expect, atol=1e-14 * rho)
    # one colour only: recolouring is the identity
    Nss = RNG.uniform(0.01, 0.5, 9)
    Nr, Nb = orc.recolor(Nss, Nss.sum(), 0.0, [0.3, -0.2], 0.99, 0.2, 0.2)
    assert np.array_equal(Nr, Nss) and np.all(Nb == 0)


def test_zouhe_west_east(orc):
    cx, cy, _, _ = orc.lattice()
    for _ in range(20):
        N = RNG.uniform(0.01, 0.3, 9)
        vx, vy = RNG.uniform(-0.05, 0.05, 2)
        rho, Nc = orc.zouhe_west(N, vx, vy)
        assert Nc.sum() == pytest.approx(rho, rel=1e-14)
        assert Nc @ cx == pytest.approx(rho * vx, abs=1e-15)
        assert Nc @ cy == pytest.approx(rho * vy, abs=1e-15)
        for i in (0, 2, 3, 4, 6, 7):
            assert Nc[i] == N[i]
        rho_out = RNG.uniform(0.5, 2)
        vx2, Ne = orc.zouhe_east(N, rho_out, 0.0)
        assert Ne.sum() == pytest.approx(rho_out, rel=1e-14)
        assert Ne @ cx == pytest.approx(rho_out * vx2, abs=1e-15)
        assert Ne @ cy == pytest.approx(0.0, abs=1e-15)
        for i in (0, 1, 2, 4, 5, 8):
            assert Ne[i] == N[i]


@pytest.mark.parametrize("alpha", [0.2, 0.95])
def test_zouhe_exact_on_equilibrium(orc, alpha):
    """An equilibrium state is completed exactly: the three unknowns come back."""
    for _ in range(10):
        rho = RNG.uniform(0.5, 2)
        ux, uy = RNG.uniform(-0.05, 0.05, 2)
        E = orc.equilibrium(rho, ux, uy, alpha)
        rho_w, Nw = orc.zouhe_west(np.where(np.isin(np.arange(9), [1, 5, 8]), 0.0, E), ux, uy)
        assert rho_w == pytest.approx(rho, rel=1e-13)
        assert np.allclose(Nw, E, atol=1e-14)
        vx, Ne = orc.zouhe_east(np.where(np.isin(np.arange(9), [3, 6, 7]), 0.0, E), rho, uy)
        assert vx == pytest.approx(ux, abs=1e-14)
        assert np.allclose(Ne, E, atol=1e-14)


def test_mrt_reduces_to_bgk_and_relaxes_moments(orc):
    M, _ = orc.mrt_matrices()
    for _ in range(10):
        N = RNG.uniform(0.01, 0.3, 9)
        E = orc.equilibrium(N.sum(), 0.03, -0.02, 0.2)
        w = RNG.uniform(0.1, 1.9)
        bgk = N - w * (N - E)
        assert np.allclose(orc.mrt_collide(N, E, w, 1.0), bgk, atol=1e-15)
        lam = 0.8
        out = orc.mrt_collide(N, E, w, lam)
        dm = M @ (out - N)
        s = np.array([lam * w] * 7 + [w, w])
        assert np.allclose(dm, -s * (M @ (N - E)), atol=1e-14)


# ------------------------------------------------------------- wetting (Sec. 2.4)
def test_wetting_keeps_length_and_sets_the_angle(orc):
    rng = np.random.default_rng(3)
    for _ in range(200):
        F = rng.standard_normal(2)
        a = rng.uniform(0, 2 * np.pi)
        ns = np.array([np.cos(a), np.sin(a)])
        theta = rng.uniform(0.05, np.pi - 0.05)
        out = orc.wetting(F, ns, theta)
        Fm = np.linalg.norm(F)
        assert np.linalg.norm(out) == pytest.approx(Fm, rel=1e-13)
        assert out @ ns == pytest.approx(Fm * np.cos(theta), abs=1e-12 * Fm)
        # the chosen direction is the candidate closer to F's own direction
        t = np.array([-ns[1], ns[0]])
        other = Fm * (np.cos(theta) * ns - np.sign(out @ t) * np.sin(theta) * t)
        assert np.linalg.norm(out / Fm - F / Fm) <= np.linalg.norm(other / Fm - F / Fm) + 1e-12


def test_wetting_special_cases(orc):
    ns = np.array([0.0, 1.0])
    F = np.array([0.3, -0.4])
    # already at the angle: unchanged
    th = np.arccos((F @ ns) / np.linalg.norm(F))
    assert np.allclose(orc.wetting(F, ns, th), F, atol=1e-14)
    # along the normal: a tie, the normal itself
    assert np.allclose(orc.wetting(np.array([0.0, 2.0]), ns, 1.0), [0.0, 2.0], atol=1e-15)
    # no gradient: nothing changes
    assert np.all(orc.wetting(np.zeros(2), ns, 1.0) == 0.0)
    # mirror symmetry: F mirrored across the normal gives the mirrored result
    a, b = orc.wetting(F, ns, 1.1), orc.wetting(F * [-1, 1], ns, 1.1)
    assert np.allclose(a * [-1, 1], b, atol=1e-15)


def test_wetting_end_angles(orc):
    """theta = 0 and pi: the two candidates coincide, every gradient is turned
    onto +ns or -ns with its length kept (whatever its tangential part)."""
    ns = np.array([0.0, -1.0])
    for F in ([0.3, -0.4], [-0.3, 0.4], [0.0, 0.5], [0.5, 0.0]):
        F = np.array(F)
        assert np.allclose(orc.wetting(F, ns, 0.0), np.linalg.norm(F) * ns, atol=1e-15)
        assert np.allclose(orc.wetting(F, ns, np.pi), -np.linalg.norm(F) * ns, atol=1e-15)


# ------------------------------------------- Navier-Stokes correction (Sec. 2.1.3)
@pytest.mark.parametrize("alpha", [0.2, 0.6, 0.95])
def test_hermite_equilibrium_moments(orc, alpha):
    """The Hermite equilibrium keeps mass, momentum and the momentum flux
    rho c_s^2 I + rho u u of the plain one; its mixed third moments become
    c_s^2 rho u (those of a Maxwellian of temperature c_s^2) while
    sum c_x^3 N^e = rho u_x stays (c_x^3 = c_x on the lattice).  A garbled
    (3 c_i - 4) read any other way breaks one of these."""
    cx, cy, _, _ = orc.lattice()
    cs2 = 3 * (1 - alpha) / 5
    for _ in range(10):
        rho = RNG.uniform(0.5, 2)
        ux, uy = RNG.uniform(-0.05, 0.05, 2)
        H = orc.equilibrium_hermite(rho, ux, uy, alpha)
        E = orc.equilibrium(rho, ux, uy, alpha)
        assert H.sum() == pytest.approx(rho, rel=1e-14)
        assert H @ cx == pytest.approx(rho * ux, abs=1e-15)
        assert H @ cy == pytest.approx(rho * uy, abs=1e-15)
        for a, b in ((cx * cx, None), (cy * cy, None), (cx * cy, None)):
            assert H @ a == pytest.approx(E @ a, abs=1e-15)
        assert H @ (cx * cx) == pytest.approx(rho * cs2 + rho * ux * ux, abs=1e-14)
        assert H @ (cx * cy) == pytest.approx(rho * ux * uy, abs=1e-15)
        assert H @ (cx * cx * cy) == pytest.approx(cs2 * rho * uy, abs=1e-15)
        assert H @ (cx * cy * cy) == pytest.approx(cs2 * rho * ux, abs=1e-15)
        assert H @ (cx ** 3) == pytest.approx(rho * ux, abs=1e-15)
    # c_s^2 = 1/3 (alpha = 4/9): the correction factor is 1, the forms agree
    assert np.allclose(orc.equilibrium_hermite(1.3, 0.02, -0.01, 4 / 9),
                       orc.equilibrium(1.3, 0.02, -0.01, 4 / 9), atol=1e-16)


def test_ns_source_conserves(orc):
    """U = M^-1 C with C in the moments e and p_xx only: no mass, no momentum."""
    cx, cy, _, _ = orc.lattice()
    for _ in range(10):
        U = orc.ns_source(*RNG.uniform(-1e-3, 1e-3, 2), *RNG.uniform(0.2, 1.9, 2))
        assert abs(U.sum()) < 1e-18 and abs(U @ cx) < 1e-18 and abs(U @ cy) < 1e-18
    assert np.all(orc.ns_source(0.0, 0.0, 1.0, 1.2) == 0.0)


@pytest.mark.parametrize("alphas", [(0.2, 0.2), (0.2, 0.92), (0.6, 0.2)])
def test_zouhe_hermite_exact_on_equilibrium(orc, alphas):
    """With the Hermite equilibrium and its term H (kap = sum chi_k (3 c_s,k^2 - 1)),
    a two-colour equilibrium state is completed exactly; without H it is not."""
    for _ in range(10):
        rho = RNG.uniform(0.5, 2)
        chi = RNG.uniform(0, 1)
        ux, uy = RNG.uniform(-0.05, 0.05, 2)
        E = (orc.equilibrium_hermite(chi * rho, ux, uy, alphas[0])
             + orc.equilibrium_hermite((1 - chi) * rho, ux, uy, alphas[1]))
        kap = sum(c * (3 * 3 * (1 - a) / 5 - 1) for c, a in zip((chi, 1 - chi), alphas))
        rho_w, Nw = orc.zouhe_west(np.where(np.isin(np.arange(9), [1, 5, 8]), 0.0, E), ux, uy, kap)
        assert rho_w == pytest.approx(rho, rel=1e-13)
        assert np.allclose(Nw, E, atol=1e-14)
        vx, Ne = orc.zouhe_east(np.where(np.isin(np.arange(9), [3, 6, 7]), 0.0, E), rho, uy, kap)
        assert vx == pytest.approx(ux, abs=1e-14)
        assert np.allclose(Ne, E, atol=1e-14)
        if abs(kap * ux) > 1e-4:
            _, N0 = orc.zouhe_west(np.where(np.isin(np.arange(9), [1, 5, 8]), 0.0, E), ux, uy, 0.0)
            assert not np.allclose(N0, E, atol=1e-8)


# --------------------------------------------- second-neighbour gradient (R15)
def _poly_patch(f, x0, y0, r):
    return np.array([[f(x0 + dx, y0 + dy) for dx in range(-r, r + 1)] for dy in range(-r, r + 1)])


@pytest.mark.parametrize("deg", [1, 3, 5, 7])
def test_isotropic_gradient_exact_on_harmonic_polynomials(orc, deg):
    """The 25-point stencil's error on a polynomial is a sum of isotropic
    tensors (moments isotropic up to 8th order) times derivatives of its
    Laplacian, so it differentiates harmonic polynomials up to degree 7
    exactly; the nearest-neighbour stencil of eq. (colorGradient) (isotropic
    to 4th order) stops at degree 3."""
    f = lambda x, y: ((x + 1j * y) ** deg).real
    x0, y0 = 0.3, -0.7
    g = deg * (x0 + 1j * y0) ** (deg - 1)
    exact = np.array([g.real, -g.imag])
    F5 = orc.gradient5x5(_poly_patch(f, x0, y0, 2))
    assert np.allclose(F5, exact, rtol=0, atol=1e-13 * max(1.0, np.abs(exact).max()))
    F3 = orc.gradient3x3(_poly_patch(f, x0, y0, 1))
    if deg <= 3:
        assert np.allclose(F3, exact, atol=1e-13)
    else:
        assert np.abs(F3 - exact).max() > 0.1


def test_isotropic_gradient_of_quadratics(orc):
    """Second moment sum w c c = I: exact gradient of any quadratic."""
    for _ in range(5):
        a = RNG.normal(size=6)
        f = lambda x, y: a[0] + a[1] * x + a[2] * y + a[3] * x * x + a[4] * x * y + a[5] * y * y
        x0, y0 = RNG.uniform(-1, 1, 2)
        exact = [a[1] + 2 * a[3] * x0 + a[4] * y0, a[2] + a[4] * x0 + 2 * a[5] * y0]
        assert np.allclose(orc.gradient5x5(_poly_patch(f, x0, y0, 2)), exact, atol=1e-13)
