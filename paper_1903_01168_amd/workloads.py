"""Seeded synthetic workloads: lattice sizes, parameters and initial fields.

This module holds no arithmetic of the method itself.  It only draws seeded
geometry (disks, slug bands, inlet-colour schedules) and fixes the parameter
recipes of the benchmark cases, so that the FP64 oracle and the HIP library
receive byte-identical inputs.  Relaxation times are derived from viscosity
ratios with the lattice relation tau = 3 nu + 1/2 of the paper's Sec. 2.1.1;
densities are sharp phase indicators times the reference densities.

Cases (stand-ins for the paper's own runs, which used data that is not
available; the paper's sizes and parameters are quoted where they exist):

* ``static_bubble``  -- square periodic lattice, a disk of one fluid in the
  other (Sec. 4 square-to-droplet / Laplace tests).
* ``bubble_sweep``   -- 512 x 512 bubbles, density ratio gamma in
  {10, 100, 1000} x dynamic-viscosity ratio M in {1, 10, 100}.
* ``gravity_slug``   -- periodic channel with walls, body force, alternating
  heavy/light slugs (Sec. 5.1 periodic case).
* ``inlet_outlet``   -- channel with a velocity inlet, pressure outlet and
  free-slip walls, stratified two-phase inflow (Sec. 5.2 open channel).
* ``square_droplet`` -- a square of light fluid relaxing to a circle (Sec. 4
  square-to-droplet Laplace test).
* ``wall_droplet``   -- a rectangular droplet on a wall relaxing to a
  prescribed contact angle (Sec. 2.4; the paper's contact-angle case).
* ``serve_trace``    -- a seeded mix of bubble and slug solve requests.
"""
from __future__ import annotations

import math

import numpy as np

DEFAULTS = dict(bc_x="periodic", bc_y="periodic", collision="bgk", storage="f32",
                rho0_r=1.0, rho0_b=1.0, alpha_light=0.2, tau_r=1.0, tau_b=1.0,
                delta=0.1, A=0.0, sigma=0.0, beta=0.7, mrt_lambda=0.8, gx=0.0, gy=0.0,
                u_in_r=0.0, u_in_b=0.0, p_out=0.0, contact_angle=-1.0, ns_correction=False,
                gradient="nearest")


def params(**kw):
    """A full parameter dict (the fields of the C struct ``lbm_params``)."""
    p = dict(DEFAULTS)
    unknown = set(kw) - set(DEFAULTS) - {"nx", "ny"}
    if unknown:
        raise KeyError(f"unknown parameters: {sorted(unknown)}")
    p.update(kw)
    return p


def tau_from_nu(nu: float) -> float:
    return 3.0 * nu + 0.5


def nu_from_tau(tau: float) -> float:
    return (tau - 0.5) / 3.0


def disk_fields(nx, ny, cx, cy, radius, rho_in, rho_out, inside_red=True):
    """Sharp disk: node (x, y) is inside iff its cell centre (x+1/2, y+1/2)
    lies strictly within ``radius`` of (cx, cy)."""
    y, x = np.mgrid[0:ny, 0:nx]
    inside = (x + 0.5 - cx) ** 2 + (y + 0.5 - cy) ** 2 < radius ** 2
    red = inside if inside_red else ~inside
    rho_r = np.where(red, rho_in if inside_red else rho_out, 0.0)
    rho_b = np.where(~red, rho_out if inside_red else rho_in, 0.0)
    return rho_r.astype(np.float64), rho_b.astype(np.float64)


def static_bubble(n=64, radius=16.0, A=1e-3, tau=1.0, beta=0.7, collision="bgk",
                  storage="f32"):
    """Static bubble, density and viscosity ratio 1: red disk of radius 16
    centred in a 64 x 64 periodic blue lattice, A = 1e-3, beta = 0.7, tau = 1."""
    p = params(nx=n, ny=n, tau_r=tau, tau_b=tau, A=A, beta=beta, collision=collision,
               storage=storage)
    rr, rb = disk_fields(n, n, n / 2, n / 2, radius, 1.0, 1.0)
    return dict(name=f"static-bubble {n}x{n} R={radius:g}", params=p, rho_r=rr, rho_b=rb,
                ux=None, uy=None, radius=radius, center=(n / 2, n / 2))


def bubble_params(gamma, M, n=512, tau_min=0.6, sigma=4.0e-3 / 9.0, beta=0.7, collision="bgk",
                  storage="f32"):
    """Parameters of a periodic n x n bubble lattice with the light fluid
    coloured red (rho0_r = 1, rho0_b = gamma).  M is the dynamic-viscosity
    ratio heavy/light, so nu_heavy / nu_light = M / gamma; the smaller tau is
    ``tau_min``.  Surface tension is fixed through sigma (A follows omega)."""
    ratio = M / gamma                       # nu_heavy / nu_light
    if ratio <= 1.0:
        tau_h = tau_min
        tau_l = tau_from_nu(nu_from_tau(tau_h) / ratio)
    else:
        tau_l = tau_min
        tau_h = tau_from_nu(nu_from_tau(tau_l) * ratio)
    return params(nx=n, ny=n, rho0_r=1.0, rho0_b=float(gamma), tau_r=tau_l, tau_b=tau_h,
                  sigma=sigma, beta=beta, collision=collision, storage=storage)


def bubble_cell(gamma, M, radius, n=512, tau_min=0.6, sigma=4.0e-3 / 9.0, beta=0.7,
                collision="bgk", storage="f32"):
    """One cell of the bubble sweep: ``bubble_params`` plus the light disk of
    the given radius at the lattice centre."""
    p = bubble_params(gamma, M, n=n, tau_min=tau_min, sigma=sigma, beta=beta, collision=collision,
                      storage=storage)
    rr, rb = disk_fields(n, n, n / 2, n / 2, radius, 1.0, float(gamma))
    return dict(name=f"bubble {n}x{n} gamma={gamma} M={M} R={radius}", params=p, rho_r=rr,
                rho_b=rb, ux=None, uy=None, radius=float(radius), center=(n / 2, n / 2),
                gamma=gamma, M=M)


SWEEP_GAMMAS = (10, 100, 1000)
SWEEP_MS = (1, 10, 100)


def bubble_sweep(seed=0, n=512, storage="f32", collision="bgk"):
    """The 3 x 3 sweep; radii drawn uniformly from {64..128} with ``seed``."""
    rng = np.random.default_rng(seed)
    cells = []
    for g in SWEEP_GAMMAS:
        for m in SWEEP_MS:
            r = int(rng.integers(64, 129))
            cells.append(bubble_cell(g, m, r, n=n, storage=storage, collision=collision))
    return cells


def slug_edges(nx, rng, lo=200, hi=600):
    """First columns of alternating heavy/light full-height bands along x,
    seeded lengths in [lo, hi]; the last band absorbs the remainder; an even
    count of at least two.  Band b is heavy for even b."""
    edges = [0]
    while True:
        length = int(rng.integers(lo, hi + 1))
        if edges[-1] + length >= nx:
            break
        edges.append(edges[-1] + length)
    if len(edges) % 2 == 1 and len(edges) > 2:
        edges.pop()                         # merge the last two bands
    if len(edges) < 2:
        edges = [0, nx // 2]
    return edges


def slug_bands(nx, rng, lo=200, hi=600):
    """Heavy-band mask along x of ``slug_edges``."""
    edges = slug_edges(nx, rng, lo, hi)
    heavy = np.zeros(nx, dtype=bool)
    for b, x0 in enumerate(edges):
        x1 = edges[b + 1] if b + 1 < len(edges) else nx
        heavy[x0:x1] = (b % 2 == 0)
    return heavy


def slug_params(nx, ny, gamma=10, Re=10, g=1e-6, A=1e-3, beta=0.7, storage="f32", collision="bgk"):
    """Periodic channel with walls top/bottom and a body force along +x,
    heavy fluid red (rho0_r = gamma), light blue.  The heavy viscosity follows
    Re = g H^3 / (8 nu_l^2) with H = ny; mu_g = mu_l / 2."""
    nu_l = math.sqrt(g * ny ** 3 / (8.0 * Re))
    nu_g = nu_l * gamma / 2.0
    return params(nx=nx, ny=ny, bc_x="periodic", bc_y="walls", rho0_r=float(gamma), rho0_b=1.0,
                  tau_r=tau_from_nu(nu_l), tau_b=tau_from_nu(nu_g), A=A, beta=beta, gx=g,
                  storage=storage, collision=collision)


def gravity_slug(seed=0, nx=4096, ny=256, gamma=10, Re=10, g=1e-6, A=1e-3, beta=0.7,
                 storage="f32", collision="bgk", band_lo=200, band_hi=600):
    """``slug_params`` with full-height heavy/light slugs of seeded lengths."""
    rng = np.random.default_rng(seed)
    p = slug_params(nx, ny, gamma=gamma, Re=Re, g=g, A=A, beta=beta, storage=storage,
                    collision=collision)
    heavy = slug_bands(nx, rng, band_lo, band_hi)
    rr = np.where(heavy[None, :], float(gamma), 0.0) * np.ones((ny, 1))
    rb = np.where(heavy[None, :], 0.0, 1.0) * np.ones((ny, 1))
    return dict(name=f"gravity-slug {nx}x{ny} gamma={gamma} Re={Re}", params=p,
                rho_r=rr.astype(np.float64), rho_b=rb.astype(np.float64), ux=None, uy=None)


def inlet_schedule(total_steps, seed=0, lo=300, hi=800, first_red=True):
    """Inlet colour segments: list of (start_step, colour) with seeded lengths."""
    rng = np.random.default_rng(seed)
    seg, t, red = [], 0, first_red
    while t < total_steps:
        seg.append((t, 1 if red else -1))
        t += int(rng.integers(lo, hi + 1))
        red = not red
    return seg


def inlet_outlet(seed=0, nx=8192, ny=512, gamma=5, u_in=0.01, A=1e-3, beta=0.7, tau_heavy=0.6,
                 gas_fraction=0.2, storage="f32", collision="bgk", alternating=False, M=None,
                 walls="freeslip", total_steps=200000):
    """Channel with a west velocity inlet, an east pressure outlet and walls
    top/bottom (``walls``: "freeslip" as in the paper, or "walls" for no
    slip), set up as the paper's open-channel case (Sec. 5.2): heavy
    liquid (red, rho0_r = gamma) below light gas (blue), volume fractions
    0.8 / 0.2 in the initial fill and in the inflow, which enters with u_in in
    both phases; mu_g = mu_l / 2 (or nu_heavy / nu_light = M / gamma when M is
    given); tau_heavy = 0.6.  The outlet pressure is the common reference
    pressure, the light fluid's rho0 times 3 (1 - alpha_light) / 5.
    ``alternating``: instead, a channel filled with gas into which whole
    columns of liquid and gas are injected in turns on a seeded 300..800-step
    schedule (``schedule``)."""
    nu_h = nu_from_tau(tau_heavy)
    nu_l = nu_h * gamma / 2.0 if M is None else nu_h * gamma / M
    p0 = 0.48   # rho0_light * 3 (1 - 0.2) / 5
    p = params(nx=nx, ny=ny, bc_x="open", bc_y=walls, rho0_r=float(gamma), rho0_b=1.0,
               tau_r=tau_heavy, tau_b=tau_from_nu(nu_l), A=A, beta=beta, u_in_r=u_in,
               u_in_b=u_in, p_out=p0, storage=storage, collision=collision)
    visc = "mu_g=mu_l/2" if M is None else f"M={M}"
    if alternating:
        return dict(name=f"inlet-outlet {nx}x{ny} gamma={gamma} {visc} alternating", params=p,
                    rho_r=np.zeros((ny, nx)), rho_b=np.ones((ny, nx)), ux=None, uy=None,
                    schedule=inlet_schedule(total_steps, seed=seed))
    heavy = np.arange(ny) < int(round((1.0 - gas_fraction) * ny))
    rr = np.where(heavy[:, None], float(gamma), 0.0) * np.ones((1, nx))
    rb = np.where(heavy[:, None], 0.0, 1.0) * np.ones((1, nx))
    return dict(name=f"inlet-outlet {nx}x{ny} gamma={gamma} {visc} stratified", params=p,
                rho_r=rr, rho_b=rb, ux=None, uy=None,
                inlet_color=np.where(heavy, 1, -1).astype(np.int8))


def square_droplet(n, gamma=1.0, M=1.0, sigma=0.01, tau_light=1.0, beta60=0.99, storage="f32",
                   collision="bgk"):
    """Square-to-droplet case (Sec. 4 static bubble tests): an n x n periodic
    lattice, a light square of side round(0.33 n) (red) centred in the heavy
    fluid (blue), density ratio gamma = rho_heavy / rho_light and dynamic
    viscosity ratio M = mu_heavy / mu_light, surface tension sigma (0.01 in
    the paper), beta scaled with the resolution as beta60 (60 / n)^(5/8).
    The paper does not give tau; the light fluid's is tau_light, the heavy
    fluid's follows from nu_heavy / nu_light = M / gamma."""
    a = int(round(0.33 * n))
    lo = (n - a) // 2
    red = np.zeros((n, n))
    red[lo:lo + a, lo:lo + a] = 1.0
    nu_l = nu_from_tau(tau_light)
    tau_h = tau_from_nu(nu_l * M / gamma)
    p = params(nx=n, ny=n, rho0_r=1.0, rho0_b=float(gamma), tau_r=tau_light, tau_b=tau_h, sigma=sigma,
               beta=beta60 * (60.0 / n) ** 0.625, storage=storage, collision=collision)
    return dict(name=f"square {n}x{n} gamma={gamma:g} M={M:g}", params=p, rho_r=red,
                rho_b=float(gamma) * (1.0 - red), ux=None, uy=None, side=a, center=(n / 2, n / 2),
                gamma=gamma, M=M)


def wall_droplet(contact_angle, n=100, sigma=0.01, tau=1.0, beta=0.7, bc_y="walls", storage="f32",
                 collision="bgk"):
    """Contact-angle case (Sec. 6 of the paper's comparison, its contact-angle
    figure): an n x n lattice, density and viscosity ratio 1, surface
    tension sigma = 0.01, walls at the bottom and top, periodic in x; a red
    rectangle of 2 round(0.165 n) x round(0.165 n) nodes sits on the bottom
    wall, centred on the lattice's middle (for even n its axis falls between
    two columns and the case is mirror-symmetric), in blue.  The red fluid's contact angle (degrees) is prescribed
    at both walls."""
    w, h = 2 * int(round(0.165 * n)), int(round(0.165 * n))     # even width: a centred axis
    y, x = np.mgrid[0:n, 0:n]
    x0 = (n - w) // 2
    red = ((x >= x0) & (x < x0 + w) & (y < h)).astype(np.float64)
    p = params(nx=n, ny=n, bc_y=bc_y, rho0_r=1.0, rho0_b=1.0, tau_r=tau, tau_b=tau, sigma=sigma, beta=beta,
               contact_angle=float(contact_angle), storage=storage, collision=collision)
    return dict(name=f"droplet_{contact_angle:g}", params=p, rho_r=red, rho_b=1.0 - red, ux=None, uy=None,
                contact_angle=float(contact_angle))


def random_fields(nx, ny, seed=0, rho0_r=1.0, rho0_b=1.0, umax=0.02, smooth=True):
    """Rough two-phase fields for parity tests: a seeded, smoothed random phase
    indicator (with mixed interface nodes) and a small random velocity."""
    rng = np.random.default_rng(seed)
    f = rng.random((ny, nx))
    if smooth:
        for _ in range(3):
            f = (f + np.roll(f, 1, 0) + np.roll(f, -1, 0) + np.roll(f, 1, 1) + np.roll(f, -1, 1)) / 5
    f = np.clip((f - f.mean()) * 8 + 0.5, 0.0, 1.0)
    rho_r = f * rho0_r
    rho_b = (1.0 - f) * rho0_b
    ux = (rng.random((ny, nx)) - 0.5) * 2 * umax
    uy = (rng.random((ny, nx)) - 0.5) * 2 * umax
    return rho_r, rho_b, ux, uy


SERVE_GAMMAS = (1, 10, 100, 1000)     # bubbles
SERVE_SLUG_GAMMAS = (1, 10)           # slugs (the gas-viscosity rule gives tau_g >> 10 beyond)


def serve_trace(seed=0, n=2000, nodes_lo=64 * 64, nodes_hi=1024 * 1024, steps_lo=1000,
                steps_hi=50000, Re=10, storage="f16s"):
    """A seeded mix of solve requests: half static bubbles (square periodic
    lattice, side a multiple of 64, light disk of radius side/4 at the centre,
    density ratio from SERVE_GAMMAS with the same kinematic viscosity in both
    fluids, i.e. dynamic-viscosity ratio M = gamma), half periodic gravity
    slugs (16:1 channel with walls, height a multiple of 16, slugs 200..600
    long, Reynolds number Re, mu_g = mu_l / 2, density ratio from
    SERVE_SLUG_GAMMAS).  Node counts and step counts are log-uniform in their
    ranges, and ``gap`` is a unit-mean exponential inter-arrival draw (divide
    by the arrival rate)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        bubble = bool(rng.random() < 0.5)
        nodes = math.exp(rng.uniform(math.log(nodes_lo), math.log(nodes_hi)))
        gamma = int(rng.choice(SERVE_GAMMAS if bubble else SERVE_SLUG_GAMMAS))
        steps = int(round(math.exp(rng.uniform(math.log(steps_lo), math.log(steps_hi)))))
        gap = float(rng.exponential(1.0))
        sub = int(rng.integers(1 << 62))
        if bubble:
            side = int(min(1024, max(64, 64 * round(math.sqrt(nodes) / 64))))
            p = bubble_params(gamma, gamma, n=side, storage=storage)
            geo = dict(kind="disk", cx=side / 2, cy=side / 2, radius=side / 4, rho_r_in=1.0, rho_b_in=0.0,
                       rho_r_out=0.0, rho_b_out=float(gamma))
        else:
            ny = int(min(256, max(16, 16 * round(math.sqrt(nodes / 16) / 16))))
            nx = 16 * ny
            p = slug_params(nx, ny, gamma=gamma, Re=Re, storage=storage)
            edges = slug_edges(nx, np.random.default_rng(sub))
            geo = dict(kind="bands", edges=edges, rho_band_r=float(gamma), rho_band_b=1.0)
        out.append(dict(index=i, kind="bubble" if bubble else "slug", gamma=gamma, params=p, geo=geo,
                        steps=steps, gap=gap, nodes=p["nx"] * p["ny"]))
    return out


def geo_fields(geo, nx, ny):
    """Host colour-density fields of a ``serve_trace`` geometry."""
    if geo["kind"] == "disk":
        y, x = np.mgrid[0:ny, 0:nx]
        inside = (x + 0.5 - geo["cx"]) ** 2 + (y + 0.5 - geo["cy"]) ** 2 < geo["radius"] ** 2
        rr = np.where(inside, geo["rho_r_in"], geo["rho_r_out"])
        rb = np.where(inside, geo["rho_b_in"], geo["rho_b_out"])
        return rr.astype(np.float64), rb.astype(np.float64)
    edges = list(geo["edges"]) + [nx]
    red = np.zeros(nx, dtype=bool)
    for b in range(len(edges) - 1):
        red[edges[b]:edges[b + 1]] = (b % 2 == 0)
    rr = np.where(red, geo["rho_band_r"], 0.0)[None, :] * np.ones((ny, 1))
    rb = np.where(red, 0.0, geo["rho_band_b"])[None, :] * np.ones((ny, 1))
    return rr.astype(np.float64), rb.astype(np.float64)
