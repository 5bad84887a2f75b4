"""FP64 CPU oracle of the colour-gradient LBM step (test infrastructure).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
import this package.  It wraps ``libcgoracle.so`` (plain C, built by
``oracle/build.py``) with ctypes and shares nothing with the HIP path.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

OR_BCX_PERIODIC, OR_BCX_OPEN = 0, 1
OR_BCY_PERIODIC, OR_BCY_WALLS = 0, 1
OR_BGK, OR_MRT = 0, 1


class OrParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int),
        ("bc_x", C.c_int), ("bc_y", C.c_int),
        ("collision", C.c_int), ("percolor", C.c_int),
        ("rho0_r", C.c_double), ("rho0_b", C.c_double),
        ("alpha_light", C.c_double),
        ("tau_r", C.c_double), ("tau_b", C.c_double),
        ("delta", C.c_double),
        ("A", C.c_double), ("sigma", C.c_double),
        ("beta", C.c_double), ("mrt_lambda", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double),
        ("u_in_r", C.c_double), ("u_in_b", C.c_double),
        ("p_out", C.c_double),
        ("slip_lo", C.c_int), ("slip_hi", C.c_int),
        ("contact_angle", C.c_double),
        ("ns_correction", C.c_int),
        ("gradient", C.c_int),
        ("alt", C.c_int),
    ]


# or_params.alt: alternative readings of rules the paper leaves open
ALT_Q_WALL_ZERO, ALT_ISO_EXTRAP, ALT_OUTLET_UPSTREAM = 1, 2, 4


_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)


def lib():
    """Load (building first if needed) the oracle shared library."""
    global _LIB
    if _LIB is None:
        if _build.is_stale():
            _build.build()
        L = C.CDLL(_build.LIB)
        L.or_create.restype = C.c_void_p
        L.or_create.argtypes = [C.POINTER(OrParams)]
        L.or_destroy.argtypes = [C.c_void_p]
        L.or_init.argtypes = [C.c_void_p, _D, _D, _D, _D]
        L.or_set_inlet_color.argtypes = [C.c_void_p, C.POINTER(C.c_int8)]
        L.or_step.argtypes = [C.c_void_p, C.c_long]
        L.or_moments.argtypes = [C.c_void_p, _D, _D, _D, _D, _D]
        L.or_get_pops.argtypes = [C.c_void_p, _D]
        L.or_set_pops.argtypes = [C.c_void_p, _D]
        L.or_gradients.argtypes = [C.c_void_p, _D, _D, _D, _D]
        L.or_round_f32.argtypes = [C.c_void_p]
        L.or_step_count.restype = C.c_long
        L.or_step_count.argtypes = [C.c_void_p]
        L.or_threads.restype = C.c_int
        L.or_lattice.argtypes = [_I, _I, _I, _D]
        L.or_tables.argtypes = [C.c_double, _D, _D, _D]
        L.or_alphas.argtypes = [C.c_double, C.c_double, C.c_double, _D, _D]
        L.or_equilibrium.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, _D]
        L.or_omega_eff.restype = C.c_double
        L.or_omega_eff.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
        L.or_gradient3x3.argtypes = [_D, _D]
        L.or_gradient5x5.argtypes = [_D, _D]
        L.or_perturbation.argtypes = [_D, C.c_double, _D]
        L.or_wetting.argtypes = [_D, _D, C.c_double, _D]
        L.or_recolor.argtypes = [_D, C.c_double, C.c_double, _D, C.c_double, C.c_double,
                                 C.c_double, _D, _D]
        L.or_zouhe_west.restype = C.c_double
        L.or_zouhe_west.argtypes = [_D, C.c_double, C.c_double, C.c_double]
        L.or_zouhe_east.restype = C.c_double
        L.or_zouhe_east.argtypes = [_D, C.c_double, C.c_double, C.c_double]
        L.or_equilibrium_hermite.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, _D]
        L.or_ns_source.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, _D]
        L.or_mrt_matrices.argtypes = [_D, _D]
        L.or_mrt_collide.argtypes = [_D, _D, C.c_double, C.c_double, _D]
        _LIB = L
    return _LIB


def _p(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- node level
def lattice():
    cx = (C.c_int * 9)(); cy = (C.c_int * 9)(); opp = (C.c_int * 9)(); W = np.zeros(9)
    lib().or_lattice(cx, cy, opp, _p(W))
    return np.array(cx[:]), np.array(cy[:]), np.array(opp[:]), W


def tables(alpha):
    phi, B, xi = np.zeros(9), np.zeros(9), np.zeros(9)
    lib().or_tables(alpha, _p(phi), _p(B), _p(xi))
    return phi, B, xi


def alphas(rho0_r, rho0_b, alpha_light=0.2):
    ar, ab = C.c_double(), C.c_double()
    lib().or_alphas(rho0_r, rho0_b, alpha_light, C.byref(ar), C.byref(ab))
    return ar.value, ab.value


def equilibrium(rho_k, ux, uy, alpha_k):
    out = np.zeros(9)
    lib().or_equilibrium(rho_k, ux, uy, alpha_k, _p(out))
    return out


def equilibrium_hermite(rho_k, ux, uy, alpha_k):
    """Sec. 2.1.3 eq. (equilibrium_hermite)."""
    out = np.zeros(9)
    lib().or_equilibrium_hermite(rho_k, ux, uy, alpha_k, _p(out))
    return out


def ns_source(dqx, dqy, s1, s7):
    """Sec. 2.1.3: U = M^-1 C of the Navier-Stokes correction."""
    out = np.zeros(9)
    lib().or_ns_source(dqx, dqy, s1, s7, _p(out))
    return out


def omega_eff(psi, omega_r, omega_b, delta=0.1):
    return lib().or_omega_eff(psi, omega_r, omega_b, delta)


def gradient3x3(patch):
    """patch[dy+1][dx+1] = psi(x+dx, y+dy)."""
    p9 = _f64(np.asarray(patch).reshape(9)); F = np.zeros(2)
    lib().or_gradient3x3(_p(p9), _p(F))
    return F


def gradient5x5(patch):
    """Second-neighbour isotropic colour gradient of a 5 x 5 patch [dy][dx]."""
    F = np.zeros(2)
    lib().or_gradient5x5(_p(_f64(np.asarray(patch).reshape(25))), _p(F))
    return F


def perturbation(F, A):
    F2 = _f64(F); out = np.zeros(9)
    lib().or_perturbation(_p(F2), A, _p(out))
    return out


def recolor(Nss, rho_r, rho_b, F, beta, alpha_r, alpha_b):
    N = _f64(Nss); F2 = _f64(F); r = np.zeros(9); b = np.zeros(9)
    lib().or_recolor(_p(N), rho_r, rho_b, _p(F2), beta, alpha_r, alpha_b, _p(r), _p(b))
    return r, b


def zouhe_west(N, vx, vy, kap=0.0):
    N = _f64(N).copy()
    rho = lib().or_zouhe_west(_p(N), vx, vy, kap)
    return rho, N


def zouhe_east(N, rho, vy, kap=0.0):
    N = _f64(N).copy()
    vx = lib().or_zouhe_east(_p(N), rho, vy, kap)
    return vx, N


def mrt_matrices():
    M, Mi = np.zeros(81), np.zeros(81)
    lib().or_mrt_matrices(_p(M), _p(Mi))
    return M.reshape(9, 9), Mi.reshape(9, 9)


def mrt_collide(N, Neq, omega, lam=0.8):
    N = _f64(N); E = _f64(Neq); out = np.zeros(9)
    lib().or_mrt_collide(_p(N), _p(E), omega, lam, _p(out))
    return out


def wetting(F2, ns2, theta):
    """Sec. 2.4: the colour gradient turned to the angle theta (radians) with
    the wall normal ns (into the fluid)."""
    out = np.zeros(2)
    lib().or_wetting(_p(_f64(F2)), _p(_f64(ns2)), float(theta), _p(out))
    return out


def threads():
    return lib().or_threads()


# ------------------------------------------------------------- lattice level
class Sim:
    """One lattice advanced by the oracle.

    Parameters mirror the public ``lbm_params`` struct: ``bc_x`` is
    "periodic" or "open" (velocity inlet west, pressure outlet east),
    ``bc_y`` is "periodic", "walls" (no-slip), "freeslip" (both walls) or
    "slip_top" (no-slip bottom, free-slip top); ``collision`` is "bgk" or
    "mrt".
    """

    BC_Y = {"periodic": (0, 0, 0), "walls": (1, 0, 0), "freeslip": (1, 1, 1), "slip_top": (1, 0, 1)}

    def __init__(self, nx, ny, *, bc_x="periodic", bc_y="periodic", collision="bgk",
                 percolor=False, rho0_r=1.0, rho0_b=1.0, alpha_light=0.2, tau_r=1.0,
                 tau_b=1.0, delta=0.1, A=0.0, sigma=0.0, beta=0.7, mrt_lambda=0.8,
                 gx=0.0, gy=0.0, u_in_r=0.0, u_in_b=0.0, p_out=0.0, contact_angle=-1.0,
                 ns_correction=False, gradient="nearest", alt=0, **_ignored):
        self.nx, self.ny = nx, ny
        by, slo, shi = self.BC_Y[bc_y]
        p = OrParams(nx=nx, ny=ny,
                     bc_x={"periodic": 0, "open": 1}[bc_x],
                     bc_y=by, slip_lo=slo, slip_hi=shi,
                     collision={"bgk": 0, "mrt": 1}[collision], percolor=int(percolor),
                     rho0_r=rho0_r, rho0_b=rho0_b, alpha_light=alpha_light,
                     tau_r=tau_r, tau_b=tau_b, delta=delta, A=A, sigma=sigma, beta=beta,
                     mrt_lambda=mrt_lambda, gx=gx, gy=gy, u_in_r=u_in_r, u_in_b=u_in_b,
                     p_out=p_out, contact_angle=contact_angle, ns_correction=int(bool(ns_correction)),
                     gradient={"nearest": 0, "isotropic": 1}[gradient], alt=int(alt))
        self._params = p
        self._h = lib().or_create(C.byref(p))
        if not self._h:
            raise ValueError("oracle: invalid lattice size")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_destroy(h)
            self._h = None

    def init(self, rho_r, rho_b, ux=None, uy=None):
        shape = (self.ny, self.nx)
        rr = _f64(rho_r).reshape(shape); rb = _f64(rho_b).reshape(shape)
        u = _f64(ux).reshape(shape) if ux is not None else None
        v = _f64(uy).reshape(shape) if uy is not None else None
        lib().or_init(self._h, _p(rr), _p(rb), _p(u) if u is not None else None,
                      _p(v) if v is not None else None)
        return self

    def set_inlet_color(self, color_y):
        c = np.ascontiguousarray(color_y, dtype=np.int8)
        assert c.shape == (self.ny,)
        lib().or_set_inlet_color(self._h, c.ctypes.data_as(C.POINTER(C.c_int8)))

    def step(self, n=1, round_f32=False):
        """n steps; round_f32: round the stored populations to FP32 after
        each (a storage model for measuring how the flow amplifies rounding)."""
        if not round_f32:
            lib().or_step(self._h, int(n))
            return self
        for _ in range(int(n)):
            lib().or_step(self._h, 1)
            lib().or_round_f32(self._h)
        return self

    @property
    def steps_done(self):
        return lib().or_step_count(self._h)

    def moments(self):
        n = self.nx * self.ny
        rr, rb, u, v, p = (np.zeros(n) for _ in range(5))
        lib().or_moments(self._h, _p(rr), _p(rb), _p(u), _p(v), _p(p))
        sh = (self.ny, self.nx)
        return dict(rho_r=rr.reshape(sh), rho_b=rb.reshape(sh), ux=u.reshape(sh),
                    uy=v.reshape(sh), p=p.reshape(sh))

    def get_pops(self):
        out = np.zeros((2, 9, self.ny, self.nx))
        lib().or_get_pops(self._h, _p(out))
        return out

    def set_pops(self, pops):
        a = _f64(pops).reshape(2, 9, self.ny, self.nx)
        lib().or_set_pops(self._h, _p(a))

    def gradients(self):
        """The colour gradient (before any contact-angle turn) and, with the
        Navier-Stokes correction, dQx/dx and dQy/dy per colour, that the next
        step would use; the state is not advanced."""
        sh = (self.ny, self.nx)
        Fx, Fy = np.zeros(sh), np.zeros(sh)
        dqx, dqy = np.zeros((2,) + sh), np.zeros((2,) + sh)
        lib().or_gradients(self._h, _p(Fx), _p(Fy), _p(dqx), _p(dqy))
        return dict(Fx=Fx, Fy=Fy, dqxdx=dqx, dqydy=dqy)
