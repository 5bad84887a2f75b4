"""ctypes binding of ``libcglbm.so`` (argument marshalling only).

Every step of the method runs in the HIP kernels of the library; this module
converts numpy arrays and parameter dicts to the C structs of
``include/cglbm.h`` and raises on error codes.  It never falls back to any
other implementation: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcglbm.so")

LBM_OK, LBM_E_INVAL, LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_UNSTABLE, LBM_E_BUSY, LBM_E_NOTFOUND = 0, -1, -2, -3, -4, -5, -6
GRADIENT = {"nearest": 0, "isotropic": 1}
BC = {"periodic": 0, "bounceback": 1, "zouhe_velocity": 2, "zouhe_pressure": 3, "freeslip": 4}
# y-face pairs (low, high) by the ``bc_y`` names of ``workloads.params``
BC_Y = {"periodic": ("periodic", "periodic"), "walls": ("bounceback", "bounceback"),
        "freeslip": ("freeslip", "freeslip"), "slip_top": ("bounceback", "freeslip")}
COLL = {"bgk": 0, "mrt": 1}
STORE = {"f32": 0, "f16s": 1, "bf16s": 2}


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cglbm error {code}: {msg}")
        self.code = code


class LbmParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("bc_xlo", C.c_int32), ("bc_xhi", C.c_int32), ("bc_ylo", C.c_int32), ("bc_yhi", C.c_int32),
        ("collision", C.c_int32), ("storage", C.c_int32),
        ("rho0_r", C.c_double), ("rho0_b", C.c_double), ("alpha_light", C.c_double),
        ("tau_r", C.c_double), ("tau_b", C.c_double), ("delta", C.c_double),
        ("A", C.c_double), ("sigma", C.c_double), ("beta", C.c_double), ("mrt_lambda", C.c_double),
        ("gx", C.c_double), ("gy", C.c_double),
        ("u_in_r", C.c_double), ("u_in_b", C.c_double), ("p_out", C.c_double),
        ("wetting", C.c_int32), ("reserved0", C.c_int32), ("contact_angle", C.c_double),
        ("ns_correction", C.c_int32), ("reserved1", C.c_int32),
        ("gradient", C.c_int32), ("reserved2", C.c_int32),
    ]


class LbmDiag(C.Structure):
    _fields_ = [
        ("mass_r", C.c_double), ("mass_b", C.c_double), ("area_r", C.c_double), ("max_u", C.c_double),
        ("p_in", C.c_double), ("p_out", C.c_double),
        ("n_in", C.c_int64), ("n_out", C.c_int64), ("n_nonfinite", C.c_int64), ("step", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = [
    "lbm_version", "lbm_last_error", "lbm_bytes_required", "lbm_buffer_bytes", "lbm_create",
    "lbm_create_ext", "lbm_destroy", "lbm_init_fields", "lbm_set_inlet_color", "lbm_step",
    "lbm_steps_done", "lbm_sync", "lbm_moments", "lbm_diag", "lbm_diag_noalloc", "lbm_get_pops", "lbm_set_pops",
    "lbm_save_state", "lbm_load_state", "lbm_set_launch", "lbm_set_exchange", "lbm_stream", "lbm_bw_copy",
    "lbm_batch_create", "lbm_batch_step", "lbm_batch_destroy", "lbm_batch_last_error", "lbm_batch_groups",
    "lbm_batch_group_launch",
]

_LIB = None
_D = C.POINTER(C.c_double)
_P = C.c_void_p


def load(path: str = LIB_PATH):
    """Load the HIP library (raises OSError when it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise OSError(f"libcglbm.so not found at {path}: build it with paper_1903_01168_amd/build.py")
    L = C.CDLL(path)
    L.lbm_version.restype = C.c_char_p
    L.lbm_last_error.restype = C.c_char_p
    L.lbm_last_error.argtypes = [_P]
    L.lbm_bytes_required.restype = C.c_size_t
    L.lbm_bytes_required.argtypes = [C.POINTER(LbmParams)]
    L.lbm_buffer_bytes.restype = C.c_size_t
    L.lbm_buffer_bytes.argtypes = [C.POINTER(LbmParams)]
    L.lbm_create.argtypes = [C.POINTER(LbmParams), _P, C.POINTER(_P)]
    L.lbm_create_ext.argtypes = [C.POINTER(LbmParams), _P, _P, _P, C.c_size_t, C.POINTER(_P)]
    L.lbm_destroy.argtypes = [_P]
    L.lbm_init_fields.argtypes = [_P, _D, _D, _D, _D]
    L.lbm_set_inlet_color.argtypes = [_P, C.POINTER(C.c_int8)]
    L.lbm_step.argtypes = [_P, C.c_int64]
    L.lbm_steps_done.restype = C.c_int64
    L.lbm_steps_done.argtypes = [_P]
    L.lbm_sync.argtypes = [_P]
    L.lbm_moments.argtypes = [_P, _D, _D, _D, _D, _D, C.POINTER(LbmDiag)]
    L.lbm_diag.argtypes = [_P, _D, C.POINTER(LbmDiag)]
    L.lbm_diag_noalloc.argtypes = [_P, _D, C.POINTER(LbmDiag)]
    L.lbm_get_pops.argtypes = [_P, _D]
    L.lbm_set_pops.argtypes = [_P, _D]
    L.lbm_save_state.argtypes = [_P, _P, C.c_size_t, C.POINTER(C.c_size_t)]
    L.lbm_load_state.argtypes = [_P, _P, C.c_size_t]
    L.lbm_set_launch.argtypes = [_P, C.c_int32, C.c_int32]
    L.lbm_set_exchange.argtypes = [_P, C.c_int32]
    L.lbm_stream.restype = _P
    L.lbm_stream.argtypes = [_P]
    L.lbm_bw_copy.argtypes = [_P, _P, _P, C.c_size_t]
    L.lbm_batch_create.argtypes = [C.POINTER(_P), C.c_int32, C.c_int32, _P, C.POINTER(_P)]
    L.lbm_batch_step.argtypes = [_P, C.c_int64]
    L.lbm_batch_destroy.argtypes = [_P]
    L.lbm_batch_last_error.restype = C.c_char_p
    L.lbm_batch_last_error.argtypes = [_P]
    L.lbm_batch_groups.argtypes = [_P]
    L.lbm_batch_group_launch.argtypes = [_P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    _LIB = L
    return L


def make_params(p: dict) -> LbmParams:
    """C struct from a parameter dict (keys of ``workloads.params``)."""
    xper = p.get("bc_x", "periodic") == "periodic"
    ylo, yhi = BC_Y[p.get("bc_y", "periodic")]
    ca = float(p.get("contact_angle", -1.0))        # < 0: no wetting adjustment
    return LbmParams(
        nx=int(p["nx"]), ny=int(p["ny"]),
        bc_xlo=BC["periodic"] if xper else BC["zouhe_velocity"],
        bc_xhi=BC["periodic"] if xper else BC["zouhe_pressure"],
        bc_ylo=BC[ylo], bc_yhi=BC[yhi],
        collision=COLL[p.get("collision", "bgk")], storage=STORE[p.get("storage", "f32")],
        rho0_r=p["rho0_r"], rho0_b=p["rho0_b"], alpha_light=p["alpha_light"],
        tau_r=p["tau_r"], tau_b=p["tau_b"], delta=p["delta"], A=p["A"], sigma=p["sigma"],
        beta=p["beta"], mrt_lambda=p["mrt_lambda"], gx=p["gx"], gy=p["gy"],
        u_in_r=p["u_in_r"], u_in_b=p["u_in_b"], p_out=p["p_out"],
        wetting=1 if ca >= 0 else 0, contact_angle=ca if ca >= 0 else 0.0,
        ns_correction=int(bool(p.get("ns_correction", False))),
        gradient=GRADIENT[p.get("gradient", "nearest")])


def _f64(a, shape):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), shape))


def _ptr(a):
    return a.ctypes.data_as(_D) if a is not None else None


class Lattice:
    """One lattice on the GPU (a ``lbm_ctx``).

    ``stream``: an integer hipStream_t (e.g. ``torch.cuda.Stream().cuda_stream``)
    or None for a stream owned by the library.  ``buffers``: optional pair of
    device pointers (e.g. from torch tensors) of ``buffer_bytes`` each.
    """

    def __init__(self, params: dict, stream=None, buffers=None):
        self.L = load()
        self.params = dict(params)
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        self._cp = make_params(params)
        h = _P()
        if buffers is None:
            rc = self.L.lbm_create(C.byref(self._cp), _P(stream) if stream else None, C.byref(h))
        else:
            a, b = buffers
            rc = self.L.lbm_create_ext(C.byref(self._cp), _P(stream) if stream else None, _P(a), _P(b),
                                       self.buffer_bytes, C.byref(h))
        if rc != LBM_OK:
            raise LbmError(rc, self.L.lbm_last_error(None).decode())
        self._h = h

    @property
    def buffer_bytes(self) -> int:
        return int(self.L.lbm_buffer_bytes(C.byref(self._cp)))

    @property
    def bytes_required(self) -> int:
        return int(self.L.lbm_bytes_required(C.byref(self._cp)))

    def _check(self, rc):
        if rc != LBM_OK:
            raise LbmError(rc, self.L.lbm_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self.L.lbm_destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def stream(self) -> int:
        return int(self.L.lbm_stream(self._h) or 0)

    def init(self, rho_r, rho_b, ux=None, uy=None):
        sh = (self.ny, self.nx)
        rr, rb = _f64(rho_r, sh), _f64(rho_b, sh)
        u = _f64(ux, sh) if ux is not None else None
        v = _f64(uy, sh) if uy is not None else None
        self._check(self.L.lbm_init_fields(self._h, _ptr(rr), _ptr(rb), _ptr(u), _ptr(v)))
        return self

    def set_inlet_color(self, color_y):
        c = np.ascontiguousarray(color_y, dtype=np.int8)
        if c.shape != (self.ny,):
            raise ValueError("one colour per row")
        self._check(self.L.lbm_set_inlet_color(self._h, c.ctypes.data_as(C.POINTER(C.c_int8))))

    def step(self, n=1):
        self._check(self.L.lbm_step(self._h, int(n)))
        return self

    @property
    def steps_done(self) -> int:
        return int(self.L.lbm_steps_done(self._h))

    def sync(self):
        self._check(self.L.lbm_sync(self._h))

    def moments(self, check=True):
        sh = (self.ny, self.nx)
        out = {k: np.zeros(sh) for k in ("rho_r", "rho_b", "ux", "uy", "p")}
        d = LbmDiag()
        rc = self.L.lbm_moments(self._h, *(_ptr(out[k]) for k in ("rho_r", "rho_b", "ux", "uy", "p")),
                                C.byref(d))
        if rc != LBM_E_UNSTABLE or check:
            self._check(rc)
        out["diag"] = d.as_dict()
        return out

    def diag(self, circle=None, check=True):
        d = LbmDiag()
        c = np.ascontiguousarray(circle, dtype=np.float64) if circle is not None else None
        rc = self.L.lbm_diag(self._h, _ptr(c), C.byref(d))
        if rc != LBM_E_UNSTABLE or check:
            self._check(rc)
        return d.as_dict()

    def get_pops(self):
        out = np.zeros((2, 9, self.ny, self.nx))
        self._check(self.L.lbm_get_pops(self._h, _ptr(out)))
        return out

    def set_pops(self, pops):
        a = _f64(pops, (2, 9, self.ny, self.nx))
        self._check(self.L.lbm_set_pops(self._h, _ptr(a)))

    def save_state(self) -> bytes:
        n = C.c_size_t()
        self._check(self.L.lbm_save_state(self._h, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(self.L.lbm_save_state(self._h, buf, n.value, C.byref(n)))
        return buf.raw

    def load_state(self, blob: bytes):
        self._check(self.L.lbm_load_state(self._h, blob, len(blob)))

    def set_launch(self, tile_x=0, strip_rows=0, exchange=None):
        """Threads per workgroup and rows per strip (0: planned); exchange:
        True / False forces the block-exchange / halo-lane step, None plans."""
        self._check(self.L.lbm_set_launch(self._h, int(tile_x), int(strip_rows)))
        self._check(self.L.lbm_set_exchange(self._h, -1 if exchange is None else int(bool(exchange))))

    def bw_copy(self, dst_ptr, src_ptr, nbytes):
        self._check(self.L.lbm_bw_copy(self._h, _P(dst_ptr), _P(src_ptr), int(nbytes)))


class Batch:
    """Several lattices advanced by one kernel launch per step (``lbm_batch``)."""

    def __init__(self, lattices, tile_x=0, stream=None):
        self.L = load()
        self.lattices = list(lattices)
        arr = (_P * len(self.lattices))(*[lat._h for lat in self.lattices])
        h = _P()
        rc = self.L.lbm_batch_create(arr, len(self.lattices), int(tile_x), _P(stream) if stream else None,
                                     C.byref(h))
        if rc != LBM_OK:
            raise LbmError(rc, self.L.lbm_last_error(None).decode())
        self._h = h

    @property
    def groups(self) -> int:
        """Cache-sized groups, i.e. kernel launches per step."""
        return int(self.L.lbm_batch_groups(self._h))

    def group_launch(self, g):
        """(threads per workgroup, block-exchange flavour) of group g."""
        tx, xch = C.c_int32(), C.c_int32()
        rc = self.L.lbm_batch_group_launch(self._h, int(g), C.byref(tx), C.byref(xch))
        if rc != LBM_OK:
            raise LbmError(rc, self.L.lbm_last_error(None).decode())
        return tx.value, bool(xch.value)

    def step(self, n=1):
        rc = self.L.lbm_batch_step(self._h, int(n))
        if rc != LBM_OK:
            raise LbmError(rc, self.L.lbm_batch_last_error(self._h).decode())
        return self

    def close(self):
        if getattr(self, "_h", None):
            self.L.lbm_batch_destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def version() -> str:
    return load().lbm_version().decode()
