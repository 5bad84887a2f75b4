"""ctypes binding of the solve server of ``include/cglbm_serve.h``.

Marshalling only: the scheduler, the admission control and the batched
stepping all run in ``libcglbm.so``.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import capi

LBM_INIT_FIELDS, LBM_INIT_DISK, LBM_INIT_BANDS = 0, 1, 2
_P = C.c_void_p
_D = C.POINTER(C.c_double)


class InitDesc(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("n_edges", C.c_int32),
        ("rho_r", _D), ("rho_b", _D), ("ux", _D), ("uy", _D),
        ("cx", C.c_double), ("cy", C.c_double), ("radius", C.c_double),
        ("rho_r_in", C.c_double), ("rho_b_in", C.c_double),
        ("rho_r_out", C.c_double), ("rho_b_out", C.c_double),
        ("edges", C.POINTER(C.c_int32)),
        ("rho_band_r", C.c_double), ("rho_band_b", C.c_double),
        ("inlet_color", C.POINTER(C.c_int8)),
    ]


class Result(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("slot", C.c_int32), ("steps_done", C.c_int64),
        ("t_arrive", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
        ("diag", capi.LbmDiag),
        ("rho_r", _D), ("rho_b", _D), ("ux", _D), ("uy", _D), ("p", _D),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("enqueued", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
        ("chunks", C.c_int64), ("launches", C.c_int64), ("peak_active", C.c_int64),
        ("peak_bytes", C.c_uint64), ("lattice_updates", C.c_double), ("busy_s", C.c_double),
        ("admit_s", C.c_double), ("retire_s", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["lbm_server_create", "lbm_server_create_fake", "lbm_enqueue_solve", "lbm_poll", "lbm_wait",
           "lbm_release", "lbm_server_stats_get", "lbm_server_inject_failure", "lbm_server_destroy",
           "lbm_server_last_error"]

_DONE = False


def _lib():
    global _DONE
    L = capi.load()
    if not _DONE:
        L.lbm_server_create.argtypes = [C.c_size_t, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, C.POINTER(_P)]
        L.lbm_server_create_fake.argtypes = [C.c_size_t, C.c_int32, C.c_int32, C.c_double, C.POINTER(_P)]
        L.lbm_enqueue_solve.argtypes = [_P, C.POINTER(capi.LbmParams), C.POINTER(InitDesc), C.c_int64, C.c_int32,
                                        C.POINTER(C.c_uint64)]
        L.lbm_poll.argtypes = [_P, C.c_uint64, C.POINTER(Result)]
        L.lbm_wait.argtypes = [_P, C.c_uint64, C.POINTER(Result)]
        L.lbm_release.argtypes = [_P, C.c_uint64]
        L.lbm_server_stats_get.argtypes = [_P, C.POINTER(Stats)]
        L.lbm_server_inject_failure.argtypes = [_P, C.c_uint64]
        L.lbm_server_destroy.argtypes = [_P]
        L.lbm_server_last_error.restype = C.c_char_p
        L.lbm_server_last_error.argtypes = [_P]
        _DONE = True
    return L


def _f64(a, n):
    return None if a is None else np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(n))


def init_fields(rho_r, rho_b, ux=None, uy=None, inlet_color=None):
    return dict(kind=LBM_INIT_FIELDS, rho_r=rho_r, rho_b=rho_b, ux=ux, uy=uy, inlet_color=inlet_color)


def init_disk(cx, cy, radius, rho_r_in, rho_b_in, rho_r_out, rho_b_out):
    return dict(kind=LBM_INIT_DISK, cx=cx, cy=cy, radius=radius, rho_r_in=rho_r_in, rho_b_in=rho_b_in,
                rho_r_out=rho_r_out, rho_b_out=rho_b_out)


def init_bands(edges, rho_band_r, rho_band_b):
    return dict(kind=LBM_INIT_BANDS, edges=list(edges), rho_band_r=rho_band_r, rho_band_b=rho_band_b)


class Server:
    """A solve server (GPU backend), or with ``fake_mlups`` the host-only
    scheduler used for tests of the scheduling logic."""

    def __init__(self, hbm_budget, max_slots=64, chunk_steps=100, storage="f32", tile_x=0, stream=None,
                 fake_mlups=None):
        self.L = _lib()
        h = _P()
        if fake_mlups is not None:
            rc = self.L.lbm_server_create_fake(int(hbm_budget), int(max_slots), int(chunk_steps),
                                               float(fake_mlups), C.byref(h))
        else:
            rc = self.L.lbm_server_create(int(hbm_budget), int(max_slots), int(chunk_steps), capi.STORE[storage],
                                          int(tile_x), _P(stream) if stream else None, C.byref(h))
        if rc != capi.LBM_OK:
            raise capi.LbmError(rc, self.L.lbm_server_last_error(None).decode())
        self._h = h
        self._shapes = {}

    def close(self):
        if getattr(self, "_h", None):
            self.L.lbm_server_destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def enqueue(self, params: dict, init: dict, steps: int, keep_fields=False) -> int:
        cp = capi.make_params(params)
        n = int(params["nx"]) * int(params["ny"])
        keep = []
        d = InitDesc(kind=init["kind"])
        if init["kind"] == LBM_INIT_FIELDS:
            for k in ("rho_r", "rho_b", "ux", "uy"):
                a = _f64(init.get(k), n)
                keep.append(a)
                setattr(d, k, a.ctypes.data_as(_D) if a is not None else None)
        elif init["kind"] == LBM_INIT_DISK:
            for k in ("cx", "cy", "radius", "rho_r_in", "rho_b_in", "rho_r_out", "rho_b_out"):
                setattr(d, k, float(init[k]))
        else:
            e = np.ascontiguousarray(init["edges"], dtype=np.int32)
            keep.append(e)
            d.edges = e.ctypes.data_as(C.POINTER(C.c_int32))
            d.n_edges = len(e)
            d.rho_band_r, d.rho_band_b = float(init["rho_band_r"]), float(init["rho_band_b"])
        if init.get("inlet_color") is not None:
            ic = np.ascontiguousarray(init["inlet_color"], dtype=np.int8)
            keep.append(ic)
            d.inlet_color = ic.ctypes.data_as(C.POINTER(C.c_int8))
        rid = C.c_uint64()
        rc = self.L.lbm_enqueue_solve(self._h, C.byref(cp), C.byref(d), int(steps), int(bool(keep_fields)),
                                      C.byref(rid))
        if rc != capi.LBM_OK:
            raise capi.LbmError(rc, self.L.lbm_server_last_error(self._h).decode())
        self._shapes[rid.value] = (int(params["ny"]), int(params["nx"]), bool(keep_fields))
        return rid.value

    def _result(self, fn, rid, fields):
        res = Result()
        ny, nx, kept = self._shapes.get(rid, (0, 0, False))
        arrays = {}
        if fields and kept:
            for k in ("rho_r", "rho_b", "ux", "uy", "p"):
                arrays[k] = np.zeros((ny, nx))
                setattr(res, k, arrays[k].ctypes.data_as(_D))
        rc = fn(self._h, C.c_uint64(rid), C.byref(res))
        out = dict(rc=rc, status=res.status, slot=res.slot, steps_done=res.steps_done, t_arrive=res.t_arrive,
                   t_admit=res.t_admit, t_done=res.t_done, diag=res.diag.as_dict())
        out.update(arrays)
        return out

    def poll(self, rid, fields=False):
        return self._result(self.L.lbm_poll, rid, fields)

    def wait(self, rid, fields=False):
        return self._result(self.L.lbm_wait, rid, fields)

    def release(self, rid):
        return self.L.lbm_release(self._h, C.c_uint64(rid))

    def inject_failure(self, rid):
        return self.L.lbm_server_inject_failure(self._h, C.c_uint64(rid))

    def stats(self):
        st = Stats()
        self.L.lbm_server_stats_get(self._h, C.byref(st))
        return st.as_dict()
