"""The no-allocation diagnostics entry point (lbm_diag_noalloc) against
lbm_diag through the C ABI: the same FP64 sums bit for bit, on two calls in a
row, the second on a smaller lattice (fewer reduction blocks than the first
left in the shared scratch), each with and without a pressure circle, after
some steps on a two-phase bubble."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_1903_01168_amd import capi
from paper_1903_01168_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-noalloc]", *a, file=sys.stderr, flush=True)


def _noalloc(L, lat, circle):
    d = capi.LbmDiag()
    c = None if circle is None else np.ascontiguousarray(circle, dtype=np.float64)
    rc = L.lbm_diag_noalloc(lat._h, None if c is None else c.ctypes.data_as(C.POINTER(C.c_double)), C.byref(d))
    assert rc == capi.LBM_OK, L.lbm_last_error(lat._h)
    return d.as_dict()


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_diag_noalloc_matches_diag(storage):
    L = capi.load()
    # 1024^2 needs the most blocks (2048), 96 x 80 a few (30)
    for n, nx, ny, r in ((1024, 1024, 1024, 300.0), (96, 96, 80, 20.0)):
        c = W.bubble_cell(10, 1, r, n=n, storage=storage)
        p = dict(c["params"], nx=nx, ny=ny)
        rr, rb = W.disk_fields(nx, ny, nx / 2, ny / 2, r, 1.0, 10.0)
        with capi.Lattice(p) as g:
            g.init(rr, rb)
            g.step(37)
            for circle in (None, (nx / 2, ny / 2, r - 4.0, r + 4.0)):
                ref = g.diag(circle=circle)
                got = _noalloc(L, g, circle)
                say(f"{storage} {nx}x{ny} circle={circle is not None}: mass_r {got['mass_r']:.17g} "
                    f"p_in {got['p_in']:.6g} max_u {got['max_u']:.3e}")
                assert got == ref
                assert got["n_nonfinite"] == 0 and got["mass_r"] > 0


def test_diag_noalloc_rejects_null():
    L = capi.load()
    p = W.params(nx=64, ny=64, A=1e-3)
    with capi.Lattice(p) as g:
        g.init(np.ones((64, 64)), np.zeros((64, 64)))
        assert L.lbm_diag_noalloc(g._h, None, None) == capi.LBM_E_INVAL
    assert L.lbm_diag_noalloc(None, None, None) == capi.LBM_E_INVAL
