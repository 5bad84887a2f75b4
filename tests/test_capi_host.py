"""Host-side checks of the C ABI: the library loads, exports every function the
header declares, and validates parameters (no GPU calls)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1903_01168_amd import build as B
from paper_1903_01168_amd import capi
from paper_1903_01168_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if B.is_stale():
        B.build()
    return capi.load()


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_\w+)\s*\(", text)))


def test_exports_match_header(lib):
    from paper_1903_01168_amd import serve
    declared = _declared("cglbm.h") + _declared("cglbm_serve.h")
    out = subprocess.run(["nm", "-D", "--defined-only", capi.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (lbm_\w+)$", out, flags=re.M))
    missing = [d for d in declared if d not in exported]
    assert not missing, missing
    for name in declared:
        assert hasattr(lib, name)
    assert set(capi.EXPORTS) | set(serve.EXPORTS) == set(declared)


def test_version(lib):
    assert capi.version().startswith("cglbm")


def _bytes(p):
    return capi.load().lbm_bytes_required(C.byref(capi.make_params(p)))


def test_layout_sizes(lib):
    p = W.params(nx=100, ny=10)
    cp = capi.make_params(p)
    # 18 planes, pitch padded to 64
    assert lib.lbm_buffer_bytes(C.byref(cp)) == 18 * 128 * 10 * 4
    p16 = W.params(nx=100, ny=10, storage="f16s")
    assert lib.lbm_buffer_bytes(C.byref(capi.make_params(p16))) == 40 * 128 * 10   # FP32 rest + 8 x 16-bit
    assert _bytes(p) > 2 * 18 * 128 * 10 * 4


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(tau_r=0.5), dict(tau_b=0.4), dict(beta=1.5), dict(rho0_r=0.0),
    dict(A=1e-3, sigma=1e-3), dict(alpha_light=1.0), dict(delta=0.0),
    dict(bc_x="open", p_out=0.0), dict(bc_x="open", nx=1, p_out=0.48),
    dict(bc_x="open", p_out=0.48, u_in_r=1.5),
    dict(contact_angle=60.0), dict(bc_y="walls", contact_angle=181.0),
    dict(ns_correction=True),                         # the correction is an MRT source
])
def test_validation_rejects(lib, bad):
    kw = dict(nx=16, ny=8, A=1e-3)
    kw.update(bad)
    assert _bytes(W.params(**kw)) == 0


def test_validation_accepts(lib):
    for kw in (dict(), dict(bc_x="open", p_out=0.48), dict(bc_y="walls", gx=1e-6), dict(bc_y="freeslip"),
               dict(bc_y="slip_top", bc_x="open", p_out=0.48), dict(collision="mrt"), dict(storage="bf16s"),
               dict(A=0.0, sigma=1e-3), dict(bc_y="walls", contact_angle=60.0),
               dict(bc_y="slip_top", contact_angle=0.0), dict(bc_y="freeslip", contact_angle=180.0),
               dict(collision="mrt", ns_correction=True),
               dict(collision="mrt", ns_correction=True, bc_x="open", p_out=0.48, bc_y="walls")):
        base = dict(nx=16, ny=8, A=1e-3)
        base.update(kw)
        assert _bytes(W.params(**base)) > 0


def test_unpaired_faces_rejected(lib):
    cp = capi.make_params(W.params(nx=16, ny=8, A=1e-3))
    cp.bc_xhi = capi.BC["zouhe_pressure"]
    assert lib.lbm_bytes_required(C.byref(cp)) == 0
    cp = capi.make_params(W.params(nx=16, ny=8, A=1e-3))
    cp.bc_ylo = capi.BC["bounceback"]
    assert lib.lbm_bytes_required(C.byref(cp)) == 0
    cp = capi.make_params(W.params(nx=16, ny=8, A=1e-3))
    cp.bc_ylo = cp.bc_yhi = capi.BC["zouhe_velocity"]
    assert lib.lbm_bytes_required(C.byref(cp)) == 0
    cp = capi.make_params(W.params(nx=16, ny=8, A=1e-3))
    cp.bc_ylo = capi.BC["freeslip"]                     # a wall against a periodic face
    assert lib.lbm_bytes_required(C.byref(cp)) == 0
    cp = capi.make_params(W.params(nx=16, ny=8, A=1e-3))
    cp.bc_xlo = cp.bc_xhi = capi.BC["freeslip"]         # free slip is a y-face condition
    assert lib.lbm_bytes_required(C.byref(cp)) == 0


def test_wetting_fields_validated(lib):
    cp = capi.make_params(W.params(nx=16, ny=8, A=1e-3, bc_y="walls"))
    assert cp.wetting == 0 and lib.lbm_bytes_required(C.byref(cp)) > 0
    cp.contact_angle = float("nan")                     # ignored while wetting is 0
    assert lib.lbm_bytes_required(C.byref(cp)) > 0
    cp.wetting = 1
    assert lib.lbm_bytes_required(C.byref(cp)) == 0
    cp.contact_angle = 45.0
    assert lib.lbm_bytes_required(C.byref(cp)) > 0
    cp.wetting = 2
    assert lib.lbm_bytes_required(C.byref(cp)) == 0
    cp.wetting, cp.reserved0 = 1, 7
    assert lib.lbm_bytes_required(C.byref(cp)) == 0


def test_ns_correction_fields_validated(lib):
    cp = capi.make_params(W.params(nx=16, ny=8, A=1e-3, collision="mrt", ns_correction=True))
    assert cp.ns_correction == 1 and lib.lbm_bytes_required(C.byref(cp)) > 0
    cp.ns_correction = 2
    assert lib.lbm_bytes_required(C.byref(cp)) == 0
    cp.ns_correction, cp.reserved1 = 1, 1
    assert lib.lbm_bytes_required(C.byref(cp)) == 0


def test_gradient_field_validated(lib):
    cp = capi.make_params(W.params(nx=16, ny=8, A=1e-3, gradient="isotropic"))
    assert cp.gradient == 1 and lib.lbm_bytes_required(C.byref(cp)) > 0
    cp.gradient = 2
    assert lib.lbm_bytes_required(C.byref(cp)) == 0
    cp.gradient, cp.reserved2 = 1, 3
    assert lib.lbm_bytes_required(C.byref(cp)) == 0


def test_header_is_c99_and_structs_match_the_binding(tmp_path):
    """The public headers compile as plain C99, and the ctypes mirrors of
    their structs have the C layout (size and every field offset)."""
    from paper_1903_01168_amd import serve
    mirrors = [("lbm_params", capi.LbmParams), ("lbm_diag_t", capi.LbmDiag), ("lbm_init_desc", serve.InitDesc),
               ("lbm_result", serve.Result), ("lbm_server_stats", serve.Stats)]
    body = []
    for cname, py in mirrors:
        body.append(f'  printf("%zu\\n", sizeof({cname}));\n')
        body += [f'  printf("%zu\\n", offsetof({cname}, {f}));\n' for f, _ in py._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "cglbm.h"\n#include "cglbm_serve.h"\n'
                   "int main(void) {\n" + "".join(body) + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                    os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = []
    for _, py in mirrors:
        want.append(C.sizeof(py))
        want += [getattr(py, f).offset for f, _ in py._fields_]
    assert out == want


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus above 1 exits with status 2 and a
    message, before touching a device."""
    import json
    import subprocess
    import sys as _sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([_sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    line = json.loads(out.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


@pytest.mark.parametrize("storage,per_node", [("f32", 36), ("f16s", 20), ("bf16s", 20)])
def test_largest_lattice_accepted_next_rejected(lib, storage, per_node):
    """A colour half of a buffer must stay below 4 GiB (32-bit buffer offsets):
    at nx = 65536 the tallest lattice accepted is the last one whose half is
    below 2^32 - 4096 bytes, one row more is rejected."""
    nx = 65536
    ny = ((1 << 32) - 4096 - 1) // (per_node * nx)
    assert _bytes(W.params(nx=nx, ny=ny, A=1e-3, storage=storage)) > 0
    assert _bytes(W.params(nx=nx, ny=ny + 1, A=1e-3, storage=storage)) == 0
