"""Launch planning on the host: the step flavour, the workgroup width and the
strip height the library picks for a lattice.  The decisions are the ones the
header and the planner's comments state (measured on MI355X); results do not
depend on them (bit-identical launch shapes are a GPU test), so these checks
pin only that the planner makes the documented choice.  The planner functions
are internal C++ symbols of the shared library, called here by their mangled
names (no GPU is touched)."""
import ctypes
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1903_01168_amd", "libcglbm.so")

F32, F16S, BF16S = 0, 1, 2          # LBM_STORE_*
NSC, ISO = 1, 2                     # kernel variant bits
MIB = 1 << 20


@pytest.fixture(scope="module")
def plan():
    if not os.path.exists(LIB):
        pytest.skip("libcglbm.so not built")
    L = ctypes.CDLL(LIB)
    f = {}
    f["exchange"] = L["_ZN3cgi13plan_exchangeEmii"]
    f["exchange"].argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_int]
    f["exchange"].restype = ctypes.c_bool
    f["xch_tx"] = L["_ZN3cgi6xch_txEiii"]
    f["xch_tx"].argtypes = [ctypes.c_int] * 3
    f["xch_tx"].restype = ctypes.c_int
    f["default_tx"] = L["_ZN3cgi10default_txEii"]
    f["default_tx"].argtypes = [ctypes.c_int] * 2
    f["default_tx"].restype = ctypes.c_int
    f["strip"] = L["_ZN3cgi10plan_stripExiiiibb"]
    f["strip"].argtypes = [ctypes.c_longlong] + [ctypes.c_int] * 4 + [ctypes.c_bool] * 2
    f["strip"].restype = ctypes.c_int
    return f


def test_flavour(plan):
    """Block exchange exactly for FP32 launches without the Navier-Stokes
    correction or the isotropic gradient whose population buffers exceed the
    256 MiB Infinity Cache; halo lanes otherwise."""
    channel = 2 * 8192 * 512 * 72       # both buffers of the 8192 x 512 channel, FP32
    assert plan["exchange"](channel, F32, 0)
    assert plan["exchange"](256 * MIB + 1, F32, 0)
    assert not plan["exchange"](256 * MIB, F32, 0)
    assert not plan["exchange"](channel, F16S, 0)
    assert not plan["exchange"](channel, BF16S, 0)
    assert not plan["exchange"](channel, F32, NSC)
    assert not plan["exchange"](channel, F32, ISO)


def test_exchange_width(plan):
    """1024 columns per workgroup, 512 where a lattice is tall enough for four
    1024-column workgroups per CU, at most 512 with the correction; narrower
    lattices get the widest workgroup their blocks fill."""
    assert plan["xch_tx"](8192, 512, 0) == 1024          # channel: 8 x 32 = 256 workgroups
    assert plan["xch_tx"](2048, 2048, 0) == 1024         # 2 x 128 = 256
    assert plan["xch_tx"](8192, 8192, 0) == 512          # 8 x 512 = 4096 >= 4 per CU
    assert plan["xch_tx"](8192, 2048, 0) == 512          # 8 x 128 = 1024: exactly four per CU
    assert plan["xch_tx"](8192, 2032, 0) == 1024         # 8 x 127: one short
    assert plan["xch_tx"](8192, 512, NSC) == 512
    assert plan["xch_tx"](1024, 4096, 0) == 512          # 16 blocks across
    assert plan["xch_tx"](512, 4096, 0) == 256           # 8 blocks
    assert plan["xch_tx"](448, 4096, 0) == 64            # 7 blocks


def test_halo_lane_width(plan):
    assert plan["default_tx"](2048, 2048) == 256         # 4M nodes and beyond
    assert plan["default_tx"](2048, 2047) == 64
    assert plan["default_tx"](512, 512) == 64


def test_exchange_strip(plan):
    """The tallest strip up to 16 rows that still gives every CU a workgroup."""
    assert plan["strip"](8192 * 512, 512, 8, F32, 0, False, True) == 16     # channel
    assert plan["strip"](8192 * 256, 256, 8, F32, 0, False, True) == 8      # 8 x 32
    assert plan["strip"](2048 * 512, 512, 1, F32, 0, False, True) == 2      # 1 x 256
    assert plan["strip"](64 * 10, 10, 8, F32, 0, False, True) == 1
    assert plan["strip"](8192 * 12, 12, 64, F32, 0, False, True) == 2       # 64 x 6 rows of strips
    assert plan["strip"](19200 * 12, 12, 300, F32, 0, False, True) == 12    # no taller than the lattice


def test_halo_lane_strip(plan):
    """Short strips for small launches (latency), 6 rows from 1M to 3M nodes
    (8 for FP32 when two launches share the chip), then 4 rows for wide FP32
    lattices, 8 for narrow ones and for 16-bit storage."""
    s = plan["strip"]
    assert s(64 * 64, 64, 2, F32, 0, False, False) == 1
    assert s(1 << 17, 512, 9, F32, 0, False, False) == 1
    assert s((1 << 17) + 1, 512, 9, F32, 0, False, False) == 2
    assert s(999_999, 1024, 18, F16S, 0, False, False) == 2
    assert s(2_000_000, 1024, 18, F32, 0, False, False) == 6
    assert s(2_000_000, 1024, 18, F32, 0, True, False) == 8
    assert s(2_000_000, 1024, 18, F16S, 0, True, False) == 6
    assert s(16_000_000, 4096, 69, F32, 0, False, False) == 4
    assert s(16_000_000, 4096, 9, F32, 0, False, False) == 8
    assert s(16_000_000, 4096, 69, F16S, 0, False, False) == 8
    assert s(16_000_000, 3, 69, F32, 0, False, False) == 3


def test_requested_strip_wins(plan):
    assert plan["strip"](8192 * 512, 512, 8, F32, 5, False, True) == 5
    assert plan["strip"](8192 * 512, 512, 8, F32, 900, False, False) == 512
