"""The numpy model of 16-bit storage used to size full-size GPU bounds:
it keeps each node's colour mass, keeps an absent colour absent, and moves a
population by no more than the format's quanta."""
import numpy as np

from paper_1903_01168_amd import workloads as W
from storage16 import quantise


def _pops(seed=0):
    rng = np.random.default_rng(seed)
    p = W.params(nx=40, ny=30, rho0_r=1.0, rho0_b=10.0)
    w = np.array([0.2] + [0.16] * 4 + [0.04] * 4)          # rho0 phi of the light fluid by class
    frac = rng.random((30, 40))
    frac[:, :10] = 1.0
    frac[:, 30:] = 0.0
    pops = np.empty((2, 9, 30, 40))
    for i in range(9):
        n = w[i] * (1 + 0.01 * rng.standard_normal((30, 40)))
        pops[0, i] = frac * n
        pops[1, i] = (1 - frac) * n * (10.0 if i == 0 else 1.0)
    return p, pops


def test_colour_mass_kept_per_node():
    p, pops = _pops()
    q = quantise(pops, p, "f16s")
    for k in range(2):
        m0, m1 = pops[k].sum(axis=0), q[k].sum(axis=0)
        assert np.max(np.abs(m1 - m0)) <= 1e-6 * np.max(m0)


def test_absent_colour_stays_absent():
    p, pops = _pops()
    for kind in ("f16s", "bf16s"):
        q = quantise(pops, p, kind)
        assert np.all(q[1, 1:, :, :10] == 0.0) and np.all(q[0, 1:, :, 30:] == 0.0)


def test_moving_populations_within_quanta():
    p, pops = _pops()
    q = quantise(pops, p, "f16s")
    n0 = pops[0, 1:] + pops[1, 1:]
    n1 = q[0, 1:] + q[1, 1:]
    dev = np.abs(n0 - np.where(np.arange(1, 9)[:, None, None] <= 4, 0.16, 0.04))
    assert np.all(np.abs(n1 - n0) <= dev * 2.0 ** -11 + 1e-12)           # FP16 half-ulp of the deviation
    share0 = pops[0, 1:] / n0
    share1 = q[0, 1:] / n1
    assert np.max(np.abs(share1 - share0)) <= 0.5 / 65535 + 1e-9
