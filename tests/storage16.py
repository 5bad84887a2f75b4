"""A plain numpy model of the 16-bit population storage (round to nearest),
applied to the FP64 oracle's stored state after every step: how far the
oracle itself moves when its populations live in that format is the floor
for comparing the 16-bit GPU path with FP64 in the max norm.

Format (as stated in include/cglbm.h): per moving direction i, the
colour-blind population N_i = N^r_i + N^b_i as a 16-bit float deviation from
rho0_k phi^k_i (the same for both fluids) scaled by 2^12 / max(rho0), and the
red share N^r_i / N_i as a 16-bit fixed-point fraction; the rest population of
each colour in FP32, holding the node's colour mass exactly."""
import numpy as np


def _to_bf16(x):
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def quantise(pops, params, kind="f16s"):
    """pops: [2][9][ny][nx] FP64 (colour, direction); returns the decoded
    state after one store in the 16-bit format."""
    r0l = min(params["rho0_r"], params["rho0_b"])
    r0h = max(params["rho0_r"], params["rho0_b"])
    alpha_l = params.get("alpha_light", 0.2)
    ref = {1: r0l * (1 - alpha_l) / 5.0, 2: r0l * (1 - alpha_l) / 20.0}   # rho0_k phi^k by class
    scale = 4096.0 / r0h
    out = pops.copy()
    moved = np.zeros((2,) + pops.shape[2:])
    for i in range(1, 9):
        m = ref[1] if i <= 4 else ref[2]
        nr, nb = pops[0, i], pops[1, i]
        n = nr + nb
        with np.errstate(divide="ignore", invalid="ignore"):
            g = np.clip(np.where(n != 0, nr / n, 0.0), 0.0, 1.0)
        g = np.where(nb == 0, 1.0, np.where(nr == 0, 0.0, g))
        gq = np.round(g * 65535.0) / 65535.0
        x = (n - m) * scale
        xq = np.float16(x).astype(np.float64) if kind == "f16s" else _to_bf16(x)
        nq = m + xq / scale
        out[0, i], out[1, i] = gq * nq, (1.0 - gq) * nq
        moved[0] += out[0, i]
        moved[1] += out[1, i]
    for k in range(2):
        out[k, 0] = pops[k].sum(axis=0) - moved[k]     # the rest keeps the colour mass
        out[k, 0] = out[k, 0].astype(np.float32).astype(np.float64)
    return out
