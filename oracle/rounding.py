"""FP16 storage codes of the oracle: round-to-nearest and stochastic rounding (CPU, numpy).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/``, ``__graft_entry__.smoke()``
and ``bench.py``'s ``cpu_baseline`` leg may import it.  It shares no code with the HIP library.

FP16 storage is an addition to the paper (which fixes no precision): a population g_i is stored as the
FP16 code of the FP32 value v = (g_i - w_i phi_ref) * 2^scale_log2.  The deterministic code rounds v to
nearest (ties to even).  The stochastic code rounds |v| up to the next FP16 value with probability equal
to its distance from the value below, in units of the FP16 spacing (Croci & Giles 2020: stochastic
rounding keeps the rounding error's mean at zero, so small updates survive on average).  The random
numbers are 13-bit integers r, one per stored value, and |v| goes up iff r < floor(2^13 (|v| - lo) / ulp)
(the 13 bits of |v| below the FP16 spacing; exact for FP16 normal values).
They come from SplitMix64 (Steele, Lea & Flood 2014), written here from its definition: the generator
keeps a 64-bit state, adds gamma = 0x9e3779b97f4a7c15 per output and returns mix(state).  Node j of a
lattice of n nodes at time level t takes outputs 2(t n + j) and 2(t n + j) + 1, the 128-bit value
hi:lo, and population i the bits 13 i .. 13 i + 12.
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1
RBITS = 13  # random bits per stored value


# ---- SplitMix64 -----------------------------------------------------------------------------------

def splitmix64_mix(z: int) -> int:
    """The output function of SplitMix64 on one 64-bit integer (Python ints, exact)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_sequence(seed: int, count: int) -> list:
    """The first `count` outputs of the generator started at state `seed`, stepped one at a time."""
    state, out = seed & MASK64, []
    for _ in range(count):
        state = (state + GAMMA) & MASK64
        out.append(splitmix64_mix(state))
    return out


def _mix_u64(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def splitmix64_at(seed: int, k) -> np.ndarray:
    """Output number k (counted from 0) of the generator started at `seed`: mix(seed + (k + 1) gamma),
    element-wise over an integer array k (arithmetic modulo 2^64)."""
    k = np.asarray(k).astype(np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & MASK64) + (k + np.uint64(1)) * np.uint64(GAMMA)
    return _mix_u64(state)


def node_random_ints(seed: int, nodes: int, node, level) -> np.ndarray:
    """The nine 13-bit integers of node `node` (y nx + x) at time level `level` of a lattice of `nodes`
    nodes: shape node.shape + (9,), dtype int64."""
    node = np.asarray(node, dtype=np.int64)
    level = np.broadcast_to(np.asarray(level, dtype=np.int64), node.shape)
    first = 2 * (level.astype(np.uint64) * np.uint64(nodes) + node.astype(np.uint64))
    lo = splitmix64_at(seed, first)
    hi = splitmix64_at(seed, first + np.uint64(1))
    out = np.empty(node.shape + (9,), dtype=np.int64)
    for i in range(9):
        b = RBITS * i
        if b + RBITS <= 64:
            v = lo >> np.uint64(b)
        elif b >= 64:
            v = hi >> np.uint64(b - 64)
        else:
            v = (lo >> np.uint64(b)) | (hi << np.uint64(64 - b))
        out[..., i] = (v & np.uint64((1 << RBITS) - 1)).astype(np.int64)
    return out


# ---- FP32 -> FP16 rounding --------------------------------------------------------------------------

F16_MAX = 65504.0


def f16_floor_neighbours(a: np.ndarray):
    """For finite a >= 0 (float64 holding FP32 values): the largest FP16 value lo <= a and the FP16
    spacing above it (lo + ulp is the next FP16 value; 65504 + 32 stands for the overflow)."""
    a = np.asarray(a, dtype=np.float64)
    with np.errstate(over="ignore"):
        h = np.minimum(a, F16_MAX).astype(np.float16)  # nearest FP16 value
    h = np.where(h.astype(np.float64) > a, np.nextafter(h, np.float16(0)), h)
    with np.errstate(over="ignore"):
        ulp = np.spacing(h).astype(np.float64)
    return h.astype(np.float64), np.where(h.astype(np.float64) == F16_MAX, 32.0, ulp)


def f16_round_nearest(v) -> np.ndarray:
    """FP32 values to FP16, round to nearest, ties to even (numpy's conversion)."""
    with np.errstate(over="ignore"):
        return np.asarray(v, dtype=np.float32).astype(np.float16)


def f16_round_stochastic(v, r) -> np.ndarray:
    """FP32 values v to FP16 by stochastic rounding with 13-bit integers r (same shape).  With lo <= |v|
    the FP16 value below and ulp the FP16 spacing above it, m = floor(2^13 (|v| - lo) / ulp) is the
    13-bit integer of |v| below the spacing (finer bits, which exist only in the FP16 subnormal range,
    are dropped); |v| goes up to lo + ulp iff r < m.  The sign is kept; rounding up from 65504, or a
    magnitude of 65536 or more, gives infinity."""
    v = np.asarray(v, dtype=np.float32)
    a = np.abs(v.astype(np.float64))
    lo, ulp = f16_floor_neighbours(a)
    m = np.floor((a - lo) / ulp * 2 ** RBITS)   # exact: power-of-two scalings of an FP32 difference
    up = np.asarray(r, dtype=np.float64) < m
    mag = np.where(a >= 65536.0, np.inf, lo + np.where(up, ulp, 0.0))
    with np.errstate(over="ignore"):
        out = np.where(mag > F16_MAX, np.inf, mag).astype(np.float16)
    return np.where(np.signbit(v), -out, out)


# ---- the stored code of a population ---------------------------------------------------------------

def f16s_value(g, wref, scale_log2: int) -> np.ndarray:
    """The FP32 value that the FP16 code stores: (float32(g) - float32(w_i phi_ref)) * 2^scale_log2,
    each operation rounded to FP32 (the scale is a power of two, exact).  g has shape (9, ...), wref (9,)."""
    g32 = np.asarray(g, dtype=np.float64).astype(np.float32)
    w32 = np.asarray(wref, dtype=np.float64).astype(np.float32).reshape((-1,) + (1,) * (g32.ndim - 1))
    return ((g32 - w32) * np.float32(2.0 ** scale_log2)).astype(np.float32)


def f16s_decode(code, wref, scale_log2: int) -> np.ndarray:
    """g_i = code * 2^-scale_log2 + w_i phi_ref (FP64; code shape (9, ...))."""
    c = np.asarray(code).astype(np.float64)
    w = np.asarray(wref, dtype=np.float64).astype(np.float32).astype(np.float64).reshape((-1,) + (1,) * (c.ndim - 1))
    return c * 2.0 ** -scale_log2 + w
