"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and arranges them in memory. It holds
none of the GEMM arithmetic: neither the oracle nor the GPU library imports it,
and it imports neither of them.

Every draw is made in float64 with ``numpy.random.default_rng(seed)`` and then
rounded to float32 by numpy's round-to-nearest-even cast, so a given seed gives
the same float32 bits on every machine.

Seed scheme: ``seed = 1000*config + role + 10*problem`` with the role offsets in
``ROLE`` below, so each operand of each workload has its own stream.
"""
from __future__ import annotations

import math

import numpy as np

ROLE = {"A": 0, "B": 1, "C": 2, "G": 3, "X": 4, "W1": 5, "W2": 6}


def seed_for(config: int, role: str, problem: int = 0) -> int:
    return 1000 * int(config) + ROLE[role] + 10 * int(problem)


def uniform(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """i.i.d. uniform[lo, hi) entries, drawn in float64, rounded to float32."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=shape).astype(np.float32)


def log_uniform_signed(shape, seed: int, lo_exp: float = -3.0, hi_exp: float = 3.0) -> np.ndarray:
    """|x| = 10**U(lo_exp, hi_exp) with a fair random sign, rounded to float32."""
    rng = np.random.default_rng(seed)
    mag = 10.0 ** rng.uniform(lo_exp, hi_exp, size=shape)
    sign = np.where(rng.random(size=shape) < 0.5, -1.0, 1.0)
    return (sign * mag).astype(np.float32)


def integers(shape, seed: int, lo: int = -8, hi: int = 8) -> np.ndarray:
    """Integer-valued float32 entries, uniform on [lo, hi] inclusive."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=shape).astype(np.float32)


def dyadic(shape, seed: int, bits: int = 4, exp_range: int = 3) -> np.ndarray:
    """Short dyadic rationals m * 2**e with |m| < 2**bits and |e| <= exp_range.

    Products and short sums of these are exact in float32 and float64, which
    makes exact-arithmetic comparisons possible.
    """
    rng = np.random.default_rng(seed)
    m = rng.integers(-(2 ** bits) + 1, 2 ** bits, size=shape).astype(np.float64)
    e = rng.integers(-exp_range, exp_range + 1, size=shape).astype(np.float64)
    return (m * np.exp2(e)).astype(np.float32)


def gaussian(shape, seed: int) -> np.ndarray:
    """i.i.d. N(0, 1) entries, rounded to float32."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=shape).astype(np.float32)


def batched_sizes(count: int, seed: int, lo: int = 32, hi: int = 2048, mult: int = 8):
    """(M, N, K) triples, each drawn log-uniformly on [lo, hi] and rounded to a multiple of ``mult``."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=(count, 3))
    v = np.rint(np.exp(u) / mult) * mult
    v = np.clip(v, lo, hi).astype(np.int64)
    return [tuple(int(x) for x in row) for row in v]


def store(logical: np.ndarray, trans: str, ld: int | None = None) -> tuple[np.ndarray, int]:
    """Lay out a logical (rows x cols) operand in row-major memory.

    trans 'N' stores it as is; 'T' stores its transpose (cols x rows). ``ld``
    (default: the minimum) is the row stride of the stored matrix in elements.
    Returns (buffer, ld) where buffer is a 1-D float32 array of
    stored_rows * ld elements (padding entries are filled with NaN so that a
    kernel that reads them shows it).
    """
    phys = logical if trans in "Nn" else logical.T
    rows, cols = phys.shape
    ld = max(cols, 1) if ld is None else int(ld)
    if ld < max(1, cols):
        raise ValueError("ld smaller than the stored row length")
    buf = np.full((max(rows, 1), ld), np.nan, dtype=np.float32)
    buf[:rows, :cols] = phys
    return buf.reshape(-1)[: rows * ld] if rows else buf.reshape(-1)[:0], ld


def sample_indices(rows: int, cols: int, count: int, seed: int):
    """``count`` distinct (i, j) output positions, always including the four corners."""
    rng = np.random.default_rng(seed)
    total = rows * cols
    count = min(count, total)
    flat = rng.choice(total, size=count, replace=False)
    corners = np.array([0, cols - 1, (rows - 1) * cols, total - 1], dtype=np.int64)
    flat = np.unique(np.concatenate([flat.astype(np.int64), corners]))
    return (flat // cols).astype(np.int64), (flat % cols).astype(np.int64)
