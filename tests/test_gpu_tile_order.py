"""GPU: the order in which the single-GEMM kernels walk their output tiles
(mg_force_tile_order) changes where each tile runs, never a result bit.

Every path, at two ragged multi-tile shapes: one whose tile counts are not a
multiple of 8 (the XCD remap does not apply) and one whose are (it does),
with groups that divide the tile rows and groups that do not.  Each order's
result is compared bit for bit with the automatic order's, and that one with
the oracle (the path's tolerance; INT8 exactly).
"""
import numpy as np
import pytest

import oracle
from helpers import Problem, tolerance
from test_gpu_i8 import I8Problem

pytestmark = pytest.mark.gpu

ORDERS = [(1, 4), (0, 4), (0, 1), (0, 3), (1, 16), (0, 64)]
SHAPES = [(600, 520, 300), (1024, 512, 384)]
PATHS = {"fp32": 0, "bf16x3": 1, "bf16": 2, "fp8": 3, "fp16": 4}


def _native():
    from paper_2305_18236_amd import _native
    return _native


@pytest.mark.parametrize("path", list(PATHS))
@pytest.mark.parametrize("M,N,K", SHAPES)
def test_tile_orders_bitwise_identical(gpu, path, M, N, K):
    nat = _native()
    pid = PATHS[path]
    p = Problem(M, N, K, "N", "T", 1.25, -0.5, seed=M + N + pid).to_device(gpu)
    assert p.run(path) == 0
    base = p.result()
    Cref, D = p.oracle()
    assert oracle.normalized_error(base, Cref, D) <= tolerance(path, K)
    for remap, gm in ORDERS:
        assert nat.mg_force_tile_order(pid, remap, gm) == 0
        try:
            p.reset_c()
            assert p.run(path) == 0
            C = p.result()
        finally:
            nat.mg_force_tile_order(pid, -1)
        assert np.array_equal(C, base), (path, M, N, K, remap, gm)
        assert p.padding_untouched()


@pytest.mark.parametrize("M,N,K", SHAPES)
def test_tile_orders_int8_exact(gpu, M, N, K):
    nat = _native()
    ref = I8Problem(M, N, K, "N", "T", alpha=3, beta=-1, seed=M + K).oracle()
    for remap, gm in ORDERS:
        assert nat.mg_force_tile_order(5, remap, gm) == 0
        try:
            C = I8Problem(M, N, K, "N", "T", alpha=3, beta=-1, seed=M + K).run(gpu)
        finally:
            nat.mg_force_tile_order(5, -1)
        assert np.array_equal(C, ref), (M, N, K, remap, gm)
