"""GPU parity of the FP16 path (operands rounded to IEEE binary16 while
packing, products on the FP16 matrix cores, FP32 accumulation).

Two bars, both against the FP64 oracle:
  * the path's own arithmetic: the oracle on the binary16-rounded operands.
    A product of two binary16 values is exact in FP32 (22 significant bits),
    so only the GPU's FP32 accumulation differs: bound 2e-6 (normalised);
  * the FP32 problem itself: <= 2e-3, the worst case of two binary16
    roundings per product (2 * 2^-11) plus FP32 accumulation at K = 8192
    (8192 * 2^-24), for operands inside the binary16 range.
"""
import itertools

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from helpers import Problem, TOL

pytestmark = pytest.mark.gpu

LAYOUTS = list(itertools.product("NT", "NT"))
EMU_TOL = 2e-6


def _native():
    from paper_2305_18236_amd import _native
    return _native


def _check(p, dev, cfg=None, use_workspace=True):
    nat = _native()
    if cfg is not None:
        assert nat.mg_force_config(4, cfg) == 0
    try:
        p.to_device(dev)
        st = p.run("fp16", use_workspace=use_workspace)
        assert st == 0, nat.status_string(st)
        C = p.result()
    finally:
        nat.mg_force_config(4, -1)
    Cref, D = p.oracle()
    err = oracle.normalized_error(C, Cref, D)
    Cemu, _ = oracle.gemm_logical(oracle.fp16_round(p.opA), oracle.fp16_round(p.opB), p.alpha, p.beta, p.C0)
    emu = oracle.normalized_error(C, Cemu, D)
    assert emu <= EMU_TOL, (p.M, p.N, p.K, p.tA, p.tB, "emulation", emu)
    assert err <= TOL["fp16"], (p.M, p.N, p.K, p.tA, p.tB, err)
    assert p.padding_untouched()
    return C, Cref, err


@pytest.mark.parametrize("tA,tB", LAYOUTS)
@pytest.mark.parametrize("M,N,K", [(256, 256, 256), (300, 517, 129), (1, 1, 1), (7, 9, 8), (33, 65, 31),
                                   (5, 300, 3)])
def test_ragged_shapes_all_layouts(gpu, tA, tB, M, N, K):
    _check(Problem(M, N, K, tA, tB, 1.5, 0.5, seed=M + 7 * N + 13 * K + 5), gpu)


@pytest.mark.parametrize("cfg", list(range(12)))
@pytest.mark.parametrize("tA,tB", LAYOUTS)
def test_every_config_every_layout(gpu, cfg, tA, tB):
    _check(Problem(530, 390, 77, tA, tB, -1.25, 0.75, seed=cfg + ord(tA) * 5 + ord(tB)), gpu, cfg=cfg)


@pytest.mark.parametrize("tA,tB", LAYOUTS)
@pytest.mark.parametrize("use_workspace", [True, False])
def test_prepacked_and_in_kernel_conversion(gpu, tA, tB, use_workspace):
    """M, N >= 512 converts each operand once into a binary16 plane in the
    workspace; without a workspace the GEMM converts while packing."""
    _check(Problem(600, 530, 300, tA, tB, 1.5, 0.5, seed=ord(tA) + 5 * ord(tB)), gpu,
           use_workspace=use_workspace)


def test_prepacked_split_k(gpu):
    """Pre-packed planes with the K loop split (few tiles, long K)."""
    _check(Problem(512, 520, 3000, "N", "T", 1.0, 0.5, seed=61), gpu)


@pytest.mark.parametrize("tA,tB", LAYOUTS)
def test_integer_inputs_bit_exact(gpu, tA, tB):
    """Integers in [-8, 8] are exact in binary16, so the result is exact."""
    C, Cref, _ = _check(Problem(200, 300, 250, tA, tB, 1.5, 0.5, seed=78, dist="integers"), gpu)
    assert np.array_equal(C, Cref)


def test_log_uniform_magnitudes(gpu):
    _check(Problem(384, 320, 640, "N", "N", 1.5, 0.5, seed=32, dist="log"), gpu)


def test_overflow_to_infinity(gpu):
    """An operand beyond the binary16 range rounds to infinity: its row of C
    is infinite (B positive), the other rows stay finite."""
    p = Problem(64, 48, 40, "N", "N", 1.0, 0.0, seed=63)
    p.opB = np.abs(p.opB) + np.float32(0.5)
    p.B, p.ldb = si.store(p.opB, "N")
    p.opA[5, 7] = np.float32(70000.0)
    p.A, p.lda = si.store(p.opA, "N")
    p.to_device(gpu)
    assert p.run("fp16") == 0
    C = p.result()
    assert np.all(np.isposinf(C[5]))
    assert np.isfinite(np.delete(C, 5, axis=0)).all()


def test_batched_fp16(gpu):
    import torch
    from paper_2305_18236_amd import gemm_batched
    shapes = [(40, 56, 33), (130, 70, 100), (8, 200, 64), (300, 260, 90)]
    probs, refs = [], []
    for i, (m, n, k) in enumerate(shapes):
        a, b = si.uniform((m, k), 70 + i), si.uniform((k, n), 80 + i)
        probs.append((torch.from_numpy(a).to(gpu), torch.from_numpy(b).to(gpu),
                      torch.zeros((m, n), device=gpu), 1.0, 0.0))
        refs.append(oracle.gemm_logical(a, b))
    gemm_batched(probs, path="fp16")
    torch.cuda.synchronize()
    for (_, _, c, _, _), (cref, d) in zip(probs, refs):
        assert oracle.normalized_error(c.cpu().numpy().astype(np.float64), cref, d) <= TOL["fp16"]


@pytest.mark.slow
@pytest.mark.parametrize("dist", ["uniform", "log"])
def test_full_size_8192_sampled(gpu, dist):
    p = Problem(8192, 8192, 8192, "N", "N", 1.0, 0.0, seed=3001, dist=dist).to_device(gpu)
    assert p.run("fp16") == 0
    C = p.result()
    I, J = si.sample_indices(8192, 8192, 4096, 98)
    cref, d = p.oracle_entries(I, J)
    err = oracle.normalized_error(C[I, J], cref, d)
    print(f"fp16 {dist} 8192^3 sampled normalised error {err:.3e}")
    assert err <= TOL["fp16"], err
