"""GPU parity of the BF16 matrix-core paths (plain BF16 and the bf16x3 split).

Two bars per path, both against the FP64 oracle:
  * the path's own arithmetic: the oracle applied to the bf16-rounded operands
    (BF16) or to the three split products hi*hi + hi*lo + lo*hi (bf16x3).
    Every bf16 product is exact in FP32, so the only difference left is the
    GPU's FP32 accumulation: bound 2e-6 (normalised);
  * the FP32 problem itself: <= 1e-2 (BF16) and <= 1e-5 (bf16x3).
And bit-exactness of the pack-stage conversion (mg_bf16_split) against the
oracle's round-to-nearest-even split.
"""
import itertools

import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si
from helpers import Problem, TOL, tolerance

pytestmark = pytest.mark.gpu

LAYOUTS = list(itertools.product("NT", "NT"))
EMU_TOL = 2e-6


def _native():
    from paper_2305_18236_amd import _native
    return _native


def _bits_to_f64(u16):
    return (u16.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _split_on_gpu(x, dev):
    nat = _native()
    n = x.size
    dx = torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(dev)
    hi = torch.empty(n, dtype=torch.int16, device=dev)
    lo = torch.empty(n, dtype=torch.int16, device=dev)
    st = nat.mg_bf16_split(dx.data_ptr(), n, hi.data_ptr(), lo.data_ptr(),
                           torch.cuda.current_stream().cuda_stream)
    assert st == 0, nat.status_string(st)
    torch.cuda.synchronize()
    return hi.cpu().numpy().view(np.uint16), lo.cpu().numpy().view(np.uint16)


def test_split_bit_exact(gpu):
    bits = (np.random.default_rng(3).integers(0x2000, 0x6000, 20000).astype(np.uint32) << 16) | 0x8000
    x = np.concatenate([si.uniform(100000, 1), si.log_uniform_signed(100000, 2),
                        si.log_uniform_signed(20000, 3, -38, 38), bits.view(np.float32),
                        np.array([0.0, -0.0, 1.0, -1.0, 1e-40, -3e-39, 2.0 ** -126], np.float32)])
    hi, lo = _split_on_gpu(x, gpu)
    ohi, olo = oracle.bf16_split(x)
    assert np.array_equal(_bits_to_f64(hi), ohi)
    assert np.array_equal(_bits_to_f64(lo), olo)


def _emulated_reference(p, terms):
    """The oracle on the path's own operands: bf16(op) or the three split products."""
    hiA, loA = oracle.bf16_split(p.opA)
    hiB, loB = oracle.bf16_split(p.opB)
    if terms == 1:
        C, _ = oracle.gemm_logical(hiA, hiB, p.alpha, p.beta, p.C0)
        return C
    C, _ = oracle.gemm_logical(hiA, hiB, p.alpha, p.beta, p.C0)
    C1, _ = oracle.gemm_logical(hiA, loB, p.alpha)
    C2, _ = oracle.gemm_logical(loA, hiB, p.alpha)
    return C + C1 + C2


def _check(p, dev, path, cfg=None, use_workspace=True):
    nat = _native()
    pid = {"bf16x3": 1, "bf16": 2}[path]
    if cfg is not None:
        assert nat.mg_force_config(pid, cfg) == 0
    try:
        p.to_device(dev)
        st = p.run(path, use_workspace=use_workspace)
        assert st == 0, nat.status_string(st)
        C = p.result()
    finally:
        nat.mg_force_config(pid, -1)
    Cref, D = p.oracle()
    err = oracle.normalized_error(C, Cref, D)
    emu = oracle.normalized_error(C, _emulated_reference(p, 3 if path == "bf16x3" else 1), D)
    assert emu <= EMU_TOL, (path, p.M, p.N, p.K, p.tA, p.tB, "emulation", emu)
    assert err <= tolerance(path, p.K), (path, p.M, p.N, p.K, p.tA, p.tB, err)
    assert p.padding_untouched()
    return C, Cref, err


@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
def test_256_cube(gpu, path):
    _check(Problem(256, 256, 256, "N", "N", 1.0, 0.0, seed=1000), gpu, path)


@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
@pytest.mark.parametrize("tA,tB", LAYOUTS)
@pytest.mark.parametrize("M,N,K", [(300, 517, 129), (1, 1, 1), (7, 9, 8), (33, 65, 31), (5, 300, 3)])
def test_ragged_shapes_all_layouts(gpu, path, tA, tB, M, N, K):
    _check(Problem(M, N, K, tA, tB, 1.5, 0.5, seed=M + 7 * N + 13 * K), gpu, path)


@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
@pytest.mark.parametrize("cfg", list(range(12)))
@pytest.mark.parametrize("tA,tB", LAYOUTS)
def test_every_config_every_layout(gpu, path, cfg, tA, tB):
    _check(Problem(530, 390, 77, tA, tB, -1.25, 0.75, seed=cfg + ord(tA) * 3 + ord(tB)), gpu, path, cfg=cfg)


@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
@pytest.mark.parametrize("tA,tB", LAYOUTS)
@pytest.mark.parametrize("use_workspace", [True, False])
def test_prepacked_and_in_kernel_conversion(gpu, path, tA, tB, use_workspace):
    """Large enough for the pre-packed form (operands converted once into
    bf16 planes in the workspace), ragged in every dimension; without a
    workspace the same problem converts inside the GEMM."""
    _check(Problem(600, 530, 300, tA, tB, 1.5, 0.5, seed=ord(tA) + 3 * ord(tB)), gpu, path,
           use_workspace=use_workspace)


@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
@pytest.mark.parametrize("cfg", list(range(12)))
def test_prepacked_every_config(gpu, path, cfg):
    _check(Problem(777, 531, 203, "T", "N", -1.0, 0.25, seed=100 + cfg), gpu, path, cfg=cfg)


@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
@pytest.mark.parametrize("tA,tB", [("N", "N"), ("T", "N"), ("N", "T")])
@pytest.mark.parametrize("use_workspace", [True, False])
def test_eight_wave_tiles_bit_identical(gpu, path, tA, tB, use_workspace):
    """Configurations 8 and 9 run configuration 2's 128 x 128 tile over eight
    waves (64 x 32, 32 x 64) instead of four 64 x 64 ones, and 10 does the
    same for the direct-copy tile 7: every output still accumulates its k in
    the same order, so the bits are the same, on pre-packed planes and with
    the conversion in the GEMM (where 7 and 10 run as 2 and 8)."""
    outs = []
    for cfg in (2, 8, 9, 7, 10):
        C, _, _ = _check(Problem(600, 530, 300, tA, tB, 1.5, 0.5, seed=7 + ord(tA)), gpu, path, cfg=cfg,
                         use_workspace=use_workspace)
        outs.append(C)
    for C in outs[1:]:
        assert np.array_equal(outs[0], C)


@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
@pytest.mark.parametrize("use_workspace", [True, False])
def test_sixteen_wave_tile_bit_identical(gpu, path, use_workspace):
    """Configuration 11 runs configuration 6's 256 x 256 direct-copy tile over
    sixteen 64 x 64 waves: the same products in the same order per output,
    so the same bits (without the planes both run as configuration 1)."""
    outs = []
    for cfg in (6, 11):
        C, _, _ = _check(Problem(600, 530, 300, "N", "T", 1.5, 0.5, seed=23), gpu, path, cfg=cfg,
                         use_workspace=use_workspace)
        outs.append(C)
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
@pytest.mark.parametrize("cfg", [6, 7, 10, 11])
@pytest.mark.parametrize("K", [1, 64, 65, 128, 192, 1000])
def test_direct_copy_panel_counts(gpu, path, cfg, K):
    """The direct-copy tiles on pre-packed planes (M, N >= 512) at one, two,
    three and many 128-byte panels and ragged K, against the oracle."""
    _check(Problem(520, 530, K, "N", "N", 1.5, 0.5, seed=K + 13 * cfg), gpu, path, cfg=cfg)


@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
def test_prepacked_integer_bit_exact_and_layout_invariant(gpu, path):
    outs = []
    for tA, tB in LAYOUTS:
        C, Cref, _ = _check(Problem(520, 610, 250, tA, tB, 1.5, 0.5, seed=5, dist="integers"), gpu, path)
        assert np.array_equal(C, Cref)
        outs.append(C)


@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
def test_log_uniform_magnitudes(gpu, path):
    """|x| = 10^U(-3, 3) with random signs (the mixed-precision workload's second distribution)."""
    _check(Problem(384, 320, 640, "N", "N", 1.5, 0.5, seed=31, dist="log"), gpu, path)


@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
@pytest.mark.parametrize("tA,tB", LAYOUTS)
def test_integer_inputs_bit_exact(gpu, path, tA, tB):
    """Integers in [-8, 8] are exact in bf16 (lo = 0), so both paths are exact."""
    C, Cref, _ = _check(Problem(200, 300, 250, tA, tB, 1.5, 0.5, seed=77, dist="integers"), gpu, path)
    assert np.array_equal(C, Cref)


@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
def test_identity_operand(gpu, path):
    """A = I: C = B on bf16x3 up to the split residual (< 2^-16 |b|), = bf16(B) on BF16."""
    n = 96
    p = Problem(n, 70, n, "N", "N", 1.0, 0.0, seed=41)
    p.opA = np.eye(n, dtype=np.float32)
    p.A, p.lda = si.store(p.opA, "N")
    p.to_device(gpu)
    assert p.run(path) == 0
    C = p.result()
    hiB, loB = oracle.bf16_split(p.opB)
    expect = hiB + loB if path == "bf16x3" else hiB
    assert np.array_equal(C, expect)


@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
def test_beta_zero_nan_c_and_determinism(gpu, path):
    p = Problem(260, 270, 90, "T", "N", 1.0, 0.0, seed=51, c0_nan=True).to_device(gpu)
    outs = []
    for _ in range(2):
        p.reset_c()
        assert p.run(path) == 0
        outs.append(p.result())
    assert not np.isnan(outs[0]).any()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.slow
@pytest.mark.parametrize("dist", ["uniform", "log"])
@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
def test_full_size_8192_sampled(gpu, path, dist):
    """The mixed-precision workload: 8192^3, both input distributions; 4096
    sampled outputs against the oracle on the FP32 inputs."""
    p = Problem(8192, 8192, 8192, "N", "N", 1.0, 0.0, seed=3001, dist=dist).to_device(gpu)
    assert p.run(path) == 0
    C = p.result()
    I, J = si.sample_indices(8192, 8192, 4096, 98)
    cref, d = p.oracle_entries(I, J)
    err = oracle.normalized_error(C[I, J], cref, d)
    print(f"{path} {dist} 8192^3 sampled normalised error {err:.3e}")
    assert err <= TOL[path], err


@pytest.mark.parametrize("path", ["bf16", "fp16", "bf16x3"])
@pytest.mark.parametrize("M,N,K,tA,tB,splits", [
    (512, 512, 32, "N", "N", -1), (777, 531, 203, "T", "N", -1), (600, 1030, 1500, "N", "T", 3),
    (513, 700, 129, "T", "T", -1), (1024, 768, 4096, "N", "N", 5)])
def test_direct_copy_equals_staged_kernel_bitwise(gpu, path, M, N, K, tA, tB, splits):
    """Configuration 6 copies the pre-packed planes' panels straight into
    LDS (bf16x3: one plane per operand with hi and lo interleaved per 32 k,
    against configuration 1's conversion inside the GEMM); its MFMA sequence
    over k is configuration 1's, so the two results must agree bit for bit
    (ragged tiles, ragged K, split K ranges), and both must meet the path's
    bound against the oracle."""
    nat = _native()
    pid = {"bf16x3": 1, "bf16": 2, "fp16": 4}[path]
    outs = []
    for cfg in (1, 6):
        p = Problem(M, N, K, tA, tB, 1.5, 0.5, seed=M + N + K)
        assert nat.mg_force_config(pid, cfg) == 0
        if splits > 0:
            assert nat.mg_force_splits(pid, splits) == 0
        try:
            p.to_device(gpu)
            st = p.run(path)
            assert st == 0, nat.status_string(st)
            outs.append(p.result())
        finally:
            nat.mg_force_config(pid, -1)
            nat.mg_force_splits(pid, -1)
        assert p.padding_untouched()
    assert np.array_equal(outs[0], outs[1])
    Cref, D = p.oracle()
    assert oracle.normalized_error(outs[1], Cref, D) <= tolerance(path, K)
