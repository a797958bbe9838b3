"""GPU parity of the FP8 (E4M3, per-128x128-tile power-of-two scales) path.

  * pack: the quantised codes and the tile scales are bit-exact against the
    oracle's quantiser (both take the rounding decision on the exact value
    x / s, s a power of two);
  * GEMM on packed operands: against the oracle's FP64 product of the exactly
    dequantised operands.  Every E4M3 x E4M3 product is exact on the matrix
    core, but the scaled FP8 MFMA of gfx950 sums the 64 products of one step
    by aligning them to the largest, dropping bits below about 2^-17.8 of it
    (measured: a lone product is exact; a product 2^-18 the size of a
    448 x 448 product beside it is lost).  Each of a step's 64 products can
    lose that much, so a step's error is at most 64 * 2^-17.8 = 2^-11.8
    (2.8e-4) of its sum of |products|, and so is the normalised error.
    Measured: 1.3e-5 (uniform, K = 64), 7.4e-5 (log-uniform), 2.7e-4 (values
    spread over the whole E4M3 range).  Bound used: 3e-4, far below the
    >= 1e-2 a wrong tile scale or a dropped K step would cause;
  * end to end from FP32: <= 6e-2 against the oracle on the FP32 inputs, and
    bit-exact on integer inputs (which quantise exactly).
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
EMU_TOL = 3e-4


def _native():
    from paper_2305_18236_amd import _native
    return _native


def _pack_on_gpu(dev, logical, trans, ld=None):
    """Pack op(X) = logical (R x K) stored per `trans`; returns (q[R,K], scales float, raw q, raw s)."""
    nat = _native()
    R, K = logical.shape
    buf, ldx = si.store(logical, trans, ld)
    dX = torch.from_numpy(buf if buf.size else np.zeros(1, np.float32)).to(dev)
    qb, sb = nat.mg_fp8_packed_size(R, K)
    q = torch.full((qb,), 0xAB, dtype=torch.uint8, device=dev)
    s = torch.full((sb,), 0xCD, dtype=torch.uint8, device=dev)
    st = nat.mg_fp8_pack(trans, R, K, dX.data_ptr(), ldx, q.data_ptr(), s.data_ptr(),
                         torch.cuda.current_stream().cuda_stream)
    assert st == 0, nat.status_string(st)
    torch.cuda.synchronize()
    Rp = -(-max(R, 1) // 256) * 256
    Kp = -(-max(K, 1) // 128) * 128
    qh = q.cpu().numpy().reshape(Rp, Kp)
    sh = s.cpu().numpy().reshape(Rp // 128, Kp // 128)
    return qh, sh, q, s


def _e8m0(b):
    return np.exp2(b.astype(np.float64) - 127.0)


@pytest.mark.parametrize("trans", ["N", "T"])
@pytest.mark.parametrize("R,K,dist", [(300, 260, "uniform"), (128, 128, "log"), (1, 1, "uniform"),
                                      (257, 385, "log"), (64, 1000, "integers")])
def test_pack_bit_exact(gpu, trans, R, K, dist):
    gen = {"uniform": si.uniform, "log": si.log_uniform_signed, "integers": si.integers}[dist]
    X = gen((R, K), R * 1000 + K)
    if R >= 128 and K >= 256:
        X[:128, 128:256] *= 1000.0    # one tile with a different range
    qh, sh, _, _ = _pack_on_gpu(gpu, X, trans)
    qo, so = oracle.fp8_quantize(X)
    assert np.array_equal(qh[:R, :K], qo)
    assert np.array_equal(_e8m0(sh[: so.shape[0], : so.shape[1]]), so.astype(np.float64))
    # padding rows/columns hold zero codes; padding tiles carry scale 1
    assert not qh[R:, :].any() and not qh[:, K:].any()
    assert np.all(sh[so.shape[0]:, :] == 127) and np.all(sh[:, so.shape[1]:] == 127)


def test_pack_zero_tile_and_padded_ld(gpu):
    X = si.uniform((200, 300), 5)
    X[128:, :128] = 0.0
    qh, sh, _, _ = _pack_on_gpu(gpu, X, "T", ld=211)
    qo, so = oracle.fp8_quantize(X)
    assert np.array_equal(qh[:200, :300], qo)
    assert sh[1, 0] == 127 and so[1, 0] == 1.0


def _fp8_reference(p):
    """Oracle on the exactly dequantised operands, plus the FP32-input oracle."""
    qa, sa = oracle.fp8_quantize(p.opA)
    qb, sb = oracle.fp8_quantize(p.opB.T)
    dA = oracle.fp8_dequantize(qa, sa)
    dBt = oracle.fp8_dequantize(qb, sb)
    Cemu, _ = oracle.gemm_logical(dA, dBt.T, p.alpha, p.beta, p.C0)
    return Cemu


def _check(p, dev, cfg=None):
    nat = _native()
    if cfg is not None:
        assert nat.mg_force_config(3, cfg) == 0
    try:
        p.to_device(dev)
        st = p.run("fp8")
        assert st == 0, nat.status_string(st)
        C = p.result()
    finally:
        nat.mg_force_config(3, -1)
    Cref, D = p.oracle()
    emu = oracle.normalized_error(C, _fp8_reference(p), D)
    err = oracle.normalized_error(C, Cref, D)
    assert emu <= EMU_TOL, (p.M, p.N, p.K, p.tA, p.tB, "emulation", emu)
    assert err <= tolerance("fp8", p.K), (p.M, p.N, p.K, p.tA, p.tB, err)
    assert p.padding_untouched()
    return C, Cref, err


def test_256_cube(gpu):
    _check(Problem(256, 256, 256, "N", "N", 1.0, 0.0, seed=1000), gpu)


@pytest.mark.parametrize("tA,tB", LAYOUTS)
@pytest.mark.parametrize("M,N,K", [(300, 517, 129), (1, 1, 1), (7, 9, 8), (33, 65, 31), (130, 260, 390)])
def test_ragged_shapes_all_layouts(gpu, tA, tB, M, N, K):
    _check(Problem(M, N, K, tA, tB, 1.5, 0.5, seed=M + 7 * N + 13 * K), gpu)


@pytest.mark.parametrize("cfg", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11])
@pytest.mark.parametrize("tA,tB", LAYOUTS)
def test_every_config_every_layout(gpu, cfg, tA, tB):
    _check(Problem(530, 390, 300, tA, tB, -1.25, 0.75, seed=cfg + ord(tA) * 3 + ord(tB)), gpu, cfg=cfg)


@pytest.mark.parametrize("cfg", [5, 6, 7, 8, 9, 10, 11])
@pytest.mark.parametrize("K", [1, 128, 129, 256, 384, 1000])
def test_interleaved_pack_panel_counts(gpu, cfg, K):
    """The two-buffer loops (interleaved staging, direct copies) and their
    one-panel-ahead scale bytes at every parity of the panel count."""
    _check(Problem(300, 260, K, "N", "T", 1.5, 0.5, seed=K + 11 * cfg), gpu, cfg=cfg)


@pytest.mark.parametrize("tA,tB", [("N", "N"), ("T", "T")])
def test_eight_wave_direct_tile_bit_identical(gpu, tA, tB):
    """Configuration 10 runs configuration 8's 128 x 128 direct-copy tile over
    eight 64 x 32 waves: each output accumulates the same products in the
    same order, so the bits match (ragged M, N and K)."""
    p = Problem(530, 390, 700, tA, tB, -1.25, 0.75, seed=17 + ord(tA))
    C8 = _check(p, gpu, cfg=8)[0]
    C10 = _check(p, gpu, cfg=10)[0]
    assert np.array_equal(C8, C10)
    # and configuration 11 runs 7's 256 x 256 tile over sixteen 64 x 64 waves
    assert np.array_equal(_check(p, gpu, cfg=7)[0], _check(p, gpu, cfg=11)[0])


def test_log_uniform_magnitudes(gpu):
    _check(Problem(384, 320, 640, "N", "N", 1.5, 0.5, seed=31, dist="log"), gpu)


@pytest.mark.parametrize("tA,tB", LAYOUTS)
def test_integer_inputs_bit_exact(gpu, tA, tB):
    C, Cref, _ = _check(Problem(200, 300, 250, tA, tB, 1.5, 0.5, seed=77, dist="integers"), gpu)
    assert np.array_equal(C, Cref)


def test_packed_gemm_entry_point(gpu):
    """Pack once, then the GEMM alone (the timing form) on the packed operands."""
    nat = _native()
    M, N, K = 300, 200, 260
    opA = si.uniform((M, K), 61)
    opB = si.uniform((K, N), 62)
    _, _, qA, sA = _pack_on_gpu(gpu, opA, "N")
    _, _, qB, sB = _pack_on_gpu(gpu, opB.T.copy(), "N")
    C = torch.zeros((M, N), dtype=torch.float32, device=gpu)
    st = nat.mg_gemm_fp8_packed(M, N, K, 1.0, qA.data_ptr(), sA.data_ptr(), qB.data_ptr(), sB.data_ptr(),
                                0.0, C.data_ptr(), N, torch.cuda.current_stream().cuda_stream)
    assert st == 0, nat.status_string(st)
    torch.cuda.synchronize()
    qa, sa = oracle.fp8_quantize(opA)
    qb, sb = oracle.fp8_quantize(opB.T)
    Cemu, D = oracle.gemm_logical(oracle.fp8_dequantize(qa, sa), oracle.fp8_dequantize(qb, sb).T)
    assert oracle.normalized_error(C.cpu().numpy(), Cemu, D) <= EMU_TOL


def test_workspace_too_small_rejected(gpu):
    nat = _native()
    p = Problem(64, 64, 64, seed=3).to_device(gpu)
    need = nat.mg_gemm_workspace_size(3, "N", "N", 64, 64, 64)
    assert need > 0
    ws = torch.empty(need - 1, dtype=torch.uint8, device=gpu)
    st = nat.mg_gemm(3, "N", "N", 64, 64, 64, 1.0, p.dA.data_ptr(), 64, p.dB.data_ptr(), 64, 0.0,
                     p.dC.data_ptr(), 64, ws.data_ptr(), need - 1, torch.cuda.current_stream().cuda_stream)
    assert st == -100
    st = nat.mg_gemm(3, "N", "N", 64, 64, 64, 1.0, p.dA.data_ptr(), 64, p.dB.data_ptr(), 64, 0.0,
                     p.dC.data_ptr(), 64, None, 0, torch.cuda.current_stream().cuda_stream)
    assert st == -100


@pytest.mark.slow
@pytest.mark.parametrize("dist", ["uniform", "log"])
def test_full_size_8192_sampled(gpu, dist):
    p = Problem(8192, 8192, 8192, "N", "N", 1.0, 0.0, seed=3001, dist=dist).to_device(gpu)
    assert p.run("fp8") == 0
    C = p.result()
    I, J = si.sample_indices(8192, 8192, 4096, 98)
    cref, d = p.oracle_entries(I, J)
    err = oracle.normalized_error(C[I, J], cref, d)
    print(f"fp8 {dist} 8192^3 sampled normalised error {err:.3e}")
    assert err <= TOL["fp8"], err
