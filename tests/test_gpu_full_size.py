"""Full-size sampled parity: every shape of the FP32 sweep workload in all four
layouts, and the 8192^3 mixed-precision and integer workloads in the layouts
their own files do not cover, each checked against the FP64 oracle on sampled
outputs (corners included), in the launch configuration the benchmark times.

Bars: the normalised error max|C - C_ref| / (|alpha||A||B| + |beta||C0|)
within the path's tolerance (FP32 and bf16x3 1e-5, BF16 1e-2, FP16 2e-3,
FP8 6e-2); INT8 bit-exact.  The sums run over K >= 256 sign-random terms, so
the statistical bars of the short-K cases do not apply.
"""
import functools
import itertools

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from helpers import Problem, TOL

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

LAYOUTS = ["".join(t) for t in itertools.product("NT", "NT")]
SAMPLES = 2048

# The FP32 sweep workload: alpha 1.5, beta 0.5, C0 ~ U[-1, 1]; the 8192^3 cube is
# in test_gpu_sgemm.py.
SWEEP = [(1024, 1024, 1024), (2048, 2048, 2048), (4096, 4096, 4096),
         (8192, 8192, 256), (256, 8192, 8192), (16384, 1024, 4096)]


@functools.lru_cache(maxsize=1)
def _operands(M, N, K, dist, seed):
    gen = {"uniform": si.uniform, "log": si.log_uniform_signed}[dist]
    return gen((M, K), seed * 10), gen((K, N), seed * 10 + 1), si.uniform((M, N), seed * 10 + 2)


def _sampled_error(p, gpu, path, seed):
    p.to_device(gpu)
    st = p.run(path)
    assert st == 0, st
    C = p.result()
    assert np.isfinite(C).all()
    I, J = si.sample_indices(p.M, p.N, SAMPLES, seed)
    cref, d = p.oracle_entries(I, J)
    return oracle.normalized_error(C[I, J], cref, d), C


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("M,N,K", SWEEP)
def test_fp32_sweep_shapes_all_layouts(gpu, M, N, K, layout):
    opA, opB, C0 = _operands(M, N, K, "uniform", 2001)
    p = Problem.from_arrays(opA, opB, C0, 1.5, 0.5, layout[0], layout[1])
    err, _ = _sampled_error(p, gpu, "fp32", 211)
    print(f"fp32 {M}x{N}x{K} {layout} sampled normalised error {err:.3e}")
    assert err <= TOL["fp32"], err


@pytest.mark.parametrize("M,N,K", SWEEP)
def test_bf16x3_sweep_shapes(gpu, M, N, K):
    """The sweep's bf16x3 row (NN), which the benchmark reports beside FP32."""
    opA, opB, C0 = _operands(M, N, K, "uniform", 2001)
    p = Problem.from_arrays(opA, opB, C0, 1.5, 0.5, "N", "N")
    err, _ = _sampled_error(p, gpu, "bf16x3", 212)
    print(f"bf16x3 {M}x{N}x{K} NN sampled normalised error {err:.3e}")
    assert err <= TOL["bf16x3"], err


@pytest.mark.parametrize("dist", ["uniform", "log"])
@pytest.mark.parametrize("layout", ["NT", "TN", "TT"])
@pytest.mark.parametrize("path", ["bf16x3", "bf16", "fp8", "fp16"])
def test_mixed_precision_8192_other_layouts(gpu, path, layout, dist):
    """The mixed-precision workload (alpha 1, beta 0) in the layouts beside NN
    (NN: test_gpu_bf16.py, test_gpu_fp8.py, test_gpu_fp16.py).  Log-uniform
    magnitudes in [1e-3, 1e3] stay inside binary16's normal range, so the FP16
    bar applies to both distributions."""
    opA, opB, _ = _operands(8192, 8192, 8192, dist, 3001)
    p = Problem.from_arrays(opA, opB, None, 1.0, 0.0, layout[0], layout[1])
    err, _ = _sampled_error(p, gpu, path, 213)
    print(f"{path} {dist} 8192^3 {layout} sampled normalised error {err:.3e}")
    assert err <= TOL[path], err


@pytest.mark.parametrize("layout", LAYOUTS)
def test_int8_8192_sampled_bit_exact(gpu, layout):
    """INT8 at 8192^3 in every layout, alpha 3, beta -2: sampled outputs equal
    the exact integer oracle (mod 2^32) bit for bit."""
    import torch
    from paper_2305_18236_amd import gemm_i8
    n = 8192
    rng = np.random.default_rng(si.seed_for(3, "A"))
    a = rng.integers(-128, 128, (n, n), dtype=np.int8)
    b = rng.integers(-128, 128, (n, n), dtype=np.int8)
    c0 = rng.integers(-2 ** 31, 2 ** 31, (n, n), dtype=np.int64).astype(np.int32)
    dA = torch.from_numpy(a).to(gpu)
    dB = torch.from_numpy(b).to(gpu)
    A = dA if layout[0] == "N" else dA.t().contiguous().t()
    B = dB if layout[1] == "N" else dB.t().contiguous().t()
    C = torch.from_numpy(c0).to(gpu)
    gemm_i8(A, B, C, alpha=3, beta=-2)
    torch.cuda.synchronize()
    out = C.cpu().numpy()
    I, J = si.sample_indices(n, n, SAMPLES, 214)
    # the integer oracle, one sampled output at a time (a 1 x K row of A by a
    # K x 1 column of B)
    want = np.array([oracle.gemm_i8("N", "N", 1, 1, n, 3, a[i], n, np.ascontiguousarray(b[:, j]), 1, -2,
                                    c0[i, j].reshape(1, 1))[0, 0] for i, j in zip(I, J)], dtype=np.int32)
    assert np.array_equal(out[I, J], want)
