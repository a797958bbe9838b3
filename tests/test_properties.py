"""Property tests (Hypothesis) on the CPU: host-side marshalling, argument
validation and the split-K plan of the library, and algebraic properties of
the oracle that the GEMM statement of Section 3 fixes.  No device call is
made: every library call here either returns before touching the device or
only computes a plan."""
import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, assume, given, settings
from hypothesis import strategies as st

import oracle
import seeded_inputs as si

SETTINGS = settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])


@pytest.fixture(scope="module")
def native():
    from paper_2305_18236_amd import _native
    _native.lib()
    return _native


# ---- operand marshalling (paper_2305_18236_amd.operand_layout)

@SETTINGS
@given(rows=st.integers(1, 12), cols=st.integers(1, 12), pad=st.integers(0, 5), transposed=st.booleans())
def test_operand_layout_reconstructs_the_logical_matrix(rows, cols, pad, transposed):
    """Whatever view the caller passes (row-major, or the .t() of a row-major
    buffer, with padded rows), (trans, ld) read from the strides address
    exactly the logical matrix in the stored buffer."""
    from paper_2305_18236_amd import operand_layout
    if not transposed:
        base = torch.arange(rows * (cols + pad), dtype=torch.float32).reshape(rows, cols + pad)
        X = base[:, :cols]
    else:
        base = torch.arange(cols * (rows + pad), dtype=torch.float32).reshape(cols, rows + pad)
        X = base[:, :rows].t()
    t, ld = operand_layout(X)
    flat = base.reshape(-1).numpy()
    for r in range(rows):
        for c in range(cols):
            off = r * ld + c if t == "N" else c * ld + r
            assert flat[off] == X[r, c].item()


# ---- argument validation (BLAS xerbla order, first invalid argument wins)

FAKE = 0x1000


def expected_code(tA, tB, M, N, K, A, lda, B, ldb, C, ldc):
    if tA not in "NnTtCc":
        return -1
    if tB not in "NnTtCc":
        return -2
    if M < 0:
        return -3
    if N < 0:
        return -4
    if K < 0:
        return -5
    a_rows, a_cols = (M, K) if tA in "Nn" else (K, M)
    b_rows, b_cols = (K, N) if tB in "Nn" else (N, K)
    if A is None and M * K > 0:
        return -7
    if lda < max(1, a_cols):
        return -8
    if B is None and K * N > 0:
        return -9
    if ldb < max(1, b_cols):
        return -10
    if C is None and M * N > 0:
        return -12
    if ldc < max(1, N):
        return -13
    return 0


@SETTINGS
@given(tA=st.sampled_from("NTnXC"), tB=st.sampled_from("NTtQc"), M=st.integers(-2, 9), N=st.integers(-2, 9),
       K=st.integers(-2, 9), lda=st.integers(-1, 12), ldb=st.integers(-1, 12), ldc=st.integers(-1, 12),
       nullA=st.booleans(), nullB=st.booleans(), nullC=st.booleans())
def test_invalid_arguments_return_the_first_bad_argument(native, tA, tB, M, N, K, lda, ldb, ldc,
                                                         nullA, nullB, nullC):
    A = None if nullA else FAKE
    B = None if nullB else FAKE
    C = None if nullC else FAKE
    code = expected_code(tA, tB, M, N, K, A, lda, B, ldb, C, ldc)
    assume(code != 0)        # valid arguments would reach the device
    got = native.mg_sgemm(tA, tB, M, N, K, 1.0, A, lda, B, ldb, 0.0, C, ldc, None)
    assert got == code


# ---- split-K plan (host logic)

@SETTINGS
@given(M=st.integers(1, 20000), N=st.integers(1, 20000), K=st.integers(1, 1 << 16), path=st.sampled_from([0, 1, 2, 4]))
def test_split_plan_bounds(native, M, N, K, path):
    s = native.mg_split_count(path, M, N, K)
    assert 1 <= s <= 16
    if K < 256:
        assert s == 1                  # ranges are whole 128-deep grains, at least two
    if s > 1:
        assert K // s >= 128           # every range holds at least one grain


@SETTINGS
@given(M=st.integers(1, 5000), N=st.integers(1, 5000), K=st.integers(1, 5000))
def test_fp8_and_int8_never_split_and_configs_are_valid(native, M, N, K):
    assert native.mg_split_count(3, M, N, K) == 1
    for path in (0, 1, 2, 3, 4):
        cfg = native.mg_tuned_config(path, M, N, K)
        assert 0 <= cfg < native.mg_num_configs(path)


# ---- the GEMM statement (oracle)

small = st.integers(1, 7)


@SETTINGS
@given(M=small, N=small, K=st.integers(0, 7), tA=st.sampled_from("NT"), tB=st.sampled_from("NT"),
       alpha=st.sampled_from([1.0, -2.0, 0.5, 3.0]), beta=st.sampled_from([0.0, 1.0, -0.5]), seed=st.integers(0, 999))
def test_oracle_equals_exact_integer_arithmetic(M, N, K, tA, tB, alpha, beta, seed):
    """On small integers every FP64 step is exact, so the oracle must equal
    the definition computed in exact integer / dyadic arithmetic."""
    a = si.integers((M, K), seed)
    b = si.integers((K, N), seed + 1)
    c0 = si.integers((M, N), seed + 2)
    A, lda = si.store(a, tA)
    B, ldb = si.store(b, tB)
    C, D = oracle.gemm(tA, tB, M, N, K, alpha, A, lda, B, ldb, beta, c0, N)
    exact = alpha * (a.astype(np.int64) @ b.astype(np.int64)).astype(np.float64) + beta * c0.astype(np.float64)
    dexact = abs(alpha) * (np.abs(a).astype(np.int64) @ np.abs(b).astype(np.int64)) + abs(beta) * np.abs(c0)
    assert np.array_equal(C, exact)
    assert np.array_equal(D, dexact)


@SETTINGS
@given(M=small, N=small, K=small, seed=st.integers(0, 999))
def test_oracle_is_linear_and_transpose_consistent(M, N, K, seed):
    """(A B)^T = B^T A^T, and scaling A by a power of two scales C by it,
    bit for bit (FP64 sums of FP32 products)."""
    a = si.uniform((M, K), seed)
    b = si.uniform((K, N), seed + 1)
    C, _ = oracle.gemm_logical(a, b)
    Ct, _ = oracle.gemm_logical(b.T.copy(), a.T.copy())
    assert np.array_equal(C, Ct.T)
    C4, _ = oracle.gemm_logical((4 * a).astype(np.float32), b)
    assert np.array_equal(C4, 4 * C)
