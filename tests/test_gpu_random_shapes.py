"""Seeded random sweep over the GEMM boundary: shapes, layouts, leading
dimensions, base pointers that are 4- but not 16-byte aligned, alpha/beta and
forced K splits, on every floating path and on INT8, each case against the
oracle (INT8 bit for bit).  Catches interactions the targeted tests do not
enumerate (e.g. an unaligned operand on a split launch)."""
import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si
from helpers import PATH_ID, TOL, tolerance

pytestmark = pytest.mark.gpu

CASES = 40


def _native():
    from paper_2305_18236_amd import _native
    return _native


def _store_at(logical, trans, ld, offset, dtype):
    """The stored matrix in a flat buffer that starts `offset` elements into
    the allocation (so the operand's base pointer is only element-aligned)."""
    st = logical if trans == "N" else logical.T
    r, c = st.shape
    buf = np.zeros(offset + max(r, 1) * ld, dtype=dtype)
    view = buf[offset:offset + r * ld].reshape(r, ld) if r else buf[offset:offset]
    if r:
        view[:, :c] = st
    return buf


def _case(rng):
    M, N, K = (int(x) for x in rng.integers(1, 400, 3))
    tA, tB = rng.choice(["N", "T"]), rng.choice(["N", "T"])
    pad = [int(x) for x in rng.integers(0, 6, 3)]
    off = [int(x) for x in rng.integers(0, 4, 3)]
    alpha = float(rng.choice([1.0, -1.5, 0.75]))
    beta = float(rng.choice([0.0, 0.5, 1.0]))
    splits = int(rng.choice([-1, -1, 1, 2, 3]))
    return M, N, K, str(tA), str(tB), pad, off, alpha, beta, splits


@pytest.mark.parametrize("path", ["fp32", "bf16x3", "bf16", "fp16"])
def test_random_float_cases(gpu, path):
    nat = _native()
    pid = PATH_ID[path]
    rng = np.random.default_rng(900 + pid)
    s = torch.cuda.current_stream().cuda_stream
    for case in range(CASES):
        M, N, K, tA, tB, pad, off, alpha, beta, splits = _case(rng)
        opA = si.uniform((M, K), 1000 * pid + 3 * case)
        opB = si.uniform((K, N), 1000 * pid + 3 * case + 1)
        C0 = si.uniform((M, N), 1000 * pid + 3 * case + 2)
        lda = (K if tA == "N" else M) + pad[0]
        ldb = (N if tB == "N" else K) + pad[1]
        ldc = N + pad[2]
        A = torch.from_numpy(_store_at(opA, tA, lda, off[0], np.float32)).to(gpu)
        B = torch.from_numpy(_store_at(opB, tB, ldb, off[1], np.float32)).to(gpu)
        Cb = np.full(off[2] + M * ldc, -7.0, np.float32)
        Cb[off[2]:].reshape(M, ldc)[:, :N] = C0
        C = torch.from_numpy(Cb).to(gpu)
        assert nat.mg_force_splits(pid, splits) == 0
        try:
            need = nat.mg_gemm_workspace_size(pid, tA, tB, M, N, K)
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=gpu)
            st = nat.mg_gemm(pid, tA, tB, M, N, K, alpha, A.data_ptr() + 4 * off[0], lda,
                             B.data_ptr() + 4 * off[1], ldb, beta, C.data_ptr() + 4 * off[2], ldc,
                             ws.data_ptr(), need, s)
        finally:
            nat.mg_force_splits(pid, -1)
        assert st == 0, (case, nat.status_string(st))
        torch.cuda.synchronize()
        out = C.cpu().numpy()
        assert np.all(out[:off[2]] == -7.0)
        got = out[off[2]:].reshape(M, ldc)
        assert np.all(got[:, N:] == -7.0), case
        Cref, D = oracle.gemm_logical(opA, opB, alpha, beta, C0)
        err = oracle.normalized_error(got[:, :N].astype(np.float64), Cref, D)
        assert err <= tolerance(path, K), (case, M, N, K, tA, tB, pad, off, alpha, beta, splits, err)


def test_random_int8_cases(gpu):
    nat = _native()
    rng = np.random.default_rng(950)
    s = torch.cuda.current_stream().cuda_stream
    for case in range(CASES):
        M, N, K, tA, tB, pad, off, _, _, _ = _case(rng)
        alpha = int(rng.integers(-5, 6))
        beta = int(rng.choice([0, 1, -3]))
        opA = rng.integers(-128, 128, (M, K)).astype(np.int8)
        opB = rng.integers(-128, 128, (K, N)).astype(np.int8)
        C0 = rng.integers(-2 ** 31, 2 ** 31, (M, N)).astype(np.int32)
        lda = (K if tA == "N" else M) + pad[0]
        ldb = (N if tB == "N" else K) + pad[1]
        ldc = N + pad[2]
        A = torch.from_numpy(_store_at(opA, tA, lda, off[0], np.int8)).to(gpu)
        B = torch.from_numpy(_store_at(opB, tB, ldb, off[1], np.int8)).to(gpu)
        Cb = np.full(off[2] + M * ldc, -7, np.int32)
        Cb[off[2]:].reshape(M, ldc)[:, :N] = C0
        C = torch.from_numpy(Cb).to(gpu)
        need = nat.mg_gemm_i8_workspace_size(M, N, K)
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=gpu)
        st = nat.mg_gemm_i8(tA, tB, M, N, K, alpha, A.data_ptr() + off[0], lda, B.data_ptr() + off[1], ldb, beta,
                            C.data_ptr() + 4 * off[2], ldc, ws.data_ptr(), need, s)
        assert st == 0, (case, nat.status_string(st))
        torch.cuda.synchronize()
        out = C.cpu().numpy()
        got = out[off[2]:].reshape(M, ldc)
        assert np.all(got[:, N:] == -7), case
        As = _store_at(opA, tA, lda, 0, np.int8)
        Bs = _store_at(opB, tB, ldb, 0, np.int8)
        ref = oracle.gemm_i8(tA, tB, M, N, K, alpha, As, lda, Bs, ldb, beta, C0, N)
        assert np.array_equal(got[:, :N], ref), (case, M, N, K, tA, tB, pad, off)
