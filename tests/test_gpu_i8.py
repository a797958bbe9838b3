"""GPU parity of the INT8 entry points against the integer oracle: every
result must be BIT-EXACT (exact int32 sums, alpha*sum + beta*C0 modulo 2^32)."""
import itertools

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

LAYOUTS = list(itertools.product("NT", "NT"))
I8 = 5   # MG_CONFIGS_I8


def _native():
    from paper_2305_18236_amd import _native
    return _native


class I8Problem:
    def __init__(self, M, N, K, tA="N", tB="N", alpha=1, beta=0, seed=0, lda=None, ldb=None, ldc=None,
                 lo=-128, hi=128):
        rng = np.random.default_rng(seed)
        self.M, self.N, self.K, self.tA, self.tB, self.alpha, self.beta = M, N, K, tA, tB, alpha, beta
        self.opA = rng.integers(lo, hi, (M, K)).astype(np.int8)
        self.opB = rng.integers(lo, hi, (K, N)).astype(np.int8)
        self.C0 = rng.integers(-2 ** 31, 2 ** 31, (M, N)).astype(np.int32)
        self.A, self.lda = self._store(self.opA, tA, lda)
        self.B, self.ldb = self._store(self.opB, tB, ldb)
        self.ldc = max(N, 1) if ldc is None else ldc
        buf = np.full((max(M, 1), max(self.ldc, 1)), -7, np.int32)
        buf[:M, :N] = self.C0
        self.Cbuf = buf

    @staticmethod
    def _store(op, t, ld):
        st = op if t == "N" else op.T
        r, c = st.shape
        ld = max(c, 1) if ld is None else ld
        buf = np.full((max(r, 1), ld), 99, np.int8)
        buf[:r, :c] = st
        return buf, ld

    def run(self, dev, cfg=None):
        nat = _native()
        dA = torch.from_numpy(self.A.reshape(-1).copy()).to(dev)
        dB = torch.from_numpy(self.B.reshape(-1).copy()).to(dev)
        self.dC = torch.from_numpy(self.Cbuf.reshape(-1).copy()).to(dev)
        need = nat.mg_gemm_i8_workspace_size(self.M, self.N, self.K)
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        if cfg is not None:
            assert nat.mg_force_config(I8, cfg) == 0
        try:
            st = nat.mg_gemm_i8(self.tA, self.tB, self.M, self.N, self.K, self.alpha, dA.data_ptr(), self.lda,
                                dB.data_ptr(), self.ldb, self.beta, self.dC.data_ptr(), self.ldc,
                                ws.data_ptr(), need, torch.cuda.current_stream().cuda_stream)
        finally:
            nat.mg_force_config(I8, -1)
        assert st == 0, nat.status_string(st)
        torch.cuda.synchronize()
        full = self.dC.cpu().numpy().reshape(max(self.M, 1), max(self.ldc, 1))
        assert np.all(full[:self.M, self.N:] == -7)
        return full[:self.M, :self.N]

    def oracle(self):
        return oracle.gemm_i8(self.tA, self.tB, self.M, self.N, self.K, self.alpha, self.A, self.lda,
                              self.B, self.ldb, self.beta, self.C0, self.N)


@pytest.mark.parametrize("tA,tB", LAYOUTS)
@pytest.mark.parametrize("M,N,K", [(256, 256, 256), (300, 517, 129), (1, 1, 1), (7, 9, 8), (33, 65, 31),
                                   (5, 300, 3), (130, 70, 1000)])
def test_bit_exact_ragged_all_layouts(gpu, tA, tB, M, N, K):
    p = I8Problem(M, N, K, tA, tB, alpha=3, beta=-2, seed=M + 7 * N + 13 * K)
    assert np.array_equal(p.run(gpu), p.oracle())


@pytest.mark.parametrize("cfg", [0, 1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("tA,tB", LAYOUTS)
def test_every_config_every_layout(gpu, cfg, tA, tB):
    p = I8Problem(530, 390, 300, tA, tB, alpha=-1, beta=1, seed=cfg + 3 * ord(tA) + ord(tB))
    assert np.array_equal(p.run(gpu, cfg=cfg), p.oracle())


@pytest.mark.parametrize("cfg", [3, 4, 5, 6, 7])
@pytest.mark.parametrize("K", [1, 128, 129, 256, 384, 1000])
def test_interleaved_pack_panel_counts(gpu, cfg, K):
    """The two-staging-set loop at every parity of the panel count (1, 2, 3
    and more panels, ragged K)."""
    p = I8Problem(300, 260, K, "N", "T", alpha=2, beta=-1, seed=K + cfg)
    assert np.array_equal(p.run(gpu, cfg=cfg), p.oracle())


def test_unaligned_leading_dimensions(gpu):
    """Leading dimensions that rule out 16-byte pack loads."""
    p = I8Problem(70, 45, 200, "N", "T", alpha=1, beta=1, seed=9, lda=203, ldb=201, ldc=47)
    assert np.array_equal(p.run(gpu), p.oracle())
    q = I8Problem(70, 45, 200, "T", "N", alpha=1, beta=0, seed=10, lda=73, ldb=51)
    assert np.array_equal(q.run(gpu), q.oracle())


def test_wraparound_of_alpha_and_beta(gpu):
    """Large alpha and beta: alpha*sum + beta*C0 wraps modulo 2^32 exactly as
    the oracle's definition says."""
    p = I8Problem(100, 90, 500, "N", "N", alpha=2 ** 30 - 3, beta=-(2 ** 30) + 11, seed=11)
    assert np.array_equal(p.run(gpu), p.oracle())


def test_extreme_values_longest_k(gpu):
    """All -128 at K = 131071: every sum is K * 16384 = 2^31 - 2^14."""
    p = I8Problem(64, 48, 131071, "N", "T", seed=12, lo=-128, hi=-127)
    C = p.run(gpu)
    assert np.all(C == 131071 * 16384)
    assert np.array_equal(C, p.oracle())


def test_too_long_k_rejected_on_host(gpu):
    nat = _native()
    assert nat.mg_gemm_i8("N", "N", 4, 4, 131072, 1, 0x1000, 131072, 0x1000, 4, 0, 0x1000, 4, None, 0,
                          None) == -102


def test_quick_returns(gpu):
    # alpha == 0: beta * C0 (wrapped); K == 0 likewise; beta == 1: untouched
    for alpha, K, beta in [(0, 50, 3), (5, 0, -2), (0, 10, 1), (0, 10, 0)]:
        p = I8Problem(40, 30, K, "N", "N", alpha=alpha, beta=beta, seed=13)
        assert np.array_equal(p.run(gpu), p.oracle())


def test_beta_zero_never_reads_c(gpu):
    p = I8Problem(60, 50, 70, "T", "T", alpha=7, beta=0, seed=14)
    p.Cbuf[:60, :50] = 12345     # would show up if read
    assert np.array_equal(p.run(gpu), p.oracle())


def test_packed_entry_points_match(gpu):
    """mg_i8_pack + mg_gemm_i8_packed give the same bits as mg_gemm_i8."""
    nat = _native()
    M, N, K = 300, 260, 700
    p = I8Problem(M, N, K, "T", "N", alpha=2, beta=1, seed=15)
    full = p.run(gpu)
    s = torch.cuda.current_stream().cuda_stream
    dA = torch.from_numpy(p.A.reshape(-1).copy()).to(gpu)
    dB = torch.from_numpy(p.B.reshape(-1).copy()).to(gpu)
    qA = torch.empty(nat.mg_i8_packed_size(M, K), dtype=torch.int8, device=gpu)
    qB = torch.empty(nat.mg_i8_packed_size(N, K), dtype=torch.int8, device=gpu)
    assert nat.mg_i8_pack("T", M, K, dA.data_ptr(), p.lda, qA.data_ptr(), s) == 0
    # op(B)^T is N x K; B is stored K x N here, i.e. transposed relative to it
    assert nat.mg_i8_pack("T", N, K, dB.data_ptr(), p.ldb, qB.data_ptr(), s) == 0
    C = torch.from_numpy(p.C0.copy()).to(gpu)
    assert nat.mg_gemm_i8_packed(M, N, K, 2, qA.data_ptr(), qB.data_ptr(), 1, C.data_ptr(), N, s) == 0
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy(), full)
    # the packed rows hold op(A) row-major, k-contiguous, zero-padded
    Kp = (K + 127) // 128 * 128
    q = qA.cpu().numpy().reshape(-1, Kp)
    assert np.array_equal(q[:M, :K], p.opA) and not q[M:].any() and not q[:, K:].any()


def test_torch_wrapper(gpu):
    from paper_2305_18236_amd import gemm_i8
    rng = np.random.default_rng(16)
    a = rng.integers(-128, 128, (200, 150)).astype(np.int8)
    b = rng.integers(-128, 128, (100, 150)).astype(np.int8)       # used transposed
    A = torch.from_numpy(a).to(gpu)
    B = torch.from_numpy(b).to(gpu).t()
    C = gemm_i8(A, B)
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy().astype(np.int64), a.astype(np.int64) @ b.T.astype(np.int64))


@pytest.mark.slow
def test_full_size_8192_sampled(gpu):
    """8192^3, the benchmark's launch; a sample of rows checked exactly."""
    M = N = K = 8192
    rng = np.random.default_rng(17)
    a = rng.integers(-128, 128, (M, K)).astype(np.int8)
    b = rng.integers(-128, 128, (K, N)).astype(np.int8)
    from paper_2305_18236_amd import gemm_i8
    C = gemm_i8(torch.from_numpy(a).to(gpu), torch.from_numpy(b).to(gpu))
    torch.cuda.synchronize()
    rows = rng.choice(M, 24, replace=False)
    Cs = C.cpu().numpy()[rows]
    ref = oracle.gemm_i8("N", "N", len(rows), N, K, 1, a[rows], K, b, N)
    assert np.array_equal(Cs, ref)
