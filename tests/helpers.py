"""Shared helpers of the GPU parity tests: stage seeded host operands on the
device in a given stored layout, call the library through its C ABI, and score
the result against the FP64 oracle."""
from __future__ import annotations

import numpy as np

import oracle
import seeded_inputs as si

TOL = {"fp32": 1e-5, "bf16x3": 1e-5, "bf16": 1e-2, "fp8": 6e-2, "fp16": 2e-3}

# bf16x3 leaves a per-product error of at most about 3 * 2^-16 |a||b| (the
# dropped lo*lo term and the two split residuals, each <= 2^-16).  The 1e-5
# bar is statistical: it needs enough sign-random terms to average out, so
# below K = 32 the worst-case bound applies instead.
BF16X3_WORST = 5e-5
# FP8: each factor is rounded to 3 mantissa bits (relative error <= 2^-4), so
# one product can be off by (2*2^-4 + 2^-8) |a||b|; the 6e-2 bar needs sums
# of enough sign-random terms, and below K = 32 the worst case applies.
FP8_WORST = 0.13


def tolerance(path: str, K: int) -> float:
    if path == "bf16x3" and K < 32:
        return BF16X3_WORST
    if path == "fp8" and K < 32:
        return FP8_WORST
    return TOL[path]


PATH_ID = {"fp32": 0, "bf16x3": 1, "bf16": 2, "fp8": 3, "fp16": 4}


def device_buffer(host_1d: np.ndarray, torch_device):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(host_1d, dtype=np.float32))
    return t.to(torch_device)


class Problem:
    """One GEMM instance: logical operands, their stored layouts and the oracle result."""

    def __init__(self, M, N, K, tA="N", tB="N", alpha=1.0, beta=0.0, seed=0, dist="uniform",
                 lda=None, ldb=None, ldc=None, c0_nan=False):
        self.M, self.N, self.K = M, N, K
        self.tA, self.tB = tA, tB
        self.alpha, self.beta = alpha, beta
        gen = {"uniform": si.uniform, "integers": si.integers, "log": si.log_uniform_signed}[dist]
        self.opA = gen((M, K), seed * 10 + 0)
        self.opB = gen((K, N), seed * 10 + 1)
        if c0_nan:
            self.C0 = np.full((M, N), np.nan, np.float32)
        else:
            self.C0 = gen((M, N), seed * 10 + 2)
        self.A, self.lda = si.store(self.opA, tA, lda)
        self.B, self.ldb = si.store(self.opB, tB, ldb)
        self.ldc = max(N, 1) if ldc is None else ldc
        Cbuf = np.full((max(M, 1), max(self.ldc, 1)), -7.0, np.float32)
        Cbuf[:M, :N] = self.C0
        self.Cbuf = Cbuf.reshape(-1)

    @classmethod
    def from_arrays(cls, opA, opB, C0=None, alpha=1.0, beta=0.0, tA="N", tB="N"):
        """A problem on given logical operands (C0 defaults to zeros)."""
        p = cls.__new__(cls)
        p.M, p.K = opA.shape
        p.N = opB.shape[1]
        p.tA, p.tB, p.alpha, p.beta = tA, tB, alpha, beta
        p.opA, p.opB = opA, opB
        p.C0 = np.zeros((p.M, p.N), np.float32) if C0 is None else C0
        p.A, p.lda = si.store(opA, tA)
        p.B, p.ldb = si.store(opB, tB)
        p.ldc = max(p.N, 1)
        p.Cbuf = np.ascontiguousarray(p.C0, np.float32).reshape(-1)
        return p

    def oracle(self, threads=None):
        return oracle.gemm(self.tA, self.tB, self.M, self.N, self.K, self.alpha, self.A, self.lda,
                           self.B, self.ldb, self.beta, self.C0, max(self.N, 1), threads=threads)

    def oracle_entries(self, I, J, threads=None):
        return oracle.gemm_entries(self.tA, self.tB, self.K, self.alpha, self.A, self.lda, self.B,
                                   self.ldb, self.beta, self.C0, self.N, I, J, threads=threads)

    def to_device(self, dev):
        self.dA = device_buffer(self.A if self.A.size else np.zeros(1, np.float32), dev)
        self.dB = device_buffer(self.B if self.B.size else np.zeros(1, np.float32), dev)
        self.dC = device_buffer(self.Cbuf, dev)
        return self

    def reset_c(self):
        import torch
        self.dC.copy_(torch.from_numpy(self.Cbuf))

    def run(self, path="fp32", workspace=None, stream=None, use_workspace=True):
        """Call mg_gemm through the C ABI; returns the status code.

        use_workspace=False passes no workspace (the BF16 paths then convert
        inside the GEMM instead of pre-packing)."""
        import torch
        from paper_2305_18236_amd import _native
        pid = PATH_ID[path]
        need = _native.mg_gemm_workspace_size(pid, self.tA, self.tB, self.M, self.N, self.K)
        if not use_workspace:
            need = 0
        ws_ptr, ws_bytes = None, 0
        if need:
            if workspace is None or workspace.numel() < need:
                workspace = torch.empty(need, dtype=torch.uint8, device=self.dA.device)
            ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel()
        if stream is None:
            stream = torch.cuda.current_stream(self.dA.device).cuda_stream
        return _native.mg_gemm(pid, self.tA, self.tB, self.M, self.N, self.K, self.alpha,
                               self.dA.data_ptr(), self.lda, self.dB.data_ptr(), self.ldb, self.beta,
                               self.dC.data_ptr(), self.ldc, ws_ptr, ws_bytes, stream)

    def result(self) -> np.ndarray:
        import torch
        torch.cuda.synchronize()
        full = self.dC.cpu().numpy().reshape(max(self.M, 1), max(self.ldc, 1))
        return full[:self.M, :self.N].astype(np.float64)

    def padding_untouched(self) -> bool:
        import torch
        torch.cuda.synchronize()
        full = self.dC.cpu().numpy().reshape(max(self.M, 1), max(self.ldc, 1))
        return bool(np.all(full[:self.M, self.N:] == -7.0))
