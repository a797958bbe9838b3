"""Differentiable GEMM: a torch.autograd.Function whose backward is written by
hand and runs the library's transposed-operand kernels.

For C = A @ B (A: M x K, B: K x N) and an upstream gradient dC (M x N):
    dA = dC @ B^T   -> mg_gemm('N', 'T'), reading B in its stored layout;
    dB = A^T @ dC   -> mg_gemm('T', 'N'), reading A in its stored layout.
No transposed copy of A or B is ever made: the transposition is absorbed by
the kernels' packing step, which is how the paper handles transposed operands
(Section 3.1: after packing, the source storage order no longer matters).
The forward, dA and dB all run on the same arithmetic path ("fp32",
"bf16x3", "bf16" or "fp8").
"""
from __future__ import annotations

import torch

from . import gemm, operand_layout


def _as_operand(X):
    """X itself when it is row- or column-major, else a row-major copy
    (an upstream gradient can arrive with broadcast strides)."""
    try:
        operand_layout(X)
        return X
    except ValueError:
        return X.contiguous()


class GemmFn(torch.autograd.Function):
    """C = A @ B on the GPU with a hand-written backward."""

    @staticmethod
    def forward(ctx, A, B, path="fp32"):
        ctx.path = path
        ctx.save_for_backward(A, B)
        return gemm(A, B, path=path)

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        dC = _as_operand(dC)
        dA = dB = None
        if ctx.needs_input_grad[0]:
            dA = gemm(dC, B.t(), path=ctx.path)      # dC (M x N) @ B^T (N x K)
        if ctx.needs_input_grad[1]:
            dB = gemm(A.t(), dC, path=ctx.path)      # A^T (K x M) @ dC (M x N)
        return dA, dB, None


def matmul(A, B, path="fp32"):
    """Differentiable A @ B through the library."""
    return GemmFn.apply(A, B, path)


def chain(X, W1, W2, path="bf16x3"):
    """Y = (X @ W1) @ W2, the two-GEMM chain, each GEMM differentiable."""
    return matmul(matmul(X, W1, path), W2, path)
