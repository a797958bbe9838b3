"""mgemm: the layered GEMM of Kuzma et al. (SPE 2023) on AMD MI355X (gfx950).

The compute runs in the HIP kernels of ``libmgemm.so`` (C ABI in
``include/mgemm.h``).  This package only marshals torch tensors into device
pointers, strides and the current HIP stream.  PyTorch provides device memory
and streams; it computes nothing on the GEMM path.
"""
from __future__ import annotations

import os

from . import _native
from ._native import MgemmError, check, status_string  # noqa: F401

PATHS = {"fp32": 0, "bf16x3": 1, "bf16": 2, "fp8": 3, "fp16": 4}


def _path_id(path) -> int:
    if isinstance(path, str):
        try:
            return PATHS[path]
        except KeyError:
            raise ValueError(f"unknown path {path!r}; expected one of {sorted(PATHS)}") from None
    return int(path)


def operand_layout(X):
    """('N', ld) for a row-major 2-D view, ('T', ld) for a column-major one.

    A contiguous tensor is 'N' with ld = stride(0); the .t() of a contiguous
    tensor is 'T' with ld = stride(1).  Any other stride pattern is rejected
    (no hidden copy is made).
    """
    if X.dim() != 2:
        raise ValueError("operands must be 2-D")
    r, c = X.shape
    s0, s1 = X.stride()
    # A stride only matters along a dimension longer than 1; where it matters
    # it is taken as it is (never raised), so a broadcast view (stride 0) or
    # rows that overlap are refused instead of being read out of bounds.
    if (s1 == 1 or c <= 1) and (r <= 1 or s0 >= max(c, 1)):
        return "N", s0 if r > 1 else max(c, 1)
    if (s0 == 1 or r <= 1) and (c <= 1 or s1 >= max(r, 1)):
        return "T", s1 if c > 1 else max(r, 1)
    raise ValueError(f"operand strides {X.stride()} are neither row- nor column-major")


def output_ld(C) -> int:
    """Row stride of an output C (M x N) with unit column stride; rows that
    overlap (a broadcast or otherwise aliased view) are refused, since the
    kernels would write past the tensor's storage."""
    M, N = C.shape
    if C.stride(1) != 1 and N > 1:
        raise ValueError("C must have unit column stride")
    if M > 1 and C.stride(0) < max(N, 1):
        raise ValueError(f"C strides {C.stride()} make rows overlap")
    return C.stride(0) if M > 1 else max(N, 1)


def _stream_ptr(device):
    import torch
    return torch.cuda.current_stream(device).cuda_stream


def gemm(A, B, C=None, *, alpha: float = 1.0, beta: float = 0.0, path="fp32", workspace=None):
    """C <- alpha * A @ B + beta * C on the GPU, with A (M x K) and B (K x N) float32.

    A and B may be row-major or transposed views; C must be row-major
    (contiguous rows).  If C is None a new M x N tensor is returned (and beta
    must be 0).  ``path`` is "fp32", "bf16x3", "bf16", "fp16" or "fp8".
    """
    import torch
    if A.dtype != torch.float32 or B.dtype != torch.float32:
        raise TypeError("A and B must be float32")
    if not (A.is_cuda and B.is_cuda):
        raise ValueError("A and B must be on the GPU")
    M, K = A.shape
    K2, N = B.shape
    if K2 != K:
        raise ValueError(f"inner dimensions differ: {tuple(A.shape)} x {tuple(B.shape)}")
    if C is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs an input C")
        C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    if C.dtype != torch.float32 or tuple(C.shape) != (M, N) or not C.is_cuda:
        raise ValueError("C must be a float32 M x N GPU tensor")
    if C.dim() != 2:
        raise ValueError("C must be 2-D")
    ldc = output_ld(C)
    for X in (A, B):
        if X.numel() and C.numel() and X.data_ptr() == C.data_ptr():
            raise ValueError("C must not alias A or B")
    tA, lda = operand_layout(A)
    tB, ldb = operand_layout(B)
    pid = _path_id(path)
    need = _native.mg_gemm_workspace_size(pid, tA, tB, M, N, K)
    ws_ptr, ws_bytes = None, 0
    if need:
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=A.device)
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    st = _native.mg_gemm(pid, tA, tB, M, N, K, float(alpha), A.data_ptr(), lda, B.data_ptr(), ldb,
                         float(beta), C.data_ptr(), ldc, ws_ptr, ws_bytes, _stream_ptr(A.device))
    check(st, "mg_gemm")
    return C


def gemm_i8(A, B, C=None, *, alpha: int = 1, beta: int = 0, workspace=None):
    """C <- alpha * A @ B + beta * C with int8 A (M x K) and B (K x N) and
    int32 C, alpha, beta (sums exact, result modulo 2^32).  A and B may be
    row-major or transposed views; C must have unit column stride."""
    import torch
    if A.dtype != torch.int8 or B.dtype != torch.int8:
        raise TypeError("A and B must be int8")
    if not (A.is_cuda and B.is_cuda):
        raise ValueError("A and B must be on the GPU")
    M, K = A.shape
    K2, N = B.shape
    if K2 != K:
        raise ValueError(f"inner dimensions differ: {tuple(A.shape)} x {tuple(B.shape)}")
    if C is None:
        if beta != 0:
            raise ValueError("beta != 0 needs an input C")
        C = torch.empty((M, N), dtype=torch.int32, device=A.device)
    if C.dtype != torch.int32 or tuple(C.shape) != (M, N) or not C.is_cuda:
        raise ValueError("C must be an int32 M x N GPU tensor")
    if C.dim() != 2:
        raise ValueError("C must be 2-D")
    ldc = output_ld(C)
    tA, lda = operand_layout(A)
    tB, ldb = operand_layout(B)
    need = _native.mg_gemm_i8_workspace_size(M, N, K)
    ws_ptr, ws_bytes = None, 0
    if need:
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=A.device)
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    st = _native.mg_gemm_i8(tA, tB, M, N, K, int(alpha), A.data_ptr(), lda, B.data_ptr(), ldb, int(beta),
                            C.data_ptr(), ldc, ws_ptr, ws_bytes, _stream_ptr(A.device))
    check(st, "mg_gemm_i8")
    return C


def gemm_batched(problems, *, path="fp32", workspace=None):
    """Run a list of GEMMs in ONE persistent kernel launch.

    problems: iterable of (A, B, C, alpha, beta) with A (M x K), B (K x N)
    float32 GPU tensors (row-major or transposed views) and C (M x N,
    row-major) updated in place as C <- alpha*A@B + beta*C.
    """
    import torch
    problems = list(problems)
    arr = (_native.mg_problem * max(len(problems), 1))()
    dev = None
    for i, (A, B, C, alpha, beta) in enumerate(problems):
        if A.dtype != torch.float32 or B.dtype != torch.float32 or C.dtype != torch.float32:
            raise TypeError("operands must be float32")
        M, K = A.shape
        K2, N = B.shape
        if K2 != K or tuple(C.shape) != (M, N):
            raise ValueError(f"problem {i}: shapes {tuple(A.shape)} x {tuple(B.shape)} -> {tuple(C.shape)}")
        try:
            ldc = output_ld(C)
        except ValueError as e:
            raise ValueError(f"problem {i}: {e}") from None
        tA, lda = operand_layout(A)
        tB, ldb = operand_layout(B)
        arr[i] = _native.mg_problem(tA.encode(), tB.encode(), M, N, K, float(alpha), float(beta),
                                    A.data_ptr(), lda, B.data_ptr(), ldb, C.data_ptr(), ldc)
        dev = A.device
    if not problems:
        return
    pid = _path_id(path)
    need = _native.mg_gemm_batched_workspace_size(pid, len(problems))
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    st, bad = _native.mg_gemm_batched(pid, len(problems), arr, workspace.data_ptr(),
                                      workspace.numel() * workspace.element_size(), _stream_ptr(dev))
    if st != 0 and bad >= 0:
        raise MgemmError(st, f"mg_gemm_batched (problem {bad})")
    check(st, "mg_gemm_batched")
