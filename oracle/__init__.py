"""FP64 CPU oracle for the layered GEMM library -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The GPU library never loads it, and it shares no
code with the GPU library.

The arithmetic lives in ``oracle.c`` (plain C, FP64, no FMA contraction, no
fast-math); this module only marshals numpy arrays.  Each wrapper names the
passage of Kuzma et al. (SPE 2023) it follows; see the header of ``oracle.c``
for the readings taken where the paper is silent.

Every function here has a pin in ``tests/test_oracle_pins.py`` that checks it
against something other than itself (exact rational arithmetic, closed forms,
library conversions, invariants).
"""
from __future__ import annotations

import ctypes
import functools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_CFLAGS = ["-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off", "-shared", "-fPIC"]

_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (the checker's own build)."""
    stale = (not os.path.exists(_LIB_PATH)) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    if force or stale:
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = ctypes.CDLL(build())
    i64, dbl, ptr = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.oracle_gemm.argtypes = [ctypes.c_char, ctypes.c_char, i64, i64, i64, dbl, ptr, i64,
                                ptr, i64, dbl, ptr, i64, ptr, ptr, i64, ctypes.c_int]
    lib.oracle_gemm.restype = ctypes.c_int
    lib.oracle_gemm_entries.argtypes = [ctypes.c_char, ctypes.c_char, i64, dbl, ptr, i64, ptr, i64,
                                        dbl, ptr, i64, i64, ptr, ptr, ptr, ptr, ctypes.c_int]
    lib.oracle_gemm_entries.restype = ctypes.c_int
    lib.oracle_round_to_bits.argtypes = [dbl, ctypes.c_int, ctypes.c_int]
    lib.oracle_round_to_bits.restype = dbl
    lib.oracle_bf16_split.argtypes = [i64, ptr, ptr, ptr]
    lib.oracle_bf16_round.argtypes = [i64, ptr, ptr]
    lib.oracle_e4m3_value.argtypes = [dbl]
    lib.oracle_e4m3_value.restype = dbl
    lib.oracle_e4m3_encode.argtypes = [dbl]
    lib.oracle_e4m3_encode.restype = ctypes.c_uint8
    lib.oracle_e4m3_decode.argtypes = [ctypes.c_uint8]
    lib.oracle_e4m3_decode.restype = dbl
    lib.oracle_tile_scale.argtypes = [dbl]
    lib.oracle_tile_scale.restype = dbl
    lib.oracle_fp8_quantize.argtypes = [i64, i64, ptr, i64, i64, ptr, ptr]
    lib.oracle_fp16_round.argtypes = [i64, ptr, ptr]
    i32 = ctypes.c_int32
    lib.oracle_gemm_i8.argtypes = [ctypes.c_char, ctypes.c_char, i64, i64, i64, i32, ptr, i64, ptr, i64,
                                   i32, ptr, i64, ptr, i64, ctypes.c_int]
    lib.oracle_gemm_i8.restype = ctypes.c_int
    lib.oracle_syr2k.argtypes = [ctypes.c_char, ctypes.c_char, i64, i64, dbl, ptr, i64, ptr, i64, dbl,
                                 ptr, i64, ptr, ctypes.c_int]
    lib.oracle_syr2k.restype = ctypes.c_int
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _threads(n):
    return max_threads() if n is None else int(n)


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _tchar(t: str) -> bytes:
    return t.encode() if isinstance(t, str) else t


def gemm(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta=0.0, C0=None, ldc0=None,
         threads=None):
    """C = alpha*op(A)*op(B) + beta*C0 and the error denominator D, both M x N float64.

    Follows the GEMM statement of Section 3 / Algorithm 1 (beta scales C once,
    alpha scales the product; lda/ldb are row strides of the stored operands).
    A, B (and C0) are 1-D or 2-D buffers in the stored layout; they are widened
    to float64, which is exact for float32 data.
    """
    lib = _load()
    A64, B64 = _f64(A).reshape(-1), _f64(B).reshape(-1)
    if beta != 0.0:
        C064 = _f64(C0).reshape(-1)
        ldc0 = N if ldc0 is None else ldc0
    else:
        C064, ldc0 = np.zeros(1), 1
    C = np.empty((M, N), dtype=np.float64)
    D = np.empty((M, N), dtype=np.float64)
    if M and N:
        rc = lib.oracle_gemm(_tchar(transA), _tchar(transB), M, N, K, float(alpha), _p(A64), lda,
                             _p(B64), ldb, float(beta), _p(C064), ldc0, _p(C), _p(D), max(N, 1),
                             _threads(threads))
        if rc != 0:
            raise ValueError("oracle_gemm: bad transpose character")
    return C, D


def gemm_logical(opA, opB, alpha=1.0, beta=0.0, C0=None, threads=None):
    """The same GEMM on logical (already transposed) operands opA (M x K), opB (K x N)."""
    opA = np.asarray(opA)
    opB = np.asarray(opB)
    M, K = opA.shape
    K2, N = opB.shape
    assert K == K2
    return gemm("N", "N", M, N, K, alpha, opA, max(K, 1), opB, max(N, 1), beta,
                None if C0 is None else np.asarray(C0), N, threads=threads)


def gemm_entries(transA, transB, K, alpha, A, lda, B, ldb, beta, C0, ldc0, I, J, threads=None):
    """The GEMM definition evaluated only at positions (I[s], J[s]); returns (C, D) vectors."""
    lib = _load()
    A64, B64 = _f64(A).reshape(-1), _f64(B).reshape(-1)
    if beta != 0.0:
        C064 = _f64(C0).reshape(-1)
    else:
        C064, ldc0 = np.zeros(1), 1
    I = np.ascontiguousarray(I, dtype=np.int64)
    J = np.ascontiguousarray(J, dtype=np.int64)
    C = np.empty(I.shape[0], dtype=np.float64)
    D = np.empty(I.shape[0], dtype=np.float64)
    rc = lib.oracle_gemm_entries(_tchar(transA), _tchar(transB), K, float(alpha), _p(A64), lda,
                                 _p(B64), ldb, float(beta), _p(C064), ldc0, I.shape[0], _p(I),
                                 _p(J), _p(C), _p(D), _threads(threads))
    if rc != 0:
        raise ValueError("oracle_gemm_entries: bad transpose character")
    return C, D


def normalized_error(C, C_ref, D) -> float:
    """max_ij |C - C_ref| / D with 0/0 = 0; a non-zero difference over D = 0 is infinite.

    A NaN anywhere in C where C_ref is finite also counts as infinite.
    """
    C = np.asarray(C, dtype=np.float64)
    C_ref = np.asarray(C_ref, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    diff = np.abs(C - C_ref)
    if np.any(np.isnan(diff) & ~np.isnan(C_ref)):
        return float("inf")
    diff = np.where(np.isnan(C_ref) & np.isnan(C), 0.0, diff)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(diff == 0.0, 0.0, diff / D)
    return float(np.max(r)) if r.size else 0.0


# ------------------------------------------------------------ precision ----

def round_to_bits(x: float, bits: int, emin: int) -> float:
    return float(_load().oracle_round_to_bits(float(x), int(bits), int(emin)))


def bf16_round(x):
    """Round each element to bfloat16, nearest-even (Table 1's 16-bit operand type)."""
    x64 = _f64(x)
    out = np.empty_like(x64)
    _load().oracle_bf16_round(x64.size, _p(x64), _p(out))
    return out


def bf16_split(x):
    """hi = bf16(x), lo = bf16(x - hi) per element, as float64 values."""
    x64 = _f64(x)
    hi = np.empty_like(x64)
    lo = np.empty_like(x64)
    _load().oracle_bf16_split(x64.size, _p(x64), _p(hi), _p(lo))
    return hi, lo


def fp16_round(x):
    """Round each element to IEEE binary16, nearest-even, overflow to infinity
    (Table 1's 16-bit floating operand type)."""
    x64 = _f64(x)
    out = np.empty_like(x64)
    _load().oracle_fp16_round(x64.size, _p(x64), _p(out))
    return out


def e4m3_value(x: float) -> float:
    return float(_load().oracle_e4m3_value(float(x)))


def e4m3_encode(v: float) -> int:
    return int(_load().oracle_e4m3_encode(float(v)))


def e4m3_decode(b) -> np.ndarray:
    lib = _load()
    b = np.asarray(b, dtype=np.uint8)
    flat = b.reshape(-1)
    out = np.array([lib.oracle_e4m3_decode(int(v)) for v in flat], dtype=np.float64)
    return out.reshape(b.shape)


def e4m3_decode_table() -> np.ndarray:
    """Value of each of the 256 E4M3 bytes."""
    lib = _load()
    return np.array([lib.oracle_e4m3_decode(v) for v in range(256)], dtype=np.float64)


def tile_scale(amax: float) -> float:
    return float(_load().oracle_tile_scale(float(amax)))


def fp8_quantize(X, tile: int = 128):
    """Per-tile E4M3 quantisation of a logical matrix X (rows x cols).

    Returns (q uint8 rows x cols, scales float32 ceil(rows/tile) x ceil(cols/tile)).
    """
    X64 = _f64(X)
    rows, cols = X64.shape
    tr, tc = -(-rows // tile), -(-cols // tile)
    q = np.zeros((rows, cols), dtype=np.uint8)
    s = np.zeros((tr, tc), dtype=np.float32)
    if rows and cols:
        _load().oracle_fp8_quantize(rows, cols, _p(X64), cols, tile, _p(q), _p(s))
    return q, s


def fp8_dequantize(q, scales, tile: int = 128) -> np.ndarray:
    """Exact value of each quantised element: decode(q) * scale of its tile."""
    vals = e4m3_decode_table()[np.asarray(q, dtype=np.uint8)]
    rows, cols = vals.shape
    s = np.asarray(scales, dtype=np.float64)
    srow = np.repeat(np.repeat(s, tile, axis=0), tile, axis=1)[:rows, :cols]
    return vals * srow


# ------------------------------------------------------------- gradients ---

def chain_forward(X, W1, W2, threads=None):
    """H = X*W1 and Y = H*W2 in FP64 (two applications of the GEMM definition)."""
    H, _ = gemm_logical(X, W1, threads=threads)
    Y, _ = gemm_logical(H, W2, threads=threads)
    return H, Y


def chain_grads(X, W1, W2, G, threads=None):
    """Gradients of loss = sum(Y * G) for Y = (X*W1)*W2, in FP64.

    dY = G; dW2 = H^T G; dH = G W2^T; dW1 = X^T dH; dX = dH W1^T.  Each is
    one oracle GEMM with a transposed operand.  Returns (grads, denominators)
    where each denominator is the same chain applied to absolute values, the
    error scale of a product of products.
    """
    X, W1, W2, G = (_f64(a) for a in (X, W1, W2, G))
    H, _ = gemm_logical(X, W1, threads=threads)
    aH, _ = gemm_logical(np.abs(X), np.abs(W1), threads=threads)
    dW2, _ = gemm_logical(H.T, G, threads=threads)
    dH, _ = gemm_logical(G, W2.T, threads=threads)
    adH, _ = gemm_logical(np.abs(G), np.abs(W2).T, threads=threads)
    dW1, _ = gemm_logical(X.T, dH, threads=threads)
    dX, _ = gemm_logical(dH, W1.T, threads=threads)
    den = {
        "dW2": gemm_logical(aH.T, np.abs(G), threads=threads)[0],
        "dW1": gemm_logical(np.abs(X).T, adH, threads=threads)[0],
        "dX": gemm_logical(adH, np.abs(W1).T, threads=threads)[0],
    }
    return {"dX": dX, "dW1": dW1, "dW2": dW2}, den


def chain_entries(X, W1, W2, G, n=16, seed=0, threads=None):
    """Y and the three gradients of chain_grads at sampled entries, with their
    chained denominators, from oracle GEMMs on slices of the operands only
    (the same definitions restricted to the sampled rows and columns, so a
    full-size chain needs no full-size FP64 product).  Returns
    {name: (I, J, values at (I x J), denominators at (I x J))} for Y, dX, dW1
    and dW2, n row indices I and n column indices J each, drawn without
    replacement from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    X, W1, W2, G = (_f64(a) for a in (X, W1, W2, G))
    Mx, D = X.shape
    Hd = W1.shape[1]
    aX, aW1, aW2, aG = (np.abs(a) for a in (X, W1, W2, G))
    gl = functools.partial(gemm_logical, threads=threads)
    out = {}
    # dW2[i, j] = sum_m H[m, i] G[m, j], with H[:, i] = X W1[:, i]
    I = rng.choice(Hd, min(n, Hd), replace=False)
    J = rng.choice(D, min(n, D), replace=False)
    H_I, aH_I = gl(X, W1[:, I])[0], gl(aX, aW1[:, I])[0]
    out["dW2"] = (I, J, gl(H_I.T, G[:, J])[0], gl(aH_I.T, aG[:, J])[0])
    # dW1[i, j] = sum_m X[m, i] dH[m, j], with dH[:, j] = G W2[j, :]^T
    I = rng.choice(D, min(n, D), replace=False)
    J = rng.choice(Hd, min(n, Hd), replace=False)
    dH_J, adH_J = gl(G, W2[J, :].T)[0], gl(aG, aW2[J, :].T)[0]
    out["dW1"] = (I, J, gl(X[:, I].T, dH_J)[0], gl(aX[:, I].T, adH_J)[0])
    # dX[i, j] = sum_h dH[i, h] W1[j, h], with dH[i, :] = G[i, :] W2^T
    I = rng.choice(Mx, min(n, Mx), replace=False)
    J = rng.choice(D, min(n, D), replace=False)
    dH_I, adH_I = gl(G[I, :], W2.T)[0], gl(aG[I, :], aW2.T)[0]
    out["dX"] = (I, J, gl(dH_I, W1[J, :].T)[0], gl(adH_I, aW1[J, :].T)[0])
    # Y[i, j] = (X W1)[i, :] W2[:, j]; its denominator (|X||W1|)|W2|
    I = rng.choice(Mx, min(n, Mx), replace=False)
    J = rng.choice(W2.shape[1], min(n, W2.shape[1]), replace=False)
    H_rows, aH_rows = gl(X[I, :], W1)[0], gl(aX[I, :], aW1)[0]
    out["Y"] = (I, J, gl(H_rows, W2[:, J])[0], gl(aH_rows, aW2[:, J])[0])
    return out


# ----------------------------------------------------------------- INT8 ----

def gemm_i8(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta=0, C0=None, ldc0=None, threads=None):
    """Integer GEMM of Table 1's 8-bit operand type: int8 A and B stored as
    for gemm (row strides lda, ldb), int32 alpha, beta and C0.  Returns the
    M x N int32 result alpha*op(A)*op(B) + beta*C0, computed exactly and
    wrapped modulo 2^32."""
    A8 = np.ascontiguousarray(A, dtype=np.int8)
    B8 = np.ascontiguousarray(B, dtype=np.int8)
    C = np.zeros((max(M, 1), max(N, 1)), dtype=np.int32)
    if C0 is None:
        C0a = np.zeros(1, dtype=np.int32)
        ldc0 = 1
        if beta != 0:
            raise ValueError("beta != 0 needs C0")
    else:
        C0a = np.ascontiguousarray(C0, dtype=np.int32)
        ldc0 = N if ldc0 is None else ldc0
    _load().oracle_gemm_i8(_tchar(transA), _tchar(transB), M, N, K, int(alpha), _p(A8), lda, _p(B8), ldb,
                           int(beta), _p(C0a), ldc0, _p(C), max(N, 1), _threads(threads))
    return C[:M, :N]


# ---------------------------------------------------------------- SYR2K ----

def syr2k(uplo, trans, N, K, alpha, A, lda, B, ldb, beta=0.0, C0=None, ldc=None, threads=None):
    """The SYR2K of Section 5.1 on one triangle, FP64.  A and B are stored as
    N x K (trans 'N') or K x N (trans 'T') with row strides lda, ldb; C0 is
    N x N with row stride ldc (default N).  Returns (C, D): C is C0 with the
    uplo triangle replaced by alpha*(X Y^T + Y X^T) + beta*C0 (the other
    triangle copied from C0 untouched), D the error denominator on the
    triangle (0 elsewhere)."""
    ldc = max(N, 1) if ldc is None else ldc
    if C0 is None:
        C = np.zeros(max(N, 1) * ldc, dtype=np.float64)
    else:
        C = np.array(C0, dtype=np.float64).reshape(-1).copy()
    D = np.zeros(max(N, 1) * max(N, 1), dtype=np.float64)
    A64, B64 = _f64(A), _f64(B)
    _load().oracle_syr2k(_tchar(uplo), _tchar(trans), N, K, float(alpha), _p(A64), lda, _p(B64), ldb,
                         float(beta), _p(C), ldc, _p(D), _threads(threads))
    return C, D.reshape(max(N, 1), max(N, 1))[:N, :N]


def syr2k_entries(trans, K, alpha, A, lda, B, ldb, beta, C0, ldc0, I, J, threads=None):
    """The SYR2K of Section 5.1 at given entries (i, j) only, with its error
    denominator: C[i][j] = alpha*(op(X) op(Y)^T)[i][j] + alpha*(op(Y) op(X)^T)[i][j]
    + beta*C0[i][j], D = |alpha| sum_k (|x_ik||y_jk| + |y_ik||x_jk|) + |beta||C0[i][j]|,
    where op(X) is A (trans 'N', stored N x K) or A^T ('T', stored K x N), and
    likewise op(Y) from B.  Built from the oracle's GEMM entries: the first
    product carries beta*C0, the second is added in FP64 (one extra rounding,
    far below every tolerance).  Which triangle (i, j) lies in is the caller's
    choice; the value does not depend on it."""
    t1 = "N" if _tchar(trans) == b"N" else "T"
    t2 = "T" if t1 == "N" else "N"
    c1, d1 = gemm_entries(t1, t2, K, alpha, A, lda, B, ldb, beta, C0, ldc0, I, J, threads=threads)
    c2, d2 = gemm_entries(t1, t2, K, alpha, B, ldb, A, lda, 0.0, None, ldc0, I, J, threads=threads)
    return c1 + c2, d1 + d2
