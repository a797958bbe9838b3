"""ctypes binding of libmgemm.so: argument marshalling only.

Every function here has the name and argument order of the C entry point
declared in include/mgemm.h and passes raw device pointers and sizes through.
No arithmetic of the GEMM happens in Python.  If the library has not been
built, loading fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmgemm.so")

_lib = None


class mg_problem(ctypes.Structure):
    """Mirror of struct mg_problem in include/mgemm.h."""
    _fields_ = [("transA", ctypes.c_char), ("transB", ctypes.c_char),
                ("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64),
                ("alpha", ctypes.c_float), ("beta", ctypes.c_float),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64)]


class MgemmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: status {status} ({status_string(status)})")


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2305_18236_amd.build` "
                          "(the HIP library is required; there is no CPU fallback)")
    # torch ships its own HIP runtime under the same soname as the system's
    # (libamdhip64.so.7).  Whichever is loaded first serves the whole
    # process, so torch is imported first: the library then shares torch's
    # runtime, devices and streams instead of bringing in a second one that
    # torch would later fail to initialise against.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    i64, f32, vp, ch, ci = ctypes.c_int64, ctypes.c_float, ctypes.c_void_p, ctypes.c_char, ctypes.c_int
    L.mg_sgemm.argtypes = [ch, ch, i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64, vp]
    L.mg_sgemm.restype = ci
    L.mg_gemm.argtypes = [ci, ch, ch, i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64, vp,
                          ctypes.c_size_t, vp]
    L.mg_gemm.restype = ci
    L.mg_gemm_noalloc.argtypes = [ci, ch, ch, i64, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64, vp]
    L.mg_gemm_noalloc.restype = ci
    L.mg_gemm_workspace_size.argtypes = [ci, ch, ch, i64, i64, i64]
    L.mg_gemm_workspace_size.restype = ctypes.c_size_t
    L.mg_num_configs.argtypes = [ci]
    L.mg_num_configs.restype = ci
    L.mg_config_info.argtypes = [ci, ci, ctypes.POINTER(ci)]
    L.mg_config_info.restype = ci
    L.mg_force_config.argtypes = [ci, ci]
    L.mg_force_config.restype = ci
    L.mg_config_uses_mfma.argtypes = [ci, ci]
    L.mg_config_uses_mfma.restype = ci
    L.mg_config_packs.argtypes = [ci, ci]
    L.mg_config_packs.restype = ci
    L.mg_force_splits.argtypes = [ci, ci]
    L.mg_force_splits.restype = ci
    L.mg_force_tile_order.argtypes = [ci, ci, ci]
    L.mg_force_tile_order.restype = ci
    L.mg_split_count.argtypes = [ci, i64, i64, i64]
    L.mg_split_count.restype = ci
    L.mg_gemm_plan.argtypes = [ci, i64, i64, i64, ctypes.c_size_t, ctypes.POINTER(ci)]
    L.mg_gemm_plan.restype = ci
    L.mg_bf16_split.argtypes = [vp, i64, vp, vp, vp]
    L.mg_bf16_split.restype = ci
    sz = ctypes.c_size_t
    L.mg_fp8_packed_size.argtypes = [i64, i64, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    L.mg_fp8_packed_size.restype = ci
    L.mg_fp8_pack.argtypes = [ch, i64, i64, vp, i64, vp, vp, vp]
    L.mg_fp8_pack.restype = ci
    L.mg_gemm_fp8_packed.argtypes = [i64, i64, i64, f32, vp, vp, vp, vp, f32, vp, i64, vp]
    L.mg_gemm_fp8_packed.restype = ci
    L.mg_syr2k.argtypes = [ci, ch, ch, i64, i64, f32, vp, i64, vp, i64, f32, vp, i64, vp, sz, vp]
    L.mg_syr2k.restype = ci
    L.mg_syr2k_workspace_size.argtypes = [ci, i64, i64]
    L.mg_syr2k_workspace_size.restype = sz
    L.mg_syr2k_plan.argtypes = [ci, i64, i64, ctypes.POINTER(ci)]
    L.mg_syr2k_plan.restype = ci
    i32 = ctypes.c_int32
    L.mg_gemm_i8.argtypes = [ch, ch, i64, i64, i64, i32, vp, i64, vp, i64, i32, vp, i64, vp, sz, vp]
    L.mg_gemm_i8.restype = ci
    L.mg_gemm_i8_workspace_size.argtypes = [i64, i64, i64]
    L.mg_gemm_i8_workspace_size.restype = sz
    L.mg_i8_packed_size.argtypes = [i64, i64, ctypes.POINTER(sz)]
    L.mg_i8_packed_size.restype = ci
    L.mg_i8_pack.argtypes = [ch, i64, i64, vp, i64, vp, vp]
    L.mg_i8_pack.restype = ci
    L.mg_gemm_i8_packed.argtypes = [i64, i64, i64, i32, vp, vp, i32, vp, i64, vp]
    L.mg_gemm_i8_packed.restype = ci
    L.mg_load_tuning.argtypes = [ctypes.c_char_p]
    L.mg_load_tuning.restype = ci
    L.mg_tuned_config.argtypes = [ci, i64, i64, i64]
    L.mg_tuned_config.restype = ci
    L.mg_batched_config.argtypes = [ci, i64, i64, i64]
    L.mg_batched_config.restype = ci
    L.mg_gemm_batched_workspace_size.argtypes = [ci, i64]
    L.mg_gemm_batched_workspace_size.restype = sz
    L.mg_gemm_batched.argtypes = [ci, i64, ctypes.POINTER(mg_problem), vp, sz, vp,
                                  ctypes.POINTER(i64)]
    L.mg_gemm_batched.restype = ci
    L.mg_batched_slots.argtypes = [ci]
    L.mg_batched_slots.restype = ci
    L.mg_gemm_batched_timed.argtypes = [ci, i64, ctypes.POINTER(mg_problem), vp, sz, vp, ctypes.POINTER(i64),
                                        vp, i64, ctypes.POINTER(ci)]
    L.mg_gemm_batched_timed.restype = ci
    L.mg_wall_clock_hz.argtypes = []
    L.mg_wall_clock_hz.restype = i64
    L.mg_shader_clock_mhz.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double)]
    L.mg_shader_clock_mhz.restype = ci
    L.mg_status_string.argtypes = [ci]
    L.mg_status_string.restype = ctypes.c_char_p
    _lib = L
    _load_default_tuning(L)
    return L


TUNING_TABLE = os.path.join(_PKG, "tuning_table.txt")


def _load_default_tuning(L):
    """Load the committed autotuner table (or $MGEMM_TUNING; "none" disables it)."""
    path = os.environ.get("MGEMM_TUNING", TUNING_TABLE)
    if path.lower() == "none" or not os.path.exists(path):
        return
    st = L.mg_load_tuning(os.fsencode(path))
    if st != 0:
        raise MgemmError(st, f"mg_load_tuning({path})")


def _c(t) -> bytes:
    return t.encode() if isinstance(t, str) else bytes(t)


def status_string(status: int) -> str:
    return lib().mg_status_string(int(status)).decode()


def check(status: int, where: str) -> None:
    if status != 0:
        raise MgemmError(status, where)


def mg_sgemm(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream) -> int:
    return lib().mg_sgemm(_c(transA), _c(transB), M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream)


def mg_gemm(path, transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
            workspace, workspace_bytes, stream) -> int:
    return lib().mg_gemm(int(path), _c(transA), _c(transB), M, N, K, alpha, A, lda, B, ldb, beta,
                         C, ldc, workspace, workspace_bytes, stream)


def mg_gemm_noalloc(path, transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream) -> int:
    return lib().mg_gemm_noalloc(int(path), _c(transA), _c(transB), M, N, K, alpha, A, lda, B, ldb, beta,
                                 C, ldc, stream)


def mg_gemm_workspace_size(path, transA, transB, M, N, K) -> int:
    return int(lib().mg_gemm_workspace_size(int(path), _c(transA), _c(transB), M, N, K))


def mg_bf16_split(x, n, hi, lo, stream) -> int:
    return lib().mg_bf16_split(x, n, hi, lo, stream)


def mg_fp8_packed_size(R, K):
    q = ctypes.c_size_t()
    s = ctypes.c_size_t()
    check(lib().mg_fp8_packed_size(R, K, ctypes.byref(q), ctypes.byref(s)), "mg_fp8_packed_size")
    return int(q.value), int(s.value)


def mg_fp8_pack(trans, R, K, X, ldx, q, scales, stream) -> int:
    return lib().mg_fp8_pack(_c(trans), R, K, X, ldx, q, scales, stream)


def mg_gemm_fp8_packed(M, N, K, alpha, qA, sA, qB, sB, beta, C, ldc, stream) -> int:
    return lib().mg_gemm_fp8_packed(M, N, K, alpha, qA, sA, qB, sB, beta, C, ldc, stream)


def mg_syr2k(path, uplo, trans, N, K, alpha, A, lda, B, ldb, beta, C, ldc, workspace, workspace_bytes,
             stream) -> int:
    return lib().mg_syr2k(int(path), _c(uplo), _c(trans), N, K, alpha, A, lda, B, ldb, beta, C, ldc, workspace,
                          workspace_bytes, stream)


def mg_syr2k_workspace_size(path, N, K) -> int:
    return int(lib().mg_syr2k_workspace_size(int(path), N, K))


def mg_syr2k_plan(path, N, K):
    """(status, config, splits) of the tiles mg_syr2k would run."""
    out = (ctypes.c_int * 2)()
    st = int(lib().mg_syr2k_plan(int(path), N, K, out))
    return st, int(out[0]), int(out[1])


def mg_gemm_i8(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, workspace, workspace_bytes,
               stream) -> int:
    return lib().mg_gemm_i8(_c(transA), _c(transB), M, N, K, int(alpha), A, lda, B, ldb, int(beta), C, ldc,
                            workspace, workspace_bytes, stream)


def mg_gemm_i8_workspace_size(M, N, K) -> int:
    return int(lib().mg_gemm_i8_workspace_size(M, N, K))


def mg_i8_packed_size(R, K) -> int:
    b = ctypes.c_size_t()
    check(lib().mg_i8_packed_size(R, K, ctypes.byref(b)), "mg_i8_packed_size")
    return int(b.value)


def mg_i8_pack(trans, R, K, X, ldx, q, stream) -> int:
    return lib().mg_i8_pack(_c(trans), R, K, X, ldx, q, stream)


def mg_gemm_i8_packed(M, N, K, alpha, qA, qB, beta, C, ldc, stream) -> int:
    return lib().mg_gemm_i8_packed(M, N, K, int(alpha), qA, qB, int(beta), C, ldc, stream)


def mg_load_tuning(path) -> int:
    return lib().mg_load_tuning(None if path is None else os.fsencode(path))


def mg_tuned_config(path, M, N, K) -> int:
    return int(lib().mg_tuned_config(int(path), M, N, K))


def mg_batched_config(path, M, N, K) -> int:
    return int(lib().mg_batched_config(int(path), M, N, K))


def mg_gemm_batched_workspace_size(path, count) -> int:
    return int(lib().mg_gemm_batched_workspace_size(int(path), int(count)))


def mg_gemm_batched(path, count, problems, workspace, workspace_bytes, stream):
    """problems: a ctypes array of mg_problem.  Returns (status, bad_problem index)."""
    bad = ctypes.c_int64(-1)
    st = lib().mg_gemm_batched(int(path), int(count), problems, workspace, workspace_bytes, stream,
                               ctypes.byref(bad))
    return int(st), int(bad.value)


def mg_batched_slots(path) -> int:
    return int(lib().mg_batched_slots(int(path)))


def mg_gemm_batched_timed(path, count, problems, workspace, workspace_bytes, stream, stamps, stamps_len):
    """As mg_gemm_batched, plus per-workgroup start/end wall-clock stamps
    (device array).  Returns (status, bad_problem index, grid)."""
    bad = ctypes.c_int64(-1)
    grid = ctypes.c_int(0)
    st = lib().mg_gemm_batched_timed(int(path), int(count), problems, workspace, workspace_bytes, stream,
                                     ctypes.byref(bad), stamps, int(stamps_len), ctypes.byref(grid))
    return int(st), int(bad.value), int(grid.value)


def mg_wall_clock_hz() -> int:
    return int(lib().mg_wall_clock_hz())


def mg_num_configs(path) -> int:
    return int(lib().mg_num_configs(int(path)))


def mg_config_info(path, index):
    out = (ctypes.c_int * 6)()
    st = lib().mg_config_info(int(path), int(index), out)
    check(st, "mg_config_info")
    return dict(zip(("id", "bm", "bn", "bk", "wm", "wn"), list(out)))


def mg_force_config(path, config_id) -> int:
    return int(lib().mg_force_config(int(path), int(config_id)))


def mg_config_packs(path, index) -> int:
    return int(lib().mg_config_packs(int(path), int(index)))


def mg_config_uses_mfma(path, index) -> int:
    return int(lib().mg_config_uses_mfma(int(path), int(index)))


def mg_force_splits(path, splits) -> int:
    return int(lib().mg_force_splits(int(path), int(splits)))


def mg_force_tile_order(path, remap, group_m=4) -> int:
    return int(lib().mg_force_tile_order(int(path), int(remap), int(group_m)))


def mg_split_count(path, M, N, K) -> int:
    return int(lib().mg_split_count(int(path), M, N, K))


def mg_gemm_plan(path, M, N, K, workspace_bytes):
    """(status, config, splits, prepacked) of the plan mg_gemm would run."""
    out = (ctypes.c_int * 3)()
    st = int(lib().mg_gemm_plan(int(path), M, N, K, int(workspace_bytes), out))
    return st, int(out[0]), int(out[1]), int(out[2])


def mg_shader_clock_mhz(stream, microseconds=50):
    """(status, MHz): the shader clock measured by a probe queued on `stream`."""
    out = ctypes.c_double(0.0)
    st = int(lib().mg_shader_clock_mhz(stream, int(microseconds), ctypes.byref(out)))
    return st, float(out.value)
