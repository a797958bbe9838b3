"""CPU-side checks of the C ABI: the library loads, exports every symbol the
public header declares, and rejects invalid arguments on the host (before any
device call), with the documented BLAS-style codes."""
import ctypes
import os
import re

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgemm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def native():
    from paper_2305_18236_amd import _native
    _native.lib()
    return _native


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mg_sgemm", "mg_gemm", "mg_gemm_workspace_size", "mg_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol(native):
    L = ctypes.CDLL(native.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


FAKE = 0x1000   # never dereferenced: validation fails before any device call


def _call(native, **kw):
    a = dict(transA="N", transB="N", M=4, N=5, K=6, alpha=1.0, A=FAKE, lda=6, B=FAKE, ldb=5,
             beta=0.0, C=FAKE, ldc=5, stream=None)
    a.update(kw)
    return native.mg_sgemm(a["transA"], a["transB"], a["M"], a["N"], a["K"], a["alpha"], a["A"],
                           a["lda"], a["B"], a["ldb"], a["beta"], a["C"], a["ldc"], a["stream"])


@pytest.mark.parametrize("kw,code", [
    (dict(transA="X"), -1), (dict(transB="Q"), -2), (dict(M=-1), -3), (dict(N=-2), -4),
    (dict(K=-3), -5), (dict(A=None), -7), (dict(lda=5), -8), (dict(B=None), -9),
    (dict(ldb=4), -10), (dict(C=None), -12), (dict(ldc=4), -13),
    # transposed storage changes the minimum leading dimensions
    (dict(transA="T", lda=3), -8), (dict(transB="t", ldb=5), -10),
    # overflow of rows * ld
    (dict(lda=2 ** 62), -8),
    # first invalid argument wins (BLAS order)
    (dict(transA="X", M=-1), -1), (dict(M=-1, lda=0), -3),
])
def test_invalid_arguments_rejected_on_host(native, kw, code):
    assert _call(native, **kw) == code


def test_null_pointer_allowed_for_empty_extent(native):
    # M == 0: A and C have no elements; quick return without touching anything
    assert _call(native, M=0, A=None, C=None) == 0
    # N == 0: B and C empty
    assert _call(native, N=0, B=None, C=None, ldb=1, ldc=1) == 0


def test_status_strings(native):
    for code in (0, -1, -2, -3, -4, -5, -7, -8, -9, -10, -12, -13, -100, -101, -102, -103):
        s = native.status_string(code)
        assert s and s != "unknown status"
    assert native.status_string(12345) == "unknown status"


def test_config_registry(native):
    n = native.mg_num_configs(0)
    assert n >= 1
    for i in range(n):
        c = native.mg_config_info(0, i)
        assert c["id"] == i and c["bm"] % c["wm"] == 0 and c["bn"] % c["wn"] == 0
        assert c["bk"] % 2 == 0
        # LDS budget of a double-buffered FP32 panel pair (160 KiB per CU on gfx950)
        assert 2 * (c["bm"] + c["bn"]) * c["bk"] * 4 <= 160 * 1024
    packs = [native.mg_config_packs(0, i) for i in range(n)]
    assert set(packs) == {0, 1} and packs[:8] == [1] * 8
    mfma = [native.mg_config_uses_mfma(0, i) for i in range(n)]
    # 10 and 11 run the vector-ALU micro-kernel, every other one the matrix cores
    assert mfma[:10] == [1] * 10 and mfma[10:12] == [0, 0] and set(mfma[12:]) <= {1}
    assert packs[12:] == [1] * (n - 12)
    assert native.mg_config_uses_mfma(0, n) == -101
    assert native.mg_config_packs(0, n) == -101 and native.mg_config_packs(1, 0) == 1
    assert native.mg_force_config(0, n) == -101
    assert native.mg_force_config(9, 0) == -101
    assert native.mg_force_config(0, -1) == 0


def test_operand_layout_from_strides():
    from paper_2305_18236_amd import operand_layout
    X = torch.empty(5, 7)
    assert operand_layout(X) == ("N", 7)
    assert operand_layout(X.t()) == ("T", 7)
    big = torch.empty(5, 12)
    assert operand_layout(big[:, :7]) == ("N", 12)
    assert operand_layout(big[:, :7].t()) == ("T", 12)
    with pytest.raises(ValueError):
        operand_layout(torch.empty(4, 6)[:, ::2])


def test_operand_layout_refuses_broadcast_views():
    """A column (M x 1) or row (1 x N) expanded from one element has stride 0
    along its long dimension: reading it with any ld >= 1 would run past the
    one stored element, so it must be refused (the autograd layer then makes
    a contiguous copy)."""
    from paper_2305_18236_amd import operand_layout
    from paper_2305_18236_amd.autograd import _as_operand
    one = torch.ones(1, 1)
    col = one.expand(6, 1)
    row = one.expand(1, 6)
    assert col.stride()[0] == 0 and row.stride()[1] == 0
    for X in (col, row, torch.ones(1, 6).expand(4, 6), torch.ones(5, 1).expand(5, 3)):
        with pytest.raises(ValueError):
            operand_layout(X)
        Y = _as_operand(X)
        assert Y.is_contiguous() and torch.equal(Y, X)
        assert operand_layout(Y) == ("N", max(X.shape[1], 1))
    # overlapping rows (row stride below the row length) are refused too
    with pytest.raises(ValueError):
        operand_layout(torch.empty(20).as_strided((4, 6), (3, 1)))
    # single rows and columns of real storage keep a valid ld
    assert operand_layout(torch.empty(6, 1)) == ("N", 1)
    assert operand_layout(torch.empty(1, 6)) == ("N", 6)
    assert operand_layout(torch.empty(6, 1).t()) == ("N", 6)
    assert operand_layout(torch.empty(3, 8)[:, :1]) == ("N", 8)


def test_output_ld_refuses_overlapping_rows():
    from paper_2305_18236_amd import output_ld
    assert output_ld(torch.empty(5, 7)) == 7
    assert output_ld(torch.empty(5, 12)[:, :7]) == 12
    assert output_ld(torch.empty(1, 7)) == 7
    with pytest.raises(ValueError):
        output_ld(torch.zeros(1, 7).expand(5, 7))
    with pytest.raises(ValueError):
        output_ld(torch.zeros(5, 1).expand(5, 7))


def _syr2k(native, **kw):
    a = dict(path=0, uplo="L", trans="N", N=4, K=6, alpha=1.0, A=FAKE, lda=6, B=FAKE, ldb=6, beta=0.0,
             C=FAKE, ldc=4)
    a.update(kw)
    return native.mg_syr2k(a["path"], a["uplo"], a["trans"], a["N"], a["K"], a["alpha"], a["A"], a["lda"],
                           a["B"], a["ldb"], a["beta"], a["C"], a["ldc"], None, 0, None)


@pytest.mark.parametrize("kw,code", [
    (dict(uplo="X"), -1), (dict(trans="Q"), -2), (dict(N=-1), -3), (dict(K=-2), -4), (dict(A=None), -6),
    (dict(lda=5), -7), (dict(B=None), -8), (dict(ldb=5), -9), (dict(C=None), -11), (dict(ldc=3), -12),
    # trans 'T': A and B are K x N, so lda, ldb >= N
    (dict(trans="T", lda=3), -7), (dict(trans="T", lda=4, ldb=3), -9),
    (dict(path=1), -101), (dict(path=3), -101),
])
def test_syr2k_arguments_rejected_on_host(native, kw, code):
    assert _syr2k(native, **kw) == code


def test_syr2k_empty_is_noop(native):
    assert _syr2k(native, N=0, A=None, B=None, C=None) == 0


def test_syr2k_split_plan(native):
    """A triangle that does not fill whole rounds of the GPU splits its tiles'
    K loops (when a workspace is given); forced splits are honoured."""
    assert native.mg_syr2k_workspace_size(0, 8192, 8192) > 0
    assert native.mg_syr2k_workspace_size(1, 8192, 8192) == 0
    try:
        assert native.mg_force_splits(0, 1) == 0
        assert native.mg_syr2k_workspace_size(0, 8192, 8192) == 0
        assert native.mg_force_splits(0, 4) == 0
        assert native.mg_syr2k_workspace_size(0, 100, 1000) == 4 * 100 * 100 * 4
    finally:
        native.mg_force_splits(0, -1)


def test_syr2k_plan_tiles(native):
    """The square tile SYR2K runs: 256 x 256 once that triangle fills four
    rounds of the compute units, the eight-wave 128 x 128 tile below that,
    64 x 64 for triangles under half a round of 128 x 128 tiles; the split
    reported is the one the workspace size is made for."""
    cus = 256   # no device here: the library plans for a full MI355X
    tri = lambda n, b: ((n + b - 1) // b) * ((n + b - 1) // b + 1) // 2
    for n, k in [(16384, 8192), (12288, 4096), (8192, 8192), (4096, 4096), (2816, 1024), (2048, 2048),
                 (1024, 1024), (100, 1000)]:
        st, cfg, splits = native.mg_syr2k_plan(0, n, k)
        assert st == 0
        want = 5 if tri(n, 256) >= 4 * cus else 18 if 2 * tri(n, 128) >= cus else 3
        assert cfg == want, (n, k)
        ws = native.mg_syr2k_workspace_size(0, n, k)
        assert (splits > 1) == (ws > 0)
        if splits > 1:
            assert ws >= splits * n * n * 4
    assert native.mg_syr2k_plan(0, 0, 5) == (0, -1, 0)
    assert native.mg_syr2k_plan(0, 5, 0) == (0, -1, 0)
    assert native.mg_syr2k_plan(1, 64, 64)[0] == -101   # MG_ERR_UNSUPPORTED
    assert native.mg_syr2k_plan(0, -1, 64)[0] == -3
    assert native.mg_syr2k_plan(0, 64, -1)[0] == -4
    try:
        assert native.mg_force_config(0, 18) == 0
        assert native.mg_syr2k_plan(0, 100, 100)[1] == 18
        assert native.mg_force_config(0, 2) == 0   # 256 x 128 is not square
        assert native.mg_syr2k_plan(0, 100, 100)[0] == -101
    finally:
        native.mg_force_config(0, -1)


def test_library_shares_torchs_hip_runtime():
    """Loading the library before anything else imports torch must not bring
    a second HIP runtime into the process (torch's and the system's share a
    soname, and the first one loaded serves both)."""
    import subprocess
    import sys
    code = ("import os, sys; sys.path.insert(0, %r)\n"
            "from paper_2305_18236_amd import _native\n"
            "_native.lib()\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "libs = {l.split()[-1] for l in maps if 'libamdhip64' in l}\n"
            "assert len(libs) == 1, libs\n"
            "assert next(iter(libs)).startswith(os.path.dirname(torch.__file__)), libs\n") % ROOT
    subprocess.run([sys.executable, "-c", code], check=True, timeout=300)


def test_queries_on_empty_and_huge_shapes(native):
    """Configuration and size queries stay defined at the edges: no tiles
    (M or N = 0) and dimensions beyond what any compute entry point takes."""
    for path in (0, 1, 2, 3, 4):
        assert 0 <= native.mg_tuned_config(path, 0, 5, 5) < native.mg_num_configs(path)
        assert 0 <= native.mg_tuned_config(path, 5, 0, 5) < native.mg_num_configs(path)
        assert native.mg_tuned_config(path, 2 ** 31, 5, 5) == -102
        assert native.mg_split_count(path, 2 ** 62, 2 ** 62, 2 ** 62) == 1
        assert native.mg_gemm_workspace_size(path, "N", "N", 2 ** 63 - 1, 8, 8) == 0
    assert native.mg_batched_config(0, 0, 0, 0) >= 0
    assert native.mg_batched_config(0, 8, 8, 2 ** 40) == -102
    assert native.mg_gemm_i8_workspace_size(2 ** 40, 8, 8) == 0
    assert native.mg_syr2k_workspace_size(0, 2 ** 40, 8) == 0
    with pytest.raises(native.MgemmError):
        native.mg_fp8_packed_size(2 ** 40, 128)
    with pytest.raises(native.MgemmError):
        native.mg_i8_packed_size(128, 2 ** 40)


def test_fp8_k_limit_is_checked_on_the_host(native):
    """The FP8 GEMM kernels address a 256-row panel with 32-bit offsets, so
    K above 2^23 is refused before any device call (the pointers here are
    never dereferenced), and the workspace query answers 0 there."""
    fake, K = 0x1000, 2 ** 23 + 1
    assert native.mg_gemm_workspace_size(3, "N", "N", 8, 8, K) == 0
    assert native.mg_gemm_workspace_size(3, "N", "N", 8, 8, K - 1) > 0
    assert native.mg_gemm(3, "N", "N", 8, 8, K, 1.0, fake, K, fake, 8, 0.0, fake, 8, fake, 1 << 40, None) == -102
    assert native.mg_gemm_fp8_packed(8, 8, K, 1.0, fake, fake, fake, fake, 0.0, fake, 8, None) == -102
