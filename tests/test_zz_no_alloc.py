"""The allocation-free GEMM entry point (mg_gemm_noalloc), through the C ABI:
its results equal mg_gemm's with a caller workspace of the same size as the
library's fixed scratch, bit for bit (same plan, same kernels), and meet the
oracle bar; two calls in a row, the second smaller, so the second runs on
what the first left in the scratch.  FP8 problems whose packed operands
exceed the scratch are refused on the host."""
import os
import re

import numpy as np
import pytest

import oracle
from helpers import PATH_ID, Problem, tolerance

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def scratch_bytes() -> int:
    """MG_NOALLOC_SCRATCH_BYTES as the public header defines it."""
    text = open(os.path.join(ROOT, "include", "mgemm.h")).read()
    m = re.search(r"#define MG_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m, "MG_NOALLOC_SCRATCH_BYTES not found in the header"
    return int(m.group(1)) << int(m.group(2))


def _native():
    from paper_2305_18236_amd import _native
    _native.lib()
    return _native


def _noalloc(nat, p, path, stream):
    return nat.mg_gemm_noalloc(PATH_ID[path], p.tA, p.tB, p.M, p.N, p.K, p.alpha, p.dA.data_ptr(), p.lda,
                               p.dB.data_ptr(), p.ldb, p.beta, p.dC.data_ptr(), p.ldc, stream)


# per path: a first problem that uses the scratch (split-K partials, pre-packed
# planes or FP8 packs), then a smaller ragged one
CASES = {
    "fp32": [(256, 320, 8192, "N", "T"), (96, 80, 1000, "T", "N")],
    "bf16x3": [(2048, 2048, 512, "N", "N"), (300, 257, 700, "T", "T")],
    "bf16": [(1024, 1024, 1024, "T", "N"), (513, 600, 129, "N", "T")],
    "fp16": [(768, 1024, 2048, "N", "N"), (130, 70, 90, "T", "N")],
    "fp8": [(1024, 768, 2048, "N", "T"), (200, 130, 300, "T", "T")],
}


@pytest.mark.parametrize("path", list(CASES))
def test_noalloc_equals_mg_gemm_with_a_scratch_sized_workspace(gpu, path):
    import torch
    nat = _native()
    S = scratch_bytes()
    stream = torch.cuda.current_stream().cuda_stream
    ws = torch.empty(S, dtype=torch.uint8, device=gpu)
    uses_scratch = False
    for i, (M, N, K, tA, tB) in enumerate(CASES[path]):
        print(f"noalloc {path} call {i}: {M}x{N}x{K} {tA}{tB}", flush=True)
        p = Problem(M, N, K, tA, tB, 1.5, 0.5, seed=7100 + 10 * i + PATH_ID[path]).to_device(gpu)
        st, cfg, splits, packed = nat.mg_gemm_plan(PATH_ID[path], M, N, K, S)
        assert st == 0
        uses_scratch |= splits > 1 or packed == 1
        st = nat.mg_gemm(PATH_ID[path], p.tA, p.tB, M, N, K, p.alpha, p.dA.data_ptr(), p.lda, p.dB.data_ptr(),
                         p.ldb, p.beta, p.dC.data_ptr(), p.ldc, ws.data_ptr(), S, stream)
        assert st == 0, nat.status_string(st)
        ref = p.result()
        p.reset_c()
        st = _noalloc(nat, p, path, stream)
        assert st == 0, nat.status_string(st)
        got = p.result()
        assert np.array_equal(got, ref), (path, i)
        assert p.padding_untouched()
        Cref, D = p.oracle()
        err = oracle.normalized_error(got, Cref, D)
        assert err <= tolerance(path, K), (path, i, err)
    assert uses_scratch, path


def test_noalloc_quick_returns_and_argument_codes(gpu):
    import torch
    nat = _native()
    stream = torch.cuda.current_stream().cuda_stream
    C = torch.full((4, 5), 3.0, device=gpu)
    A = torch.ones((4, 6), device=gpu)
    B = torch.ones((6, 5), device=gpu)
    # alpha = 0: C <- beta*C without touching A, B or the scratch
    assert nat.mg_gemm_noalloc(0, "N", "N", 4, 5, 6, 0.0, A.data_ptr(), 6, B.data_ptr(), 5, 0.5,
                               C.data_ptr(), 5, stream) == 0
    torch.cuda.synchronize()
    assert torch.equal(C, torch.full((4, 5), 1.5, device=gpu))
    # argument errors as mg_gemm, before any device work
    assert nat.mg_gemm_noalloc(0, "X", "N", 4, 5, 6, 1.0, A.data_ptr(), 6, B.data_ptr(), 5, 0.0,
                               C.data_ptr(), 5, stream) == -1
    assert nat.mg_gemm_noalloc(0, "N", "N", 4, 5, 6, 1.0, A.data_ptr(), 5, B.data_ptr(), 5, 0.0,
                               C.data_ptr(), 5, stream) == -8
    assert nat.mg_gemm_noalloc(9, "N", "N", 4, 5, 6, 1.0, A.data_ptr(), 6, B.data_ptr(), 5, 0.0,
                               C.data_ptr(), 5, stream) == -101


def test_noalloc_fp8_beyond_the_scratch_is_refused():
    """16384 x 16384 x 8192 in FP8 needs 256 MiB of packed operands plus their
    scales: more than the scratch, refused on the host (the pointers are never
    dereferenced)."""
    nat = _native()
    fake = 0x1000
    n, k = 16384, 8192
    assert nat.mg_gemm_workspace_size(3, "N", "N", n, n, k) > scratch_bytes()
    assert nat.mg_gemm_noalloc(3, "N", "N", n, n, k, 1.0, fake, k, fake, n, 0.0, fake, n, None) == -104
    assert nat.status_string(-104) != "unknown status"
