"""GPU parity of split-K launches (K cut into ranges multiplied by separate
workgroups, partial products summed by a reduction kernel) against the FP64
oracle, through the C ABI, on every path that splits."""
import itertools

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from helpers import PATH_ID, Problem, TOL

pytestmark = pytest.mark.gpu

LAYOUTS = list(itertools.product("NT", "NT"))


@pytest.fixture()
def nat():
    from paper_2305_18236_amd import _native
    _native.lib()
    yield _native
    for p in range(4):
        _native.mg_force_splits(p, -1)
        _native.mg_force_config(p, -1)


def _run(p, dev, path, nat, splits=None, cfg=None, expect_split=True):
    pid = PATH_ID[path]
    if splits is not None:
        assert nat.mg_force_splits(pid, splits) == 0
    if cfg is not None:
        assert nat.mg_force_config(pid, cfg) == 0
    if expect_split:
        assert nat.mg_split_count(pid, p.M, p.N, p.K) > 1
    p.to_device(dev)
    st = p.run(path)
    assert st == 0, nat.status_string(st)
    return p.result()


@pytest.mark.parametrize("tA,tB", LAYOUTS)
@pytest.mark.parametrize("splits", [2, 3, 5, 16])
def test_fp32_forced_splits_all_layouts(gpu, nat, tA, tB, splits):
    """Ragged M, N and K (the last K range is short), ldc with padding and not
    a multiple of 4 (scalar path of the reduction)."""
    p = Problem(150, 270, 2100 if splits == 16 else 1100, tA, tB, -1.25, 0.75,
                seed=300 + splits + ord(tA) + 2 * ord(tB), ldc=273)
    C = _run(p, gpu, "fp32", nat, splits=splits, cfg=0)
    Cref, D = p.oracle()
    assert oracle.normalized_error(C, Cref, D) <= TOL["fp32"]
    assert p.padding_untouched()


@pytest.mark.parametrize("cfg", [0, 3, 5])
def test_fp32_split_every_tile_shape(gpu, nat, cfg):
    p = Problem(300, 260, 777, "N", "N", 1.5, 0.5, seed=310 + cfg)
    C = _run(p, gpu, "fp32", nat, splits=4, cfg=cfg)
    Cref, D = p.oracle()
    assert oracle.normalized_error(C, Cref, D) <= TOL["fp32"]


@pytest.mark.parametrize("path", ["bf16x3", "bf16"])
@pytest.mark.parametrize("tA,tB", LAYOUTS)
def test_bf16_paths_forced_splits(gpu, nat, path, tA, tB):
    p = Problem(200, 136, 1000, tA, tB, 1.5, 0.5, seed=320 + ord(tA) + ord(tB))
    C = _run(p, gpu, path, nat, splits=3)
    Cref, D = p.oracle()
    assert oracle.normalized_error(C, Cref, D) <= TOL[path]


def test_bf16_prepacked_planes_split(gpu, nat):
    """Plain BF16 with M, N >= 512 multiplies pre-packed planes; the split
    offsets the packed rows along K."""
    p = Problem(520, 600, 1500, "T", "N", 1.0, 0.5, seed=330)
    C = _run(p, gpu, "bf16", nat, splits=4, cfg=2)
    Cref, D = p.oracle()
    assert oracle.normalized_error(C, Cref, D) <= TOL["bf16"]


@pytest.mark.parametrize("path", ["fp32", "bf16x3"])
def test_automatic_split_on_few_tiles(gpu, nat, path):
    """Few output tiles and a long K: the automatic rule splits."""
    p = Problem(256, 512, 4096, "N", "N", 1.5, 0.5, seed=340)
    C = _run(p, gpu, path, nat)
    Cref, D = p.oracle()
    assert oracle.normalized_error(C, Cref, D) <= TOL[path]


def test_integer_inputs_bit_exact_under_split(gpu, nat):
    """Integer partial sums are exact, so the split result is the exact one."""
    p = Problem(190, 210, 1200, "N", "T", 1.5, 0.5, seed=350, dist="integers")
    C = _run(p, gpu, "fp32", nat, splits=5)
    Cref, _ = p.oracle()
    assert np.array_equal(C, Cref)


def test_split_deterministic_bitwise(gpu, nat):
    p = Problem(256, 384, 3000, "N", "N", 1.5, 0.5, seed=360)
    outs = []
    for _ in range(3):
        outs.append(_run(p, gpu, "fp32", nat, splits=6))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])


def test_beta_zero_split_never_reads_c(gpu, nat):
    p = Problem(100, 130, 900, "N", "N", 1.0, 0.0, seed=370, c0_nan=True)
    C = _run(p, gpu, "fp32", nat, splits=3)
    assert not np.isnan(C).any()
    Cref, D = oracle.gemm("N", "N", 100, 130, 900, 1.0, p.A, p.lda, p.B, p.ldb)
    assert oracle.normalized_error(C, Cref, D) <= TOL["fp32"]


def test_short_workspace_runs_unsplit(gpu, nat):
    """Too little workspace: the GEMM runs without the split, same contract."""
    import torch
    from paper_2305_18236_amd import _native
    p = Problem(128, 128, 2048, "N", "N", 1.5, 0.5, seed=380).to_device(gpu)
    assert nat.mg_force_splits(0, 4) == 0
    need = _native.mg_gemm_workspace_size(0, "N", "N", 128, 128, 2048)
    assert need >= 4 * 128 * 128 * 4
    ws = torch.empty(need - 256, dtype=torch.uint8, device=gpu)
    stream = torch.cuda.current_stream().cuda_stream
    st = _native.mg_gemm(0, "N", "N", 128, 128, 2048, 1.5, p.dA.data_ptr(), p.lda, p.dB.data_ptr(), p.ldb,
                         0.5, p.dC.data_ptr(), p.ldc, ws.data_ptr(), ws.numel(), stream)
    assert st == 0
    Cref, D = p.oracle()
    assert oracle.normalized_error(p.result(), Cref, D) <= TOL["fp32"]
    # mg_sgemm takes no workspace: never splits
    p.reset_c()
    assert _native.mg_sgemm("N", "N", 128, 128, 2048, 1.5, p.dA.data_ptr(), p.lda, p.dB.data_ptr(), p.ldb,
                            0.5, p.dC.data_ptr(), p.ldc, stream) == 0
    assert oracle.normalized_error(p.result(), Cref, D) <= TOL["fp32"]


@pytest.mark.slow
@pytest.mark.parametrize("path", ["fp32", "bf16x3"])
def test_full_size_skinny_m_sampled(gpu, nat, path):
    """256 x 8192 x 8192, the sweep shape the split exists for, in the launch
    the automatic rule picks; 2048 sampled outputs against the oracle."""
    p = Problem(256, 8192, 8192, "N", "N", 1.5, 0.5, seed=1006)
    C = _run(p, gpu, path, nat)
    I, J = si.sample_indices(256, 8192, 2048, 98)
    cref, d = p.oracle_entries(I, J)
    assert oracle.normalized_error(C[I, J], cref, d) <= TOL[path]
    assert np.isfinite(C).all()
