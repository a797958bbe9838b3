"""GPU parity of the FP32-MFMA path against the FP64 oracle, through the C ABI.

Bar: normalised error max|C - C_ref| / (|alpha||A||B| + |beta||C0|) <= 1e-5,
and bit-exact results where the inputs make the exact result representable
(integer-valued operands).
"""
import itertools

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from helpers import Problem, TOL

pytestmark = pytest.mark.gpu

LAYOUTS = list(itertools.product("NT", "NT"))


def _native():
    from paper_2305_18236_amd import _native
    return _native


def _check(p, dev, path="fp32", tol=None, cfg=None):
    nat = _native()
    if cfg is not None:
        assert nat.mg_force_config(0, cfg) == 0
    try:
        p.to_device(dev)
        st = p.run(path)
        assert st == 0, nat.status_string(st)
        C = p.result()
    finally:
        nat.mg_force_config(0, -1)
    Cref, D = p.oracle()
    err = oracle.normalized_error(C, Cref, D)
    assert err <= (TOL[path] if tol is None else tol), (p.M, p.N, p.K, p.tA, p.tB, err)
    assert p.padding_untouched()
    return C, Cref, err


def test_config1_256_cube_nn(gpu):
    """M = N = K = 256, NN, alpha = 1, beta = 0, U[-1, 1]."""
    p = Problem(256, 256, 256, "N", "N", 1.0, 0.0, seed=1000)
    _check(p, gpu)


@pytest.mark.parametrize("tA,tB", LAYOUTS)
@pytest.mark.parametrize("M,N,K", [(300, 517, 129), (1, 1, 1), (7, 9, 8), (33, 65, 31),
                                   (129, 257, 64), (64, 64, 1000), (5, 300, 3)])
def test_ragged_shapes_all_layouts(gpu, tA, tB, M, N, K):
    p = Problem(M, N, K, tA, tB, 1.5, 0.5, seed=M + 7 * N + 13 * K)
    _check(p, gpu)


@pytest.mark.parametrize("cfg", list(range(21)))
@pytest.mark.parametrize("tA,tB", LAYOUTS)
def test_every_config_every_layout(gpu, cfg, tA, tB):
    """Each tile configuration over several tiles and a ragged tail (8 and 9
    without packing, 10 and 11 with the vector-ALU micro-kernel)."""
    p = Problem(530, 390, 77, tA, tB, -1.25, 0.75, seed=cfg * 4 + ord(tA) + ord(tB))
    _check(p, gpu, cfg=cfg)


@pytest.mark.parametrize("deep,single", [(12, 3), (13, 4), (14, 0), (17, 5), (18, 0), (19, 0), (20, 4)])
@pytest.mark.parametrize("tA,tB", LAYOUTS)
def test_two_staging_sets_bit_identical(gpu, deep, single, tA, tB):
    """Configurations 12-14 and 17 are 3, 4, 0 and 5 with each panel fetched a panel
    earlier into a second register staging set: the same products in the
    same order, so the same bits (odd and even panel counts, ragged edges).
    18 and 19 split configuration 0's 128 x 128 tile over eight waves
    instead of four, and 20 configuration 4's 128 x 64 tile; each output
    still accumulates its k in the same order, so they match bit for bit
    too."""
    for K in (77, 160, 1000):
        C1, _, _ = _check(Problem(300, 260, K, tA, tB, 1.5, 0.5, seed=K + deep), gpu, cfg=single)
        C2, _, _ = _check(Problem(300, 260, K, tA, tB, 1.5, 0.5, seed=K + deep), gpu, cfg=deep)
        assert np.array_equal(C1, C2), (deep, K, tA, tB)


@pytest.mark.parametrize("cfg", [15, 16])
@pytest.mark.parametrize("K", [1, 32, 33, 64, 96, 1000])
def test_k_groups_every_panel_count(gpu, cfg, K):
    """Two K groups of waves per workgroup (each every other 32-deep panel,
    sums added through LDS): one panel (the second group idles), two, three
    and many, ragged K."""
    _check(Problem(300, 260, K, "N", "T", 1.5, 0.5, seed=K + 7 * cfg), gpu, cfg=cfg)


@pytest.mark.parametrize("cfg", [15, 16])
def test_k_groups_integer_bit_exact(gpu, cfg):
    """Integer inputs: every partial sum is exact, so the two groups' sums
    and their addition give the exact result."""
    C, Cref, _ = _check(Problem(330, 270, 250, "T", "N", 1.5, 0.5, seed=3 + cfg, dist="integers"), gpu, cfg=cfg)
    assert np.array_equal(C, Cref)


@pytest.mark.parametrize("tA,tB", LAYOUTS)
def test_integer_inputs_bit_exact(gpu, tA, tB):
    """Integers in [-8, 8]: partial sums stay below 2^24, so the exact result
    is representable and any summation order gives it."""
    p = Problem(200, 300, 250, tA, tB, 1.5, 0.5, seed=77, dist="integers")
    C, Cref, _ = _check(p, gpu)
    assert np.array_equal(C, Cref)


def test_padded_leading_dimensions_and_misaligned(gpu):
    """lda/ldb/ldc above the minimum and not multiples of 4 (scalar paths)."""
    p = Problem(70, 45, 33, "T", "N", 1.0, 0.5, seed=5, lda=71, ldb=47, ldc=49)
    _check(p, gpu)
    p = Problem(70, 45, 33, "N", "T", 1.0, 0.5, seed=6, lda=36, ldb=40, ldc=48)
    _check(p, gpu)


def test_beta_zero_never_reads_c(gpu):
    p = Problem(100, 130, 40, "N", "N", 1.0, 0.0, seed=8, c0_nan=True)
    p.to_device(gpu)
    assert p.run() == 0
    C = p.result()
    assert not np.isnan(C).any()
    Cref, D = oracle.gemm("N", "N", 100, 130, 40, 1.0, p.A, p.lda, p.B, p.ldb)
    assert oracle.normalized_error(C, Cref, D) <= TOL["fp32"]


def test_alpha_zero_and_k_zero_scale_c(gpu):
    p = Problem(50, 60, 20, "N", "N", 0.0, 0.5, seed=9)
    p.opA[:] = np.nan   # alpha == 0: A must not be read
    p.A[:] = np.nan
    p.to_device(gpu)
    assert p.run() == 0
    assert np.array_equal(p.result(), 0.5 * p.C0.astype(np.float64))
    # beta == 0 with NaN C: zeros
    q = Problem(50, 60, 20, "N", "N", 0.0, 0.0, seed=10, c0_nan=True)
    q.to_device(gpu)
    assert q.run() == 0
    assert np.array_equal(q.result(), np.zeros((50, 60)))
    # beta == 1: untouched
    r = Problem(50, 60, 20, "N", "N", 0.0, 1.0, seed=11)
    r.to_device(gpu)
    assert r.run() == 0
    assert np.array_equal(r.result(), r.C0.astype(np.float64))


def test_m_or_n_zero_touches_nothing(gpu):
    p = Problem(0, 5, 7, seed=12)
    p.to_device(gpu)
    assert p.run() == 0


def test_layouts_bitwise_identical(gpu):
    """Packing hands the micro-kernel the same panels for every stored layout,
    so NN/NT/TN/TT of the same logical operands give identical bits."""
    outs = []
    for tA, tB in LAYOUTS:
        p = Problem(333, 290, 300, tA, tB, 1.5, 0.5, seed=21).to_device(gpu)
        assert p.run() == 0
        outs.append(p.result())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_deterministic_bitwise(gpu):
    """No atomics in the reduction: repeated runs give identical bits; a
    missing barrier or an LDS race would show up here."""
    p = Problem(1000, 900, 700, "N", "N", 1.5, 0.5, seed=13).to_device(gpu)
    outs = []
    for _ in range(3):
        p.reset_c()
        assert p.run() == 0
        outs.append(p.result())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])


@pytest.mark.slow
@pytest.mark.parametrize("tA,tB", LAYOUTS)
def test_full_size_8192_sampled(gpu, tA, tB):
    """The benchmark's launch: 8192^3, alpha 1.5, beta 0.5, in every layout;
    4096 sampled outputs (corners included) against the oracle."""
    p = Problem(8192, 8192, 8192, tA, tB, 1.5, 0.5, seed=1001).to_device(gpu)
    assert p.run() == 0
    C = p.result()
    I, J = si.sample_indices(8192, 8192, 4096, 99)
    cref, d = p.oracle_entries(I, J)
    err = oracle.normalized_error(C[I, J], cref, d)
    assert err <= TOL["fp32"], err
    assert np.isfinite(C).all()


@pytest.mark.parametrize("cfg", [8, 9])
@pytest.mark.parametrize("tA,tB", LAYOUTS)
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (16, 16, 16), (33, 70, 13), (64, 64, 8), (130, 129, 100),
                                   (5, 300, 3)])
def test_unpacked_tiling_small_shapes(gpu, cfg, tA, tB, M, N, K):
    """The no-packing configurations on the small shapes they are for: K not a
    multiple of the 8-deep chunk, partial tiles in M and N."""
    p = Problem(M, N, K, tA, tB, 1.5, 0.5, seed=M * 3 + N * 5 + K + cfg)
    _check(p, gpu, cfg=cfg)


@pytest.mark.parametrize("cfg", [8, 9])
def test_unpacked_tiling_unaligned_and_exact(gpu, cfg):
    """Leading dimensions that rule out 16-byte loads, and integer inputs for
    which the result is exact."""
    p = Problem(70, 45, 37, "N", "T", 1.0, 0.5, seed=40 + cfg, lda=39, ldb=41, ldc=47)
    _check(p, gpu, cfg=cfg)
    q = Problem(150, 170, 200, "N", "N", 1.5, 0.5, seed=42 + cfg, dist="integers")
    C, Cref, _ = _check(q, gpu, cfg=cfg)
    assert np.array_equal(C, Cref)


def test_packed_and_unpacked_agree(gpu):
    """Tiling and Tiling+Packing compute the same product (up to rounding
    order) on every layout."""
    for tA, tB in LAYOUTS:
        p = Problem(200, 180, 300, tA, tB, 1.0, 0.0, seed=44)
        C8, Cref, _ = _check(p, gpu, cfg=8)
        C0, _, _ = _check(p, gpu, cfg=0)
        assert np.max(np.abs(C8 - C0)) <= 2e-5 * np.max(np.abs(Cref))


@pytest.mark.parametrize("cfg", [10, 11])
def test_valu_microkernel_exact_and_unaligned(gpu, cfg):
    """The vector-ALU micro-kernel: integer inputs give the exact result; odd
    leading dimensions take the scalar load and store paths."""
    q = Problem(257, 130, 300, "T", "N", 1.5, 0.5, seed=50 + cfg, dist="integers")
    C, Cref, _ = _check(q, gpu, cfg=cfg)
    assert np.array_equal(C, Cref)
    p = Problem(70, 45, 33, "N", "T", 1.0, 0.5, seed=52 + cfg, lda=35, ldb=37, ldc=47)
    _check(p, gpu, cfg=cfg)


@pytest.mark.slow
def test_valu_full_size_sampled(gpu):
    """8192^3 on the vector-ALU micro-kernel, as the engine comparison runs it."""
    nat = _native()
    assert nat.mg_force_config(0, 10) == 0
    try:
        p = Problem(8192, 8192, 8192, "N", "N", 1.5, 0.5, seed=1001).to_device(gpu)
        assert p.run() == 0
        C = p.result()
    finally:
        nat.mg_force_config(0, -1)
    I, J = si.sample_indices(8192, 8192, 2048, 97)
    cref, d = p.oracle_entries(I, J)
    assert oracle.normalized_error(C[I, J], cref, d) <= TOL["fp32"]
