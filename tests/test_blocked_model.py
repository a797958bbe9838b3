"""A CPU model of the layered algorithm as the library's kernels carry it out
(Algorithm 1 of Kuzma et al., SPE 2023, with the micro-kernel of
Algorithm 2 on 32 x 32 matrix-core blocks), checked against the oracle.

The model reads the stored operands (either layout, any leading dimension,
NaN in every padding entry), cuts C into BM x BN workgroup tiles, walks K in
BK-deep panels, packs each op(A) / op(B) panel with zeros outside the matrix
on BOTH operands (Section 3.1's remainder rule; one-sided padding would turn
0 * NaN into NaN), splits each workgroup tile into WM x WN wave tiles of
32 x 32 accumulator blocks updated kr = 2 at a time (the FP32 instruction's
depth), optionally cuts the K loop into split-K ranges summed in a fixed
order, and applies C = alpha*acc + beta*C0 once at the end, never reading C0
when beta = 0.  The tile shapes are the library's own configurations.

On integer-valued inputs every partial sum is exact in float64, so the model
must equal the oracle bit for bit whatever the blocking: any mistake in
panel bounds, remainders, transposition or the epilogue shows.  This pins
the decomposition on the CPU; the GPU parity tests pin the kernels.
"""
import math

import numpy as np
import pytest

import oracle
import seeded_inputs as si


def logical(buf, trans, rows, cols, ld):
    """The logical rows x cols operand from its stored form (reads only the
    entries that belong to it)."""
    if trans == "N":
        return np.stack([buf[r * ld: r * ld + cols] for r in range(rows)]) if rows else np.zeros((0, cols))
    stored = np.stack([buf[c * ld: c * ld + rows] for c in range(cols)]) if cols else np.zeros((0, rows))
    return stored.T


SPLIT_GRAIN = 128   # K ranges of a split are whole multiples of this (every BK divides it)


def split_ranges(K, splits):
    """The K ranges of a split-K launch, as the library cuts them: a range
    length of ceil(K / splits) rounded up to a multiple of 128, so the last
    range is the remainder and fewer than `splits` ranges can result."""
    if splits < 2:
        return [(0, K)]
    chunk = -(-(-(-K // splits)) // SPLIT_GRAIN) * SPLIT_GRAIN
    return [(k0, min(K, k0 + chunk)) for k0 in range(0, K, chunk)]


def layered_gemm(tA, tB, M, N, K, alpha, A, lda, B, ldb, beta, C0, cfg, splits=1, partials_out=None):
    """Algorithm 1's loops as the GPU runs them; returns C (M x N, float64).
    partials_out (a list), if given, receives each K range's unscaled M x N
    partial product."""
    BM, BN, BK, WM, WN = cfg
    opA = logical(np.asarray(A, np.float64), tA, M, K, lda)
    opB = logical(np.asarray(B, np.float64), tB, K, N, ldb)
    ranges = split_ranges(K, splits)
    C = np.zeros((M, N))
    full = [np.zeros((M, N)) for _ in ranges]
    for tm in range(math.ceil(M / BM)):
        for tn in range(math.ceil(N / BN)):
            m0, n0 = tm * BM, tn * BN
            partials = []
            for r, (ks, ke) in enumerate(ranges):
                acc = np.zeros((BM, BN))
                for k0 in range(ks, ke, BK):
                    # pack both panels, zero outside the matrix
                    Ap = np.zeros((BM, BK))
                    Bp = np.zeros((BK, BN))
                    mr, kr_, nr = min(BM, M - m0), min(BK, ke - k0), min(BN, N - n0)
                    Ap[:mr, :kr_] = opA[m0:m0 + mr, k0:k0 + kr_]
                    Bp[:kr_, :nr] = opB[k0:k0 + kr_, n0:n0 + nr]
                    # wave tiles, 32 x 32 accumulator blocks, rank-2 updates
                    for wm in range(0, BM, WM):
                        for wn in range(0, BN, WN):
                            for i in range(wm, wm + WM, 32):
                                for j in range(wn, wn + WN, 32):
                                    for k in range(0, BK, 2):
                                        acc[i:i + 32, j:j + 32] += Ap[i:i + 32, k:k + 2] @ Bp[k:k + 2, j:j + 32]
                partials.append(acc)
                mr, nr = min(BM, M - m0), min(BN, N - n0)
                full[r][m0:m0 + mr, n0:n0 + nr] = acc[:mr, :nr]
            total = partials[0]
            for p in partials[1:]:      # fixed order, as the reduction kernel sums them
                total = total + p
            mr, nr = min(BM, M - m0), min(BN, N - n0)
            out = alpha * total[:mr, :nr]
            if beta != 0.0:
                out = out + beta * C0[m0:m0 + mr, n0:n0 + nr]
            C[m0:m0 + mr, n0:n0 + nr] = out
    if partials_out is not None:
        partials_out.extend(full)
    return C


@pytest.fixture(scope="module")
def configs():
    from paper_2305_18236_amd import _native
    _native.lib()
    out = {}
    for i in range(_native.mg_num_configs(0)):
        c = _native.mg_config_info(0, i)
        if _native.mg_config_uses_mfma(0, i):
            out[c["id"]] = (c["bm"], c["bn"], c["bk"], c["wm"], c["wn"])
    return out


CASES = [
    # (M, N, K, tA, tB, pad) -- ragged against every tile size, both layouts, padded ld
    (1, 1, 1, "N", "N", 0), (7, 9, 5, "T", "N", 3), (33, 65, 17, "N", "T", 0),
    (70, 40, 37, "T", "T", 5), (130, 67, 49, "N", "N", 1), (64, 64, 64, "T", "N", 0),
    (5, 300, 33, "N", "T", 2),
]


@pytest.mark.parametrize("M,N,K,tA,tB,pad", CASES)
@pytest.mark.parametrize("cfg_id", [0, 3, 4, 5])
def test_model_equals_oracle_on_integer_inputs(configs, cfg_id, M, N, K, tA, tB, pad):
    cfg = configs[cfg_id]
    seed = 7000 + M + 3 * N + 7 * K
    a = si.integers((M, K), seed)
    b = si.integers((K, N), seed + 1)
    c0 = si.integers((M, N), seed + 2)
    A, lda = si.store(a, tA, (M if tA == "T" else K) + pad)
    B, ldb = si.store(b, tB, (K if tB == "T" else N) + pad)
    for alpha, beta in [(1.0, 0.0), (1.5, 0.5), (-2.0, 1.0)]:
        ref, _ = oracle.gemm(tA, tB, M, N, K, alpha, A, lda, B, ldb, beta, c0, N)
        got = layered_gemm(tA, tB, M, N, K, alpha, A, lda, B, ldb, beta, c0, cfg)
        assert np.array_equal(got, ref), (cfg, alpha, beta)


@pytest.mark.parametrize("K,splits,expect", [
    (333, 2, [(0, 256), (256, 333)]), (333, 3, [(0, 128), (128, 256), (256, 333)]),
    (333, 5, [(0, 128), (128, 256), (256, 333)]),
    (1000, 3, [(0, 384), (384, 768), (768, 1000)]), (1000, 4, [(0, 256), (256, 512), (512, 768), (768, 1000)]),
    (4096, 16, [(256 * i, 256 * i + 256) for i in range(16)]), (300, 7, [(0, 128), (128, 256), (256, 300)]),
])
def test_split_k_ranges(configs, K, splits, expect):
    """The model's K ranges are the library's: the count mg_split_count gives
    under a forced split, range starts on multiples of 128 (so every panel
    depth divides them), and each range's partial product equals the oracle's
    product over exactly that K slice, bit for bit (integer inputs)."""
    from paper_2305_18236_amd import _native
    ranges = split_ranges(K, splits)
    assert ranges == expect
    assert _native.mg_force_splits(0, splits) == 0
    try:
        assert _native.mg_split_count(0, 70, 45, K) == len(ranges)
    finally:
        _native.mg_force_splits(0, -1)
    M, N = 70, 45
    a = si.integers((M, K), 11)
    b = si.integers((K, N), 12)
    c0 = si.integers((M, N), 13)
    A, lda = si.store(a, "N")
    B, ldb = si.store(b, "T")
    parts = []
    got = layered_gemm("N", "T", M, N, K, 1.5, A, lda, B, ldb, 0.5, c0, configs[0], splits=splits,
                       partials_out=parts)
    ref, _ = oracle.gemm("N", "T", M, N, K, 1.5, A, lda, B, ldb, 0.5, c0, N)
    assert np.array_equal(got, ref)
    assert len(parts) == len(ranges)
    for (ks, ke), part in zip(ranges, parts):
        sa = np.ascontiguousarray(a[:, ks:ke])
        sb = np.ascontiguousarray(b[ks:ke, :])
        want, _ = oracle.gemm("N", "N", M, N, ke - ks, 1.0, sa, ke - ks, sb, N, 0.0, None, N)
        assert np.array_equal(part, want), (ks, ke)


def test_beta_zero_never_reads_c0_and_padding_never_read(configs):
    """NaN everywhere outside the operands (the stored padding) and in C0
    with beta = 0: the result must stay finite."""
    M, N, K = 37, 29, 41
    a = si.integers((M, K), 21)
    b = si.integers((K, N), 22)
    A, lda = si.store(a, "T", M + 7)
    B, ldb = si.store(b, "N", N + 3)
    c0 = np.full((M, N), np.nan)
    got = layered_gemm("T", "N", M, N, K, 1.0, A, lda, B, ldb, 0.0, c0, configs[4])
    ref, _ = oracle.gemm("T", "N", M, N, K, 1.0, A, lda, B, ldb, 0.0, None, N)
    assert np.isfinite(got).all() and np.array_equal(got, ref)


def test_one_sided_padding_would_fail(configs):
    """The reason both operands are zero-padded: with op(B)'s K padding
    filled with NaN instead of zeros, the zero-padded op(A) panel still
    multiplies it and the NaN reaches C."""
    BM, BN, BK, _, _ = configs[0]
    M, N, K = 5, 6, BK + 3                   # ragged last panel
    Ap = np.zeros((BM, BK))
    Bp = np.full((BK, BN), np.nan)
    Bp[:K - BK, :N] = 1.0                    # the real rows of the last panel
    acc = Ap @ Bp
    assert np.isnan(acc).any()
