"""GPU parity of SYR2K (Section 5.1's extension of the macro level) against the
FP64 oracle: the stored triangle within the FP32 bar (normalised error
<= 1e-5 with the SYR2K denominator), the other triangle untouched bit for bit."""
import itertools

import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si

pytestmark = pytest.mark.gpu
TOL = 1e-5
SENTINEL = -7.0


def _native():
    from paper_2305_18236_amd import _native
    return _native


def _run(dev, uplo, trans, N, K, alpha, beta, seed, dist="uniform", ldc=None, cfg=None, c0_nan=False,
         splits=None, use_workspace=True):
    gen = {"uniform": si.uniform, "integers": si.integers}[dist]
    X, Y = gen((N, K), seed), gen((N, K), seed + 1)
    A, B = (X, Y) if trans == "N" else (np.ascontiguousarray(X.T), np.ascontiguousarray(Y.T))
    ld = K if trans == "N" else N
    ldc = N if ldc is None else ldc
    C0 = np.full((N, N), np.nan, np.float32) if c0_nan else gen((N, N), seed + 2)
    Cbuf = np.full((max(N, 1), ldc), SENTINEL, np.float32)
    Cbuf[:N, :N] = C0
    # the triangle outside uplo holds sentinels too: it must come back unchanged
    outside = np.triu_indices(N, 1) if uplo == "L" else np.tril_indices(N, -1)
    Cbuf[outside] = SENTINEL
    nat = _native()
    dA = torch.from_numpy(A.reshape(-1).copy()).to(dev)
    dB = torch.from_numpy(B.reshape(-1).copy()).to(dev)
    dC = torch.from_numpy(Cbuf.reshape(-1).copy()).to(dev)
    if cfg is not None:
        assert nat.mg_force_config(0, cfg) == 0
    if splits is not None:
        assert nat.mg_force_splits(0, splits) == 0
    try:
        need = nat.mg_syr2k_workspace_size(0, N, K) if use_workspace else 0
        if splits is not None and splits > 1 and use_workspace:
            assert need > 0
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        st = nat.mg_syr2k(0, uplo, trans, N, K, alpha, dA.data_ptr(), ld, dB.data_ptr(), ld, beta, dC.data_ptr(),
                          ldc, ws.data_ptr(), need, torch.cuda.current_stream().cuda_stream)
    finally:
        nat.mg_force_config(0, -1)
        nat.mg_force_splits(0, -1)
    assert st == 0, nat.status_string(st)
    torch.cuda.synchronize()
    out = dC.cpu().numpy().reshape(max(N, 1), ldc)
    assert np.all(out[:N, N:] == SENTINEL)
    assert np.all(out[outside] == SENTINEL)
    ref, D = oracle.syr2k(uplo, trans, N, K, alpha, A, ld, B, ld, beta, np.where(np.isnan(Cbuf), 0, Cbuf)
                          if c0_nan else Cbuf, ldc)
    ref = ref.reshape(max(N, 1), ldc)[:N, :N]
    inside = np.tril_indices(N) if uplo == "L" else np.triu_indices(N)
    return out[:N, :N][inside].astype(np.float64), ref[inside], D[inside]


@pytest.mark.parametrize("uplo,trans", list(itertools.product("LU", "NT")))
@pytest.mark.parametrize("N,K", [(256, 256), (300, 129), (1, 1), (7, 8), (65, 31), (130, 500)])
def test_ragged_all_variants(gpu, uplo, trans, N, K):
    C, ref, D = _run(gpu, uplo, trans, N, K, 1.5, 0.5, seed=N + 3 * K)
    assert oracle.normalized_error(C, ref, D) <= TOL


@pytest.mark.parametrize("cfg", [0, 3, 5, 18])
@pytest.mark.parametrize("uplo,trans", list(itertools.product("LU", "NT")))
def test_every_square_config(gpu, cfg, uplo, trans):
    C, ref, D = _run(gpu, uplo, trans, 530, 77, -1.25, 0.75, seed=cfg + 7, ldc=533, cfg=cfg)
    assert oracle.normalized_error(C, ref, D) <= TOL


@pytest.mark.parametrize("splits", [1, 3])
@pytest.mark.parametrize("uplo,trans", [("L", "N"), ("U", "T")])
def test_eight_wave_tile_bit_identical(gpu, splits, uplo, trans):
    """The 128 x 128 tile over eight 64 x 32 waves (configuration 18) adds
    every entry's products in the same order as the four-wave tile
    (configuration 0): the results agree bit for bit."""
    a = _run(gpu, uplo, trans, 390, 203, 1.5, -0.5, seed=97, ldc=395, cfg=0, splits=splits)
    b = _run(gpu, uplo, trans, 390, 203, 1.5, -0.5, seed=97, ldc=395, cfg=18, splits=splits)
    assert np.array_equal(a[0], b[0])
    assert oracle.normalized_error(b[0], b[1], b[2]) <= TOL


def test_non_square_config_rejected(gpu):
    nat = _native()
    assert nat.mg_force_config(0, 2) == 0      # 256 x 128
    try:
        assert nat.mg_syr2k(0, "L", "N", 8, 8, 1.0, 0x1000, 8, 0x1000, 8, 0.0, 0x1000, 8, None, 0, None) == -101
    finally:
        nat.mg_force_config(0, -1)


@pytest.mark.parametrize("uplo,trans", list(itertools.product("LU", "NT")))
def test_integer_inputs_exact(gpu, uplo, trans):
    C, ref, _ = _run(gpu, uplo, trans, 200, 250, 1.5, 0.5, seed=21, dist="integers")
    assert np.array_equal(C, ref)


@pytest.mark.parametrize("cfg", [0, 18])
@pytest.mark.parametrize("splits", [2, 3, 7, 16])
@pytest.mark.parametrize("uplo,trans", list(itertools.product("LU", "NT")))
def test_split_k_loop(gpu, cfg, splits, uplo, trans):
    """Each tile's K loop (both products) cut into ranges whose partial tiles
    a reduction sums: ragged K, so a range can straddle the two products."""
    C, ref, D = _run(gpu, uplo, trans, 270, 333, 1.5, 0.5, seed=splits + 61, ldc=274, splits=splits, cfg=cfg)
    assert oracle.normalized_error(C, ref, D) <= TOL


def test_split_without_workspace_runs_unsplit(gpu):
    C, ref, D = _run(gpu, "L", "T", 200, 300, 1.0, 0.5, seed=71, splits=4, use_workspace=False)
    assert oracle.normalized_error(C, ref, D) <= TOL


def test_split_integer_exact_and_deterministic(gpu):
    a = _run(gpu, "U", "N", 300, 400, 1.5, 0.5, seed=81, dist="integers", splits=5)
    b = _run(gpu, "U", "N", 300, 400, 1.5, 0.5, seed=81, dist="integers", splits=5)
    assert np.array_equal(a[0], a[1]) and np.array_equal(a[0], b[0])


def test_beta_zero_never_reads_c(gpu):
    C, ref, D = _run(gpu, "L", "N", 150, 90, 1.0, 0.0, seed=31, c0_nan=True)
    assert not np.isnan(C).any()
    assert oracle.normalized_error(C, ref, D) <= TOL


@pytest.mark.parametrize("alpha,K,beta", [(0.0, 50, 0.5), (1.0, 0, -2.0), (0.0, 10, 0.0), (0.0, 10, 1.0)])
def test_quick_returns(gpu, alpha, K, beta):
    C, ref, _ = _run(gpu, "U", "T", 70, K, alpha, beta, seed=41)
    assert np.array_equal(C, ref)


@pytest.mark.slow
def test_full_size_8192_sampled(gpu):
    """N = K = 8192, the benchmark's launch; a sample of rows of the triangle."""
    N = K = 8192
    X, Y = si.uniform((N, K), 51), si.uniform((N, K), 52)
    C0 = si.uniform((N, N), 53)
    dA = torch.from_numpy(X).to(gpu)
    dB = torch.from_numpy(Y).to(gpu)
    dC = torch.from_numpy(C0).to(gpu)
    nat = _native()
    need = nat.mg_syr2k_workspace_size(0, N, K)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=gpu)
    assert nat.mg_syr2k(0, "L", "N", N, K, 1.5, dA.data_ptr(), K, dB.data_ptr(), K, 0.5, dC.data_ptr(), N,
                        ws.data_ptr(), need, torch.cuda.current_stream().cuda_stream) == 0
    torch.cuda.synchronize()
    out = dC.cpu().numpy()
    rng = np.random.default_rng(54)
    for i in rng.choice(np.arange(100, N), 12, replace=False):
        # entries (i, j), j in a sample below i: the oracle's SYR2K on the rows
        # S = sample + [i] gives them as the last row of its lower triangle
        J = np.sort(rng.choice(i, 64, replace=False))
        S = np.concatenate([J, [i]])
        Cs = C0[np.ix_(S, S)].copy()
        ref, D = oracle.syr2k("L", "N", len(S), K, 1.5, X[S], K, Y[S], K, 0.5, Cs)
        ref = ref.reshape(len(S), len(S))[-1]
        err = oracle.normalized_error(out[i, S].astype(np.float64), ref, D[-1])
        assert err <= TOL, (i, err)
        assert np.array_equal(out[i, i + 1:], C0[i, i + 1:])
