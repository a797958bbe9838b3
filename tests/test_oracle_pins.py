"""Pins of the FP64 oracle against things other than itself.

Each test names what fixes the expected value: exact rational arithmetic,
integer arithmetic, closed forms, invariants of the GEMM definition, or a
library conversion routine.  A plausible mistake in the oracle (a dropped
term, a wrong sign or index, a transposed operand, alpha/beta swapped, beta
applied when zero, a wrong rounding tie) fails at least one of them.
"""
from fractions import Fraction
import itertools

import numpy as np
import pytest
import torch

import oracle
import seeded_inputs as si


def _stored(logical, trans):
    buf, ld = si.store(logical, trans)
    return buf, ld


def _run(opA, opB, tA="N", tB="N", alpha=1.0, beta=0.0, C0=None, threads=None):
    M, K = opA.shape
    N = opB.shape[1]
    A, lda = _stored(opA, tA)
    B, ldb = _stored(opB, tB)
    return oracle.gemm(tA, tB, M, N, K, alpha, A, lda, B, ldb, beta, C0, N, threads=threads)


# ---------------------------------------------------------------- GEMM ----

@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (2, 3, 4), (5, 4, 3), (3, 5, 6), (6, 6, 6), (4, 1, 5)])
@pytest.mark.parametrize("tA,tB", [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")])
def test_gemm_exact_rational_dyadic(M, N, K, tA, tB):
    """Short dyadic inputs: every product and partial sum is exact, so the
    oracle must equal the exact rational result of the definition."""
    opA = si.dyadic((M, K), 11 + M)
    opB = si.dyadic((K, N), 12 + N)
    C0 = si.dyadic((M, N), 13 + K)
    alpha, beta = 1.5, -0.75
    C, D = _run(opA, opB, tA, tB, alpha, beta, C0)
    for i in range(M):
        for j in range(N):
            s = sum(Fraction(float(opA[i, k])) * Fraction(float(opB[k, j])) for k in range(K))
            d = sum(abs(Fraction(float(opA[i, k])) * Fraction(float(opB[k, j]))) for k in range(K))
            exact = Fraction(alpha) * s + Fraction(beta) * Fraction(float(C0[i, j]))
            dexact = Fraction(abs(alpha)) * d + Fraction(abs(beta)) * abs(Fraction(float(C0[i, j])))
            assert Fraction(C[i, j]) == exact
            assert Fraction(D[i, j]) == dexact


@pytest.mark.parametrize("M,N,K", [(3, 4, 5), (6, 2, 6), (5, 5, 1)])
def test_gemm_random_float32_within_fp64_bound(M, N, K):
    """Random float32 inputs: the oracle lies within the FP64 summation bound
    of the exact result (each product is exact; at most K roundings)."""
    opA = si.uniform((M, K), 21)
    opB = si.uniform((K, N), 22)
    C0 = si.uniform((M, N), 23)
    alpha, beta = 1.5, 0.5
    C, _ = _run(opA, opB, alpha=alpha, beta=beta, C0=C0)
    u = Fraction(1, 2 ** 53)
    for i in range(M):
        for j in range(N):
            terms = [Fraction(float(opA[i, k])) * Fraction(float(opB[k, j])) for k in range(K)]
            exact = Fraction(alpha) * sum(terms) + Fraction(beta) * Fraction(float(C0[i, j]))
            bound = (K + 3) * u * (Fraction(alpha) * sum(abs(t) for t in terms)
                                   + Fraction(beta) * abs(Fraction(float(C0[i, j])))) * 2
            assert abs(Fraction(C[i, j]) - exact) <= bound


def test_gemm_integer_exact_vs_int64_matmul():
    """Integer entries: the FP64 result is exact and equals int64 arithmetic."""
    opA = si.integers((37, 53), 31)
    opB = si.integers((53, 29), 32)
    C0 = si.integers((37, 29), 33)
    C, D = _run(opA, opB, alpha=3.0, beta=-2.0, C0=C0)
    ref = 3 * (opA.astype(np.int64) @ opB.astype(np.int64)) - 2 * C0.astype(np.int64)
    dref = 3 * (np.abs(opA).astype(np.int64) @ np.abs(opB).astype(np.int64)) + 2 * np.abs(C0).astype(np.int64)
    assert np.array_equal(C, ref.astype(np.float64))
    assert np.array_equal(D, dref.astype(np.float64))


def test_gemm_layouts_bitwise_identical():
    """NN/NT/TN/TT of the same logical operands must give identical bits:
    the transpose only changes how elements are fetched."""
    opA = si.uniform((19, 23), 41)
    opB = si.uniform((23, 17), 42)
    C0 = si.uniform((19, 17), 43)
    outs = [_run(opA, opB, tA, tB, 1.5, 0.5, C0)[0] for tA in "NT" for tB in "NT"]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    # lower-case and 'C' (conjugate == transpose for real data) are accepted
    Cc = _run(opA, opB, "c", "n", 1.5, 0.5, C0)[0]
    assert np.array_equal(Cc, outs[0])


def test_gemm_padded_leading_dimension():
    """lda/ldb larger than the row length: the padding (NaN) is never read."""
    opA = si.uniform((7, 9), 51)
    opB = si.uniform((9, 5), 52)
    A, lda = si.store(opA, "T", ld=13)
    B, ldb = si.store(opB, "N", ld=11)
    C, _ = oracle.gemm("T", "N", 7, 5, 9, 1.0, A, lda, B, ldb)
    C2, _ = _run(opA, opB)
    assert np.array_equal(C, C2)
    assert not np.isnan(C).any()


def test_gemm_column_major_operand_swap_identity():
    """A column-major GEMM is the row-major GEMM of the swapped operands:
    colmajor(C) = A B  <=>  rowmajor(C^T) = B^T A^T."""
    opA = si.uniform((6, 8), 61)
    opB = si.uniform((8, 4), 62)
    # column-major storage of opA is the row-major storage of opA^T
    A_cm = np.ascontiguousarray(opA.T).reshape(-1)
    B_cm = np.ascontiguousarray(opB.T).reshape(-1)
    # row-major call computing C^T = opB^T opA^T, with B_cm as the first operand ('N')
    Ct, _ = oracle.gemm("N", "N", 4, 6, 8, 1.0, B_cm, 8, A_cm, 6)
    C, _ = _run(opA, opB)
    assert np.array_equal(Ct.T, C)


@pytest.mark.parametrize("tA,tB", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
def test_gemm_identity_and_permutation(tA, tB):
    """A = I gives alpha*B + beta*C0; A = P gives the permuted rows of B."""
    n = 11
    B = si.uniform((n, 7), 71)
    C0 = si.uniform((n, 7), 72)
    C, _ = _run(np.eye(n, dtype=np.float32), B, tA, tB, 2.0, 0.5, C0)
    assert np.array_equal(C, 2.0 * B.astype(np.float64) + 0.5 * C0.astype(np.float64))
    perm = np.random.default_rng(73).permutation(n)
    P = np.eye(n, dtype=np.float32)[perm]
    C, _ = _run(P, B, tA, tB)
    assert np.array_equal(C, B[perm].astype(np.float64))
    # permutation on the right permutes columns
    Q = np.eye(7, dtype=np.float32)[np.random.default_rng(74).permutation(7)]
    C, _ = _run(B, Q, tA, tB)
    assert np.array_equal(C, (B @ Q).astype(np.float64))


def test_gemm_ones_closed_form():
    """All-ones A and B: every entry is alpha*K + beta*C0."""
    M, N, K = 9, 10, 77
    C0 = si.integers((M, N), 81)
    C, D = _run(np.ones((M, K), np.float32), np.ones((K, N), np.float32), alpha=1.5, beta=0.5, C0=C0)
    assert np.array_equal(C, 1.5 * K + 0.5 * C0.astype(np.float64))
    assert np.array_equal(D, 1.5 * K + 0.5 * np.abs(C0).astype(np.float64))


def test_gemm_alpha_beta_not_swapped_and_signs():
    """Distinguish alpha from beta and both signs with a 1x1x1 problem."""
    for alpha, beta in [(2.0, 3.0), (-2.0, 3.0), (2.0, -3.0), (0.5, 0.25)]:
        C, D = oracle.gemm("N", "N", 1, 1, 1, alpha, np.array([5.0]), 1, np.array([7.0]), 1,
                           beta, np.array([11.0]), 1)
        assert C[0, 0] == alpha * 35.0 + beta * 11.0
        assert D[0, 0] == abs(alpha) * 35.0 + abs(beta) * 11.0


def test_gemm_special_values():
    """BLAS readings: beta = 0 never reads C0; alpha = 0 or K = 0 give beta*C0;
    M = 0 or N = 0 is empty; a NaN in A only touches its own row."""
    M, N, K = 5, 6, 7
    opA = si.uniform((M, K), 91)
    opB = si.uniform((K, N), 92)
    C0 = si.uniform((M, N), 93)
    nanC = np.full((M, N), np.nan, np.float32)
    C, _ = _run(opA, opB, beta=0.0, C0=nanC)
    assert not np.isnan(C).any()
    A_nan = opA.copy()
    A_nan[2, 3] = np.nan
    C, _ = _run(A_nan, opB, alpha=0.0, beta=0.5, C0=C0)
    assert np.array_equal(C, 0.5 * C0.astype(np.float64))
    C, _ = oracle.gemm("N", "N", M, N, 0, 1.0, np.zeros(1), 1, np.zeros(1), N, 0.5, C0, N)
    assert np.array_equal(C, 0.5 * C0.astype(np.float64))
    C, _ = oracle.gemm("N", "N", M, N, 0, 1.0, np.zeros(1), 1, np.zeros(1), N, 0.0, nanC, N)
    assert np.array_equal(C, np.zeros((M, N)))
    C, _ = oracle.gemm("N", "N", 0, N, K, 1.0, np.zeros(1), K, opB, N)
    assert C.shape == (0, N)
    C, _ = _run(A_nan, opB)
    assert np.isnan(C[2]).all()
    assert not np.isnan(np.delete(C, 2, axis=0)).any()
    A_inf = opA.copy()
    A_inf[1, 0] = np.inf
    C, _ = _run(A_inf, np.abs(opB) + 1)
    assert np.isinf(C[1]).all() and not np.isinf(np.delete(C, 1, axis=0)).any()


def test_gemm_thread_count_invariant():
    opA = si.uniform((33, 41), 101)
    opB = si.uniform((41, 27), 102)
    C1, D1 = _run(opA, opB, threads=1)
    C8, D8 = _run(opA, opB, threads=8)
    assert np.array_equal(C1, C8) and np.array_equal(D1, D8)


def test_gemm_entries_match_full():
    M, N, K = 31, 29, 43
    for tA, tB in itertools.product("NT", "NT"):
        opA = si.uniform((M, K), 111)
        opB = si.uniform((K, N), 112)
        C0 = si.uniform((M, N), 113)
        A, lda = si.store(opA, tA)
        B, ldb = si.store(opB, tB)
        C, D = oracle.gemm(tA, tB, M, N, K, 1.5, A, lda, B, ldb, 0.5, C0, N)
        I, J = si.sample_indices(M, N, 100, 114)
        c, d = oracle.gemm_entries(tA, tB, K, 1.5, A, lda, B, ldb, 0.5, C0, N, I, J)
        assert np.array_equal(c, C[I, J]) and np.array_equal(d, D[I, J])


def test_normalized_error_metric():
    Cref = np.array([[1.0, 0.0], [2.0, -1.0]])
    D = np.array([[2.0, 0.0], [4.0, 1.0]])
    assert oracle.normalized_error(Cref, Cref, D) == 0.0
    C = Cref + np.array([[0.5, 0.0], [0.0, 0.0]])
    assert oracle.normalized_error(C, Cref, D) == 0.25
    C = Cref + np.array([[0.0, 1e-30], [0.0, 0.0]])   # nonzero over a zero denominator
    assert oracle.normalized_error(C, Cref, D) == float("inf")
    C = Cref.copy()
    C[1, 1] = np.nan
    assert oracle.normalized_error(C, Cref, D) == float("inf")


# ------------------------------------------------------------ bfloat16 ----

def _torch_bf16(x):
    return torch.from_numpy(np.asarray(x, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def test_bf16_round_matches_library_conversion():
    """torch's float32 -> bfloat16 cast is round-to-nearest-even."""
    x = np.concatenate([si.uniform(20000, 121), si.log_uniform_signed(20000, 122, -30, 30),
                        np.array([0.0, -0.0, 1.0, -1.0, 3.0e38, -3.0e38, 1e-39, -1e-40], np.float32)])
    # exact ties: low 16 bits == 0x8000, with both even and odd kept parts
    bits = (np.random.default_rng(123).integers(0x3000, 0x5000, 4000).astype(np.uint32) << 16) | 0x8000
    ties = bits.view(np.float32)
    x = np.concatenate([x, ties])
    assert np.array_equal(oracle.bf16_round(x), _torch_bf16(x))


def test_bf16_round_tie_cases_by_hand():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> even (1)
    assert oracle.round_to_bits(1 + 2 ** -8, 8, -126) == 1.0
    # 1 + 3*2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6 -> even (1 + 2^-6)
    assert oracle.round_to_bits(1 + 3 * 2 ** -8, 8, -126) == 1 + 2 ** -6
    assert oracle.round_to_bits(-(1 + 3 * 2 ** -8), 8, -126) == -(1 + 2 ** -6)
    assert oracle.round_to_bits(1 + 2 ** -8 + 2 ** -20, 8, -126) == 1 + 2 ** -7


def test_bf16_split_properties():
    x = np.concatenate([si.uniform(50000, 131), si.log_uniform_signed(50000, 132)]).astype(np.float64)
    hi, lo = oracle.bf16_split(x)
    assert np.array_equal(hi, _torch_bf16(x))
    assert np.array_equal(lo, _torch_bf16((x - hi).astype(np.float32)))
    # hi + lo carries 16 significant bits: the residual is below 2^-16 |x|
    assert np.all(np.abs(x - hi - lo) <= 2.0 ** -16 * np.abs(x))
    # the residual x - hi is exactly representable in float32
    assert np.array_equal((x - hi).astype(np.float32).astype(np.float64), x - hi)


# ------------------------------------------------------------- FP8 E4M3 ---

def _torch_e4m3_table():
    b = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn)
    return b.to(torch.float64).numpy()


def test_e4m3_decode_matches_library():
    ours = oracle.e4m3_decode_table()
    ref = _torch_e4m3_table()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan)
    assert np.array_equal(ours[~nan], ref[~nan])
    assert ours[0x7E] == 448.0 and ours[0x08] == 2.0 ** -6 and ours[0x01] == 2.0 ** -9


def test_e4m3_encode_roundtrip_all_bytes():
    table = oracle.e4m3_decode_table()
    for b in range(256):
        if np.isnan(table[b]):
            continue
        assert oracle.e4m3_encode(table[b]) == b


def test_e4m3_round_matches_library():
    """Below the format maximum, torch's cast to float8_e4m3fn is RNE."""
    x = np.concatenate([si.uniform(20000, 141, -448, 448), si.log_uniform_signed(20000, 142, -4, 2.6)])
    x = x[np.abs(x) <= 448]
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    ours = np.array([oracle.e4m3_value(float(v)) for v in x])
    assert np.array_equal(ours, ref)
    # saturation (satfinite) above the maximum
    assert oracle.e4m3_value(500.0) == 448.0 and oracle.e4m3_value(-1e9) == -448.0
    # ties: 9*2^-? halfway cases, 17/16 is between 1 and 1.125 -> even (1)
    assert oracle.e4m3_value(1.0625) == 1.0
    assert oracle.e4m3_value(1.1875) == 1.25


def test_tile_scale_by_hand():
    """s is the smallest power of two with amax <= 448*s."""
    cases = {448.0: 1.0, 448.5: 2.0, 224.0: 0.5, 224.25: 1.0, 1.0: 2.0 ** -8, 1.75: 2.0 ** -8,
             1.76: 2.0 ** -7, 8.0: 2.0 ** -5, 0.0: 1.0, 896.0: 2.0, 3.5e-3: 2.0 ** -16, 3.4e-3: 2.0 ** -17}
    for amax, s in cases.items():
        assert oracle.tile_scale(amax) == s, amax


def test_fp8_quantize_properties():
    X = si.uniform((300, 260), 151)
    X[:128, 128:256] *= 1000.0   # one tile with a very different range
    q, s = oracle.fp8_quantize(X)
    assert s.shape == (3, 3)
    deq = oracle.fp8_dequantize(q, s)
    # each element within half an E4M3 ulp (relative 2^-4) of its value, or of the subnormal quantum
    tile_s = np.repeat(np.repeat(s.astype(np.float64), 128, 0), 128, 1)[:300, :260]
    err = np.abs(deq - X)
    assert np.all(err <= np.maximum(2.0 ** -4 * np.abs(X), 2.0 ** -10 * tile_s))
    # every tile's max magnitude lands in (224, 448] * s
    for bi in range(3):
        for bj in range(3):
            t = np.abs(X[bi * 128:(bi + 1) * 128, bj * 128:(bj + 1) * 128]).max()
            assert 224 * s[bi, bj] < t <= 448 * s[bi, bj]


def test_fp8_quantize_integers_exact():
    """Integers in [-8, 8] have at most 3 significant bits, so with a power-of-two
    scale they quantise exactly."""
    X = si.integers((200, 150), 161)
    q, s = oracle.fp8_quantize(X)
    assert np.array_equal(oracle.fp8_dequantize(q, s), X.astype(np.float64))


# ------------------------------------------------------------ gradients ---

def test_chain_grads_match_finite_differences():
    """loss = sum(((X W1) W2) * G) is linear in each single entry, so central
    differences of the FP64 forward equal the analytic gradient up to rounding."""
    X = si.uniform((6, 4), 171)
    W1 = si.uniform((4, 5), 172)
    W2 = si.uniform((5, 3), 173)
    G = si.gaussian((6, 3), 174)
    grads, _ = oracle.chain_grads(X, W1, W2, G)

    def loss(X_, W1_, W2_):
        _, Y = oracle.chain_forward(X_, W1_, W2_)
        return float(np.sum(Y * G.astype(np.float64)))

    eps = 1e-3
    for name, mat in (("dX", X), ("dW1", W1), ("dW2", W2)):
        for idx in itertools.product(*(range(n) for n in mat.shape)):
            p = [X.astype(np.float64), W1.astype(np.float64), W2.astype(np.float64)]
            k = {"dX": 0, "dW1": 1, "dW2": 2}[name]
            plus = [a.copy() for a in p]
            minus = [a.copy() for a in p]
            plus[k][idx] += eps
            minus[k][idx] -= eps
            fd = (loss(*plus) - loss(*minus)) / (2 * eps)
            assert abs(fd - grads[name][idx]) <= 1e-9 * (1 + abs(fd))


def test_chain_grads_shapes_and_denominators():
    X = si.uniform((8, 3), 181)
    W1 = si.uniform((3, 6), 182)
    W2 = si.uniform((6, 2), 183)
    G = si.gaussian((8, 2), 184)
    g, den = oracle.chain_grads(X, W1, W2, G)
    assert g["dX"].shape == (8, 3) and g["dW1"].shape == (3, 6) and g["dW2"].shape == (6, 2)
    for k in g:
        assert np.all(np.abs(g[k]) <= den[k] * (1 + 1e-12))


def _brute_chain(X, W1, W2, G):
    """Gradients of sum(((X W1) W2) * G) and their absolute-value chains, as
    explicit sums over Python integers (exact): for H = X W1,
      dW2[h][d] = sum_m H[m][h] G[m][d],  den = sum_{m,k} |X[m][k]||W1[k][h]||G[m][d]|
      dW1[k][h] = sum_{m,d} X[m][k] G[m][d] W2[h][d],  den = the same over |.|
      dX[m][k]  = sum_{h,d} G[m][d] W2[h][d] W1[k][h], den = the same over |.|"""
    Xi, W1i, W2i, Gi = ([[int(v) for v in row] for row in a] for a in (X, W1, W2, G))
    Mx, D = len(Xi), len(Xi[0])
    Hd = len(W1i[0])
    Do = len(W2i[0])
    g = {"dW2": np.zeros((Hd, Do), dtype=object), "dW1": np.zeros((D, Hd), dtype=object),
         "dX": np.zeros((Mx, D), dtype=object)}
    den = {k: np.zeros(v.shape, dtype=object) for k, v in g.items()}
    for h in range(Hd):
        for d in range(Do):
            for m in range(Mx):
                for k in range(D):
                    g["dW2"][h, d] += Xi[m][k] * W1i[k][h] * Gi[m][d]
                    den["dW2"][h, d] += abs(Xi[m][k]) * abs(W1i[k][h]) * abs(Gi[m][d])
    for k in range(D):
        for h in range(Hd):
            for m in range(Mx):
                for d in range(Do):
                    g["dW1"][k, h] += Xi[m][k] * Gi[m][d] * W2i[h][d]
                    den["dW1"][k, h] += abs(Xi[m][k]) * abs(Gi[m][d]) * abs(W2i[h][d])
    for m in range(Mx):
        for k in range(D):
            for h in range(Hd):
                for d in range(Do):
                    g["dX"][m, k] += Gi[m][d] * W2i[h][d] * W1i[k][h]
                    den["dX"][m, k] += abs(Gi[m][d]) * abs(W2i[h][d]) * abs(W1i[k][h])
    return g, den


def test_chain_grads_and_denominators_equal_brute_force_sums():
    """On small integers every sum is exact in FP64, so the oracle's gradients
    AND its denominators must equal the explicit quadruple sums bit for bit.
    Mixed signs make |dH| smaller than |G||W2|^T, so a denominator built on
    the wrong chain (or any over-estimate) fails here."""
    X = si.integers((5, 3), 185)
    W1 = si.integers((3, 4), 186)
    W2 = si.integers((4, 2), 187)
    G = si.integers((5, 2), 188)
    g, den = oracle.chain_grads(X, W1, W2, G)
    bg, bden = _brute_chain(X, W1, W2, G)
    for k in ("dX", "dW1", "dW2"):
        assert np.array_equal(g[k], bg[k].astype(np.float64)), k
        assert np.array_equal(den[k], bden[k].astype(np.float64)), k
    # the inputs do cancel: at least one denominator exceeds |gradient| somewhere
    assert any(np.any(den[k] > np.abs(g[k])) for k in g)


def test_chain_denominators_equal_int64_chains():
    """The three denominators are the chains |X|^T (|G||W2|^T), (|X||W1|)^T |G|
    and (|G||W2|^T) |W1|^T, checked against numpy's int64 products at a size
    whose sums are still exact in FP64 (entries <= 8, sums < 2^53)."""
    X = si.integers((40, 24), 191).astype(np.int64)
    W1 = si.integers((24, 48), 192).astype(np.int64)
    W2 = si.integers((48, 16), 193).astype(np.int64)
    G = si.integers((40, 16), 194).astype(np.int64)
    _, den = oracle.chain_grads(X.astype(np.float32), W1.astype(np.float32), W2.astype(np.float32),
                                G.astype(np.float32))
    aX, aW1, aW2, aG = np.abs(X), np.abs(W1), np.abs(W2), np.abs(G)
    aGW2 = aG @ aW2.T
    assert np.array_equal(den["dW1"], (aX.T @ aGW2).astype(np.float64))
    assert np.array_equal(den["dW2"], ((aX @ aW1).T @ aG).astype(np.float64))
    assert np.array_equal(den["dX"], (aGW2 @ aW1.T).astype(np.float64))


def test_chain_entries_equal_the_full_chain():
    """chain_entries (sliced oracle GEMMs) equals chain_grads / chain_forward
    and their denominators at its sampled entries, bit for bit on integer
    inputs, where every sum is exact whatever the slicing."""
    X = si.integers((12, 5), 201)
    W1 = si.integers((5, 9), 202)
    W2 = si.integers((9, 5), 203)
    G = si.integers((12, 5), 204)
    g, den = oracle.chain_grads(X, W1, W2, G)
    H, Y = oracle.chain_forward(X, W1, W2)
    aH, aY = oracle.chain_forward(np.abs(X), np.abs(W1), np.abs(W2))
    full = dict(g, Y=Y)
    fden = dict(den, Y=aY)
    got = oracle.chain_entries(X, W1, W2, G, n=4, seed=3)
    assert sorted(got) == ["Y", "dW1", "dW2", "dX"]
    for k, (I, J, vals, dens) in got.items():
        assert len(set(I)) == len(I) and len(set(J)) == len(J)
        assert np.array_equal(vals, full[k][np.ix_(I, J)]), k
        assert np.array_equal(dens, fden[k][np.ix_(I, J)]), k


def test_chain_denominators_equal_gradients_for_nonnegative_inputs():
    """With every input >= 0 the absolute values change nothing, so each
    denominator is its gradient exactly (integers: exact sums)."""
    X = np.abs(si.integers((9, 4), 195))
    W1 = np.abs(si.integers((4, 7), 196))
    W2 = np.abs(si.integers((7, 3), 197))
    G = np.abs(si.integers((9, 3), 198))
    g, den = oracle.chain_grads(X, W1, W2, G)
    for k in g:
        assert np.array_equal(g[k], den[k]), k


# ------------------------------------------------------------------ FP16 ----

def test_fp16_round_matches_library_conversion():
    """numpy's float64 -> float16 cast rounds to nearest even and overflows to
    infinity: the oracle's rounding must agree on normals, subnormals, ties
    and the overflow edge."""
    rng = np.random.default_rng(140)
    x = np.concatenate([si.uniform(20000, 141).astype(np.float64),
                        si.log_uniform_signed(20000, 142, -9, 5).astype(np.float64),
                        rng.uniform(-70000, 70000, 5000),
                        np.array([0.0, -0.0, 65504.0, 65519.99, 65520.0, -65520.0, 2.0 ** -24, 2.0 ** -25,
                                  3 * 2.0 ** -25, 2.0 ** -14, 1e-9])])
    # exact ties: halfway between two adjacent binary16 values
    h = rng.integers(0x0400, 0x7bff, 5000).astype(np.uint16).view(np.float16).astype(np.float64)
    ulp = np.spacing(h.astype(np.float16)).astype(np.float64)
    x = np.concatenate([x, h + ulp / 2, -(h + ulp / 2)])
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(oracle.fp16_round(x), ref)


def test_fp16_round_by_hand():
    r = oracle.fp16_round
    assert r([1 / 3])[0] == 0.333251953125            # 0x3555
    assert r([65504.0])[0] == 65504.0                 # largest finite
    assert r([65519.99])[0] == 65504.0                # below the midpoint to 2^16
    assert np.isinf(r([65520.0])[0])                  # the midpoint rounds to even: 2^16 -> inf
    assert r([2.0 ** -24])[0] == 2.0 ** -24           # smallest subnormal
    assert r([2.0 ** -25])[0] == 0.0                  # tie between 0 and 2^-24 -> even (0)
    assert r([3 * 2.0 ** -25])[0] == 2.0 ** -23       # tie between 2^-24 and 2^-23 -> even (2^-23)
    assert r([1 + 2.0 ** -11])[0] == 1.0              # tie -> even
    assert r([1 + 3 * 2.0 ** -11])[0] == 1 + 2.0 ** -9


# ------------------------------------------------------------------ INT8 ----

def _wrap32(v: int) -> int:
    return ((v + 2 ** 31) % 2 ** 32) - 2 ** 31


@pytest.mark.parametrize("tA,tB", [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (3, 4, 5), (6, 2, 7), (5, 5, 0)])
def test_gemm_i8_exact_vs_python_integers(tA, tB, M, N, K):
    """Python's unbounded integers give the exact value; the wrap modulo 2^32
    is applied by hand (large alpha and beta force it)."""
    rng = np.random.default_rng(150 + M + N + K)
    opA = rng.integers(-128, 128, (M, K)).astype(np.int8)
    opB = rng.integers(-128, 128, (K, N)).astype(np.int8)
    C0 = rng.integers(-2 ** 31, 2 ** 31, (M, N)).astype(np.int32)
    for alpha, beta in [(1, 0), (-3, 2), (2 ** 30 - 7, -(2 ** 29) + 3), (0, 5)]:
        A = opA if tA == "N" else np.ascontiguousarray(opA.T)
        B = opB if tB == "N" else np.ascontiguousarray(opB.T)
        lda = max(A.shape[1], 1)
        ldb = max(B.shape[1], 1)
        got = oracle.gemm_i8(tA, tB, M, N, K, alpha, A, lda, B, ldb, beta, C0, N)
        for i in range(M):
            for j in range(N):
                acc = sum(int(opA[i, k]) * int(opB[k, j]) for k in range(K))
                want = _wrap32(alpha * acc + (beta * int(C0[i, j]) if beta else 0))
                assert int(got[i, j]) == want


def test_gemm_i8_matches_library_int64_matmul():
    rng = np.random.default_rng(151)
    opA = rng.integers(-128, 128, (64, 300)).astype(np.int8)
    opB = rng.integers(-128, 128, (300, 48)).astype(np.int8)
    got = oracle.gemm_i8("N", "N", 64, 48, 300, 1, opA, 300, opB, 48)
    ref = opA.astype(np.int64) @ opB.astype(np.int64)
    assert np.array_equal(got.astype(np.int64), ref)


def test_gemm_i8_extremes_closed_form():
    """All entries -128 at the largest K whose sums stay below 2^31:
    every sum is K * 16384; doubling it wraps."""
    K = 131071
    A = np.full((2, K), -128, np.int8)
    B = np.full((K, 3), -128, np.int8)
    got = oracle.gemm_i8("N", "N", 2, 3, K, 1, A, K, B, 3)
    assert np.all(got == K * 16384)
    got2 = oracle.gemm_i8("N", "N", 2, 3, K, 2, A, K, B, 3)
    assert np.all(got2 == 2 * K * 16384 - 2 ** 32)


def test_gemm_i8_quick_returns():
    A = np.ones((2, 3), np.int8)
    B = np.ones((3, 2), np.int8)
    C0 = np.array([[7, -9], [2 ** 31 - 1, 5]], np.int32)
    # beta == 0: C0 is not read
    assert np.array_equal(oracle.gemm_i8("N", "N", 2, 2, 3, 4, A, 3, B, 2, 0, C0, 2), np.full((2, 2), 12))
    # alpha == 0: beta * C0, wrapped
    got = oracle.gemm_i8("N", "N", 2, 2, 3, 0, A, 3, B, 2, 2, C0, 2)
    assert np.array_equal(got, np.array([[14, -18], [-2, 10]]))


# ----------------------------------------------------------------- SYR2K ----

def _syr2k_inputs(N, K, trans, seed, dist=si.dyadic):
    X = dist((N, K), seed)
    Y = dist((N, K), seed + 1)
    if trans == "N":
        return X, Y, X.copy(), Y.copy(), K
    return X, Y, np.ascontiguousarray(X.T), np.ascontiguousarray(Y.T), N


@pytest.mark.parametrize("uplo", ["L", "U"])
@pytest.mark.parametrize("trans", ["N", "T"])
@pytest.mark.parametrize("N,K", [(1, 1), (3, 2), (4, 5), (5, 3)])
def test_syr2k_exact_rational(uplo, trans, N, K):
    """Dyadic inputs: exact rational arithmetic of the definition equals the
    oracle exactly on the triangle, and the other triangle is untouched."""
    X, Y, A, B, ld = _syr2k_inputs(N, K, trans, 160 + N + K)
    C0 = si.dyadic((N, N), 170 + N)
    alpha, beta = 1.5, -0.75
    C, _ = oracle.syr2k(uplo, trans, N, K, alpha, A, ld, B, ld, beta, C0)
    C = C.reshape(N, N)
    for i in range(N):
        for j in range(N):
            inside = (i >= j) if uplo == "L" else (i <= j)
            if not inside:
                assert C[i, j] == C0[i, j]
                continue
            s = sum(Fraction(float(X[i, k])) * Fraction(float(Y[j, k])) +
                    Fraction(float(Y[i, k])) * Fraction(float(X[j, k])) for k in range(K))
            assert Fraction(C[i, j]) == Fraction(alpha) * s + Fraction(beta) * Fraction(float(C0[i, j]))


def test_syr2k_matches_library_matmul():
    N, K = 50, 30
    X, Y = si.uniform((N, K), 180), si.uniform((N, K), 181)
    C0 = si.uniform((N, N), 182)
    C, D = oracle.syr2k("L", "N", N, K, -1.25, X, K, Y, K, 0.5, C0)
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    ref = -1.25 * (X64 @ Y64.T + Y64 @ X64.T) + 0.5 * C0
    low = np.tril_indices(N)
    assert np.allclose(C.reshape(N, N)[low], ref[low], rtol=0, atol=1e-12)
    dref = 1.25 * (np.abs(X64) @ np.abs(Y64).T + np.abs(Y64) @ np.abs(X64).T) + 0.5 * np.abs(C0)
    assert np.allclose(D[low], dref[low], rtol=1e-13, atol=0)


def test_syr2k_symmetries():
    """Swapping A and B changes nothing; the upper triangle is the transpose
    of the lower one when C0 is symmetric; beta == 0 never reads C."""
    N, K = 23, 17
    X, Y = si.uniform((N, K), 190), si.uniform((N, K), 191)
    S = si.uniform((N, N), 192)
    C0 = (S + S.T) / 2
    L, _ = oracle.syr2k("L", "N", N, K, 0.7, X, K, Y, K, 0.3, C0)
    L2, _ = oracle.syr2k("L", "N", N, K, 0.7, Y, K, X, K, 0.3, C0)
    U, _ = oracle.syr2k("U", "N", N, K, 0.7, X, K, Y, K, 0.3, C0)
    assert np.array_equal(L, L2)
    L, U = L.reshape(N, N), U.reshape(N, N)
    low = np.tril_indices(N)
    assert np.array_equal(L[low], U.T[low])
    Cn = np.full((N, N), np.nan)
    Z, _ = oracle.syr2k("L", "N", N, K, 0.7, X, K, Y, K, 0.0, Cn)
    assert not np.isnan(Z.reshape(N, N)[low]).any()


def test_syr2k_equal_operands_closed_form():
    """A == B (integers): C = 2*alpha*A*A^T + beta*C0, exactly."""
    N, K = 31, 40
    X = si.integers((N, K), 193)
    C0 = si.integers((N, N), 194)
    C, _ = oracle.syr2k("U", "N", N, K, 1.5, X, K, X, K, 0.5, C0)
    Xi = X.astype(np.int64)
    ref = 1.5 * 2 * (Xi @ Xi.T) + 0.5 * C0
    up = np.triu_indices(N)
    assert np.array_equal(C.reshape(N, N)[up], ref[up])


@pytest.mark.parametrize("trans", ["N", "T"])
def test_syr2k_entries_equal_the_full_syr2k(trans):
    """syr2k_entries (two oracle GEMM entry sums) equals the full SYR2K oracle
    and its denominator at sampled entries of both triangles: bit for bit on
    integer inputs, where the one extra FP64 addition is exact."""
    N, K = 23, 17
    shape = (N, K) if trans == "N" else (K, N)
    A = si.integers(shape, 211 + (trans == "T"))
    B = si.integers(shape, 213 + (trans == "T"))
    C0 = si.integers((N, N), 215)
    lda = ldb = shape[1]
    I, J = si.sample_indices(N, N, 60, 216)
    vals, dens = oracle.syr2k_entries(trans, K, 1.5, A, lda, B, ldb, -0.5, C0, N, I, J)
    for uplo in "LU":
        full, D = oracle.syr2k(uplo, trans, N, K, 1.5, A, lda, B, ldb, -0.5, C0)
        full = full.reshape(N, N)
        tri = (I >= J) if uplo == "L" else (I <= J)
        assert np.array_equal(vals[tri], full[I[tri], J[tri]])
        assert np.array_equal(dens[tri], D[I[tri], J[tri]])
