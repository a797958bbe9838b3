#pragma once
// FP32 GEMM tile WITHOUT packing: the "Tiling" strategy of Kuzma et al.
// (SPE 2023, Section 4.1.3), next to the packed "Tiling+Packing" scheme of
// tile_f32.h.
//
// The GEMM loops are still tiled (workgroup tile, wave tile, an 8-deep K
// chunk) and the innermost computation is still the matrix intrinsic, but the
// operands are never reorganised into a packed buffer: every lane loads the
// MFMA operand values it needs straight from the stored matrices in global
// memory into registers, and the only reuse is through registers and the
// caches.  No LDS and no workgroup barrier are involved, so a wave starts its
// first MFMA as soon as its own loads land; the price is that neighbouring
// waves fetch the same A rows and B columns again (from L1/L2), and loads
// along a matrix's leading dimension do not coalesce.  The paper finds this
// strategy best for small matrices and packing best for large ones; the same
// trade-off is measured here across the size sweep.
//
// Operand mapping.  v_mfma_f32_32x32x2_f32 sums over two k slots per
// instruction: lane (c, h) = (lane % 32, lane / 32) supplies op(A)[row c][slot
// h] and op(B)[slot h][col c].  The k index is only a summation index, so any
// assignment of k values to (step, slot) that A and B share gives the same
// product.  Over an 8-deep chunk starting at k0, step t (0..3) puts
// k = k0 + 4h + t in slot h: each lane then needs 4 CONSECUTIVE k of its row
// of op(A) and of its column of op(B), which is one 16-byte load whenever that
// operand is stored k-contiguous (A as M x K, B as N x K).
#include "common.h"
#include "epilogue.h"

namespace mg {

// One 8-deep chunk of operand values for one lane: 4 consecutive k of one row
// (A) or column (B).  `kcontig`: the stored matrix is k-contiguous for this
// operand (element (r, k) at src[r * ld + k]); else element (r, k) is at
// src[k * ld + r].  R and Kd bound the valid rows and k; out-of-range values
// read 0 (both operands are zero-padded along K, Section 3.1's remainder rule).
template <bool KCONTIG>
MG_DEVICE floatx4 direct_fetch(const float* __restrict__ src, int64_t ld, int64_t r, int64_t k,
                               int64_t R, int64_t Kd, bool vec, bool interior)
{
    if (interior) {
        if (KCONTIG) {
            if (vec) return *reinterpret_cast<const floatx4*>(src + r * ld + k);
            const float* p = src + r * ld + k;
            return floatx4{p[0], p[1], p[2], p[3]};
        }
        const float* p = src + k * ld + r;
        return floatx4{p[0], p[ld], p[2 * ld], p[3 * ld]};
    }
    floatx4 x = {0.f, 0.f, 0.f, 0.f};
    if (r >= R) return x;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        if (k + t < Kd) x[t] = KCONTIG ? src[r * ld + k + t] : src[(k + t) * ld + r];
    return x;
}

// Workgroup of WAVES_M x WAVES_N waves, each owning a WM x WN block of the
// BM x BN tile (tm, tn) of C; BM = WAVES_M * WM, BN = WAVES_N * WN.
template <int WAVES_M, int WAVES_N, int WM, int WN, bool TA, bool TB>
MG_DEVICE void direct_tile(const GemmArgs& g, int tm, int tn)
{
    constexpr int V = WM / 32, H = WN / 32;
    constexpr int BM = WAVES_M * WM, BN = WAVES_N * WN;
    static_assert(V >= 1 && V <= 4 && H >= 1 && H <= 4, "wave tile of 32..128");

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int c = lane & 31, h = lane >> 5;
    const int64_t mw = int64_t(tm) * BM + (wave / WAVES_N) * WM;   // first row of this wave
    const int64_t nw = int64_t(tn) * BN + (wave % WAVES_N) * WN;   // first column
    // op(A) row r, k: A is K-contiguous when stored M x K ('N').
    // op(B) k, column n: B is K-contiguous when stored N x K ('T').
    constexpr bool A_KCONTIG = !TA, B_KCONTIG = TB;
    const bool rows_in = mw + WM <= g.M, cols_in = nw + WN <= g.N;

    floatx16 acc[V][H];
#pragma unroll
    for (int i = 0; i < V; ++i)
#pragma unroll
        for (int j = 0; j < H; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    floatx4 fa[V], fb[H];
    auto fetch = [&](int64_t k0, floatx4 (&a)[V], floatx4 (&b)[H]) {
        const int64_t k = k0 + 4 * h;
        const bool kin = k0 + 8 <= g.K;
#pragma unroll
        for (int i = 0; i < V; ++i)
            a[i] = direct_fetch<A_KCONTIG>(g.A, g.lda, mw + 32 * i + c, k, g.M, g.K, g.vec_a, kin && rows_in);
#pragma unroll
        for (int j = 0; j < H; ++j)
            b[j] = direct_fetch<B_KCONTIG>(g.B, g.ldb, nw + 32 * j + c, k, g.N, g.K, g.vec_b, kin && cols_in);
    };

    const int64_t nchunks = (g.K + 7) / 8;
    if (nchunks > 0) fetch(0, fa, fb);
    for (int64_t kc = 0; kc < nchunks; ++kc) {
        // the next chunk's loads are in flight while this chunk multiplies
        floatx4 na[V], nb[H];
        const bool more = kc + 1 < nchunks;
        if (more) fetch((kc + 1) * 8, na, nb);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < V; ++i)
#pragma unroll
                for (int j = 0; j < H; ++j) acc[i][j] = mfma_f32_32x32x2(fa[i][t], fb[j][t], acc[i][j]);
        if (more) {
#pragma unroll
            for (int i = 0; i < V; ++i) fa[i] = na[i];
#pragma unroll
            for (int j = 0; j < H; ++j) fb[j] = nb[j];
        }
    }

    // Epilogue C = alpha*acc + beta*C0 (C0 not read when beta == 0).
    const float alpha = g.alpha, beta = g.beta;
    store_acc_blocks<V, H>(g.C, g.ldc, g.M, g.N, mw, nw, h, c, beta != 0.f, acc,
                           [&](float a, float c0) { return beta != 0.f ? __builtin_fmaf(alpha, a, beta * c0) : alpha * a; });
}

}  // namespace mg
