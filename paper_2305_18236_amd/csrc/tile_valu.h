#pragma once
// FP32 GEMM tile whose micro-kernel runs on the vector ALUs instead of the
// matrix cores: the GPU counterpart of the paper's "generic lowering" of the
// matrix-multiply intrinsic to ordinary vector FMAs (Section 3.2), measured
// against the matrix-core lowering as in its VSX-vs-MMA comparison
// (Section 4.4).
//
// The macro level is the one of tile_f32.h unchanged: the same BM x BN
// workgroup tile, the same double-buffered k-major LDS panels written by the
// same PanelLoader (transposition absorbed, zero padding, bank swizzle).  Only
// the micro-kernel differs: each thread owns an 8 x 8 block of C in 64 VGPRs
// and, for every k of the panel, reads 8 values of op(A) and 8 of op(B) from
// LDS (four 16-byte reads) and issues 64 scalar v_fma_f32 (the outer product).
// Thread (tx, ty) = (tid % 16, tid / 16) of 256 owns rows ty*4 + {0..3} and
// 64 + ty*4 + {0..3}, columns tx*4 + {0..3} and 64 + tx*4 + {0..3}: the 16 lanes
// of a quarter-wave read one A address (broadcast) and 16 consecutive float4
// of B (conflict-free).
#include "tile_f32.h"

namespace mg {

template <int BK, bool TA, bool TB>
MG_DEVICE void valu_tile(const GemmArgs& g, int tm, int tn, float* smem)
{
    constexpr int BM = 128, BN = 128, NT = 256;
    float (*As)[BK * BM] = reinterpret_cast<float (*)[BK * BM]>(smem);
    float (*Bs)[BK * BN] = reinterpret_cast<float (*)[BK * BN]>(smem + 2 * BK * BM);

    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int64_t m0 = int64_t(tm) * BM, n0 = int64_t(tn) * BN;

    using LA = PanelLoader<TA ? BK : BM, TA ? BM : BK, NT>;
    using LB = PanelLoader<TB ? BN : BK, TB ? BK : BN, NT>;
    LA la;
    LB lb;
    const int64_t Ra = TA ? g.K : g.M, Ca = TA ? g.M : g.K;
    const int64_t Rb = TB ? g.N : g.K, Cb = TB ? g.K : g.N;
    auto fetch = [&](int64_t k0) {
        if (TA) la.load(g.A, g.lda, k0, m0, Ra, Ca, g.vec_a, tid);
        else    la.load(g.A, g.lda, m0, k0, Ra, Ca, g.vec_a, tid);
        if (TB) lb.load(g.B, g.ldb, n0, k0, Rb, Cb, g.vec_b, tid);
        else    lb.load(g.B, g.ldb, k0, n0, Rb, Cb, g.vec_b, tid);
    };
    auto pack = [&](int buf) {
        la.template store<TA, BM>(As[buf], tid);
        lb.template store<!TB, BN>(Bs[buf], tid);
    };

    float acc[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = 0.f;

    const int nk = int((g.K + BK - 1) / BK);
    if (nk > 0) {
        fetch(0);
        pack(0);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) fetch(int64_t(kt + 1) * BK);
        // unrolled by 2 only: full unrolling lets the compiler hoist every
        // LDS read of the panel ahead of the FMAs (128+ live registers)
#pragma unroll 2
        for (int k = 0; k < BK; ++k) {
            const int sw = panel_swizzle<BK>(k);
            const float* ar = As[cur] + k * BM;
            const float* br = Bs[cur] + k * BN;
            const floatx4 a0 = *reinterpret_cast<const floatx4*>(ar + ((ty * 4) ^ sw));
            const floatx4 a1 = *reinterpret_cast<const floatx4*>(ar + ((64 + ty * 4) ^ sw));
            const floatx4 b0 = *reinterpret_cast<const floatx4*>(br + ((tx * 4) ^ sw));
            const floatx4 b1 = *reinterpret_cast<const floatx4*>(br + ((64 + tx * 4) ^ sw));
            const float a[8] = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
            const float b[8] = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[i][j] = __builtin_fmaf(a[i], b[j], acc[i][j]);
        }
        // the next panel goes into the other buffer, last read before the
        // previous barrier; the barrier then publishes it
        if (kt + 1 < nk) pack(cur ^ 1);
        __syncthreads();
    }

    // Epilogue: C = alpha*acc + beta*C0 (C0 not read when beta == 0).  C0 is
    // read through the pointer C is written through, so a load placed between
    // the stores could not be moved ahead of them: all 16 of the thread's C0
    // pieces are loaded first (out-of-range rows and columns read a clamped
    // in-range element that is never stored), then the results are stored.
    const float alpha = g.alpha, beta = g.beta;
    auto row_of = [&](int i) { return m0 + (i < 4 ? ty * 4 + i : 64 + ty * 4 + (i - 4)); };
    floatx4 c0[8][2];
    if (beta != 0.f) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int64_t m = row_of(i);
            const float* crow = g.C + (m < g.M ? m : g.M - 1) * g.ldc;
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int64_t n = n0 + half * 64 + tx * 4;
                if (g.vec_c && n + 3 < g.N) {
                    c0[i][half] = *reinterpret_cast<const floatx4*>(crow + n);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) c0[i][half][e] = crow[n + e < g.N ? n + e : g.N - 1];
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t m = row_of(i);
        if (m >= g.M) continue;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int64_t n = n0 + half * 64 + tx * 4;
            float* cp = g.C + m * g.ldc + n;
            const float* v = &acc[i][half * 4];
            floatx4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                o[e] = beta != 0.f ? __builtin_fmaf(alpha, v[e], beta * c0[i][half][e]) : alpha * v[e];
            if (g.vec_c && n + 3 < g.N) {
                *reinterpret_cast<floatx4*>(cp) = o;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (n + e < g.N) cp[e] = o[e];
            }
        }
    }
}

}  // namespace mg
