#pragma once
// The fused C update after the K loop (the step that follows the kk loop in
// Algorithm 1 of Kuzma et al., SPE 2023) for a wave's V x H grid of 32 x 32
// matrix-core accumulators: C[m][n] = combine(acc, C0[m][n]) for every
// in-range element.  Register r of lane (c = l % 32, h = l / 32) of block
// (i, j) holds row mw + 32i + 8(r/4) + 4h + r%4, column nw + 32j + c, so the
// 32 lanes of a half-wave store 32 consecutive elements of one row.
//
// C0 is read through the pointer C is written through, so a load placed
// between the stores could not be moved ahead of them and would wait a whole
// memory round trip.  When read_c0 is set, the C0 values of one block row i
// are therefore all loaded first (16 x H loads in flight), then the block row
// is stored.  When it is clear C0 is not read and combine receives 0.
#include "common.h"

namespace mg {

template <int V, int H, typename T, typename Acc, typename Combine>
MG_DEVICE void store_acc_blocks(T* C, int64_t ldc, int64_t M, int64_t N, int64_t mw, int64_t nw, int h, int c,
                                bool read_c0, const Acc (&acc)[V][H], Combine combine)
{
    // rows per batch: half a block row for the largest accumulator grids,
    // whose registers leave no room for 16 x H loaded values and addresses
    constexpr int RB = V * H >= 16 ? 4 : 16;
#pragma unroll
    for (int i = 0; i < V; ++i) {
#pragma unroll
        for (int r0 = 0; r0 < 16; r0 += RB) {
            T c0[RB][H];
            if (read_c0) {
#pragma unroll
                for (int rr = 0; rr < RB; ++rr) {
                    // out-of-range lanes read a clamped in-range element
                    // that is never stored, so the loads need no branches
                    const int r = r0 + rr;
                    const int64_t m = mw + 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
                    const T* crow = C + (m < M ? m : M - 1) * ldc;
#pragma unroll
                    for (int j = 0; j < H; ++j) {
                        const int64_t n = nw + 32 * j + c;
                        c0[rr][j] = crow[n < N ? n : N - 1];
                    }
                }
            } else {
#pragma unroll
                for (int rr = 0; rr < RB; ++rr)
#pragma unroll
                    for (int j = 0; j < H; ++j) c0[rr][j] = T(0);
            }
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
                const int r = r0 + rr;
                const int64_t m = mw + 32 * i + 8 * (r >> 2) + 4 * h + (r & 3);
                if (m >= M) continue;
                T* crow = C + m * ldc;
#pragma unroll
                for (int j = 0; j < H; ++j) {
                    const int64_t n = nw + 32 * j + c;
                    if (n < N) crow[n] = combine(acc[i][j][r], c0[rr][j]);
                }
            }
        }
    }
}

}  // namespace mg
