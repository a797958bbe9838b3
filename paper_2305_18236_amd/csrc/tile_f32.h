#pragma once
// FP32 GEMM tile on the FP32 matrix cores of gfx950 (v_mfma_f32_32x32x2_f32).
//
// This is the layered scheme of Kuzma et al. (SPE 2023), Algorithm 1, mapped
// onto one GPU:
//   * the j (nc) and i (mc) block loops become the workgroup grid: each
//     workgroup owns one BM x BN tile of C (tile_of() orders the tiles so that
//     concurrently running workgroups share panels in L2, the role the paper
//     gives its L2/L3 blocking, Eq. 3-4);
//   * the k (kc) loop becomes the in-kernel loop over BK-deep K-panels;
//   * "pack A" / "pack B" (Algorithm 1, Section 3.1) become the copy of one
//     BM x BK panel of op(A) and one BK x BN panel of op(B) from HBM into LDS,
//     in the order the micro-kernel reads them.  The stored layout (N or T)
//     only changes how the copy reads global memory: after packing every
//     layout looks the same, which is how the paper absorbs transposition in
//     the packing step.  Out-of-range rows, columns and K entries are packed as
//     zeros (the remainder rule of Section 3.1);
//   * the jj/ii/kk loops and the matrix intrinsic (Algorithm 2) become the
//     wave micro-kernel: each wave keeps a WM x WN block of C in registers for
//     the whole K loop as (WM/32) x (WN/32) accumulators of 32x32, and every
//     operand register fetched from LDS feeds a whole row or column of
//     accumulators (the VAccs x HAccs reuse of Algorithm 2);
//   * the C update (Algorithm 1, after the kk loop) is fused into one epilogue
//     C = alpha*acc + beta*C0 applied once after the full K, with C0 not read
//     when beta == 0.
//
// Packed LDS layout.  Both panels are stored "k-major": row k of the A panel
// holds the BM values op(A)[m0 .. m0+BM)[k], row k of the B panel the BN values
// op(B)[k][n0 .. n0+BN).  A lane of a wave reads V = WM/32 consecutive floats of
// one A row in one instruction; value j of lane c belongs to accumulator row
// block j, row c, i.e. row m = wm0 + V*c + j (row blocks are interleaved).  The
// same holds for B with H = WN/32.  The interleave makes each fragment read a
// single 4*V-byte LDS access over contiguous addresses (no bank conflicts) and
// lets the epilogue write H consecutive columns per lane.
//
// Bank swizzle.  Panel rows are BM or BN floats, a multiple of the 64 LDS
// banks, so without a remedy the transposing pack (a K-contiguous source,
// e.g. op(A) = A stored M x K) writes four k-rows at the same banks.  The
// m (n) offset of every element of row k is therefore XORed with
// panel_swizzle(k), a multiple of 64 / (BK/4) below 64 that changes with k/4:
// the 64 lanes of one pack store then hit 64 distinct banks, while every
// aligned group of 4 consecutive m (n) stays together (the fragment reads and
// the 16-byte k-major stores are unchanged in shape).
//
// MFMA 32x32x2 f32 operand layout (per lane l of 64): A supplies
// op(A)[row l%32][k l/32], B supplies op(B)[k l/32][col l%32]; result register
// r of lane l is C[row 8*(r/4) + 4*(l/32) + r%4][col l%32].
#include <type_traits>

#include "common.h"

namespace mg {

template <int BK>
MG_DEVICE constexpr int panel_swizzle(int k)
{
    constexpr int NC = BK / 4;   // 4-float chunks per stored row of a transposing panel
    return ((k >> 2) % NC) * (64 / NC);
}

// ---------------------------------------------------------------------------
// Global -> register staging of one panel, in the stored layout.
//
// The stored panel is SR x SC floats (SR stored rows, SC stored columns, SC a
// multiple of 4) starting at (r0, c0) of a stored matrix with R x Cn valid
// entries and row stride ld.  Thread t fetches chunks q = t + s*NT, each four
// consecutive stored columns of one stored row.  Out-of-range entries read 0.
template <int SR, int SC, int NT>
struct PanelLoader {
    static constexpr int CHUNKS = SR * SC / 4;
    static constexpr int PER_THREAD = (CHUNKS + NT - 1) / NT;
    static_assert(CHUNKS % NT == 0, "panel must split evenly over the workgroup");

    floatx4 v[PER_THREAD];

    MG_DEVICE void load(const float* __restrict__ src, int64_t ld, int64_t r0, int64_t c0,
                        int64_t R, int64_t Cn, bool vec, int tid)
    {
        // Wave-uniform test: an interior panel with 16-byte access takes the
        // branch-free path, so all its loads are in flight at once; edge
        // panels take the guarded path.
        if (vec && r0 + SR <= R && c0 + SC <= Cn) {
            // uniform base + 32-bit per-lane offset (vec guarantees it fits)
            const float* __restrict__ base = src + r0 * ld + c0;
            const uint32_t ld32 = uint32_t(ld);
#pragma unroll
            for (int s = 0; s < PER_THREAD; ++s) {
                const int q = tid + s * NT;
                const uint32_t r = q / (SC / 4), c = (q % (SC / 4)) * 4;
                v[s] = load16(base, (r * ld32 + c) * 4u);
            }
        } else {
#pragma unroll
            for (int s = 0; s < PER_THREAD; ++s) {
                const int q = tid + s * NT;
                const int r = q / (SC / 4), c = (q % (SC / 4)) * 4;
                v[s] = fetch4_guarded(src, ld, r0 + r, c0 + c, R, Cn, vec);
            }
        }
    }

    // Write into a k-major LDS panel with row length L (floats), swizzled by
    // panel_swizzle.  kmajor_src: the stored rows are k (stored columns are m
    // or n), so a chunk is four consecutive m/n of one k row and is written as
    // one 16-byte store.  Otherwise the stored rows are m/n and a chunk is four
    // consecutive k of one m/n: it is transposed into four 4-byte stores.
    template <bool KMAJOR_SRC, int L>
    MG_DEVICE void store(float* lds, int tid) const
    {
        constexpr int BK = KMAJOR_SRC ? SR : SC;
#pragma unroll
        for (int s = 0; s < PER_THREAD; ++s) {
            const int q = tid + s * NT;
            const int r = q / (SC / 4);
            const int c = (q % (SC / 4)) * 4;
            if (KMAJOR_SRC) {
                *reinterpret_cast<floatx4*>(lds + r * L + (c ^ panel_swizzle<BK>(r))) = v[s];
            } else {
                const int m = r ^ panel_swizzle<BK>(c);   // same for k = c .. c+3
                lds[(c + 0) * L + m] = v[s][0];
                lds[(c + 1) * L + m] = v[s][1];
                lds[(c + 2) * L + m] = v[s][2];
                lds[(c + 3) * L + m] = v[s][3];
            }
        }
    }
};

template <int V>
MG_DEVICE void lds_read(const float* p, float (&out)[V])
{
    if constexpr (V == 4) {
        floatx4 t = *reinterpret_cast<const floatx4*>(p);
        out[0] = t[0]; out[1] = t[1]; out[2] = t[2]; out[3] = t[3];
    } else if constexpr (V == 2) {
        floatx2 t = *reinterpret_cast<const floatx2*>(p);
        out[0] = t[0]; out[1] = t[1];
    } else {
        out[0] = p[0];
    }
}

// ---------------------------------------------------------------------------
// LDS floats one tile configuration needs (two stages of both panels, per
// K group).
template <int BM, int BN, int BK, int KG = 1>
constexpr int sgemm_lds_floats() { return KG * 2 * BK * (BM + BN); }

// One BM x BN output tile (tm, tn) of the GEMM in g, computed by the whole
// workgroup ((BM/WM) * (BN/WN) waves).  smem: sgemm_lds_floats() floats of LDS,
// 16-byte aligned.  Ends with a workgroup barrier after the last LDS read, so
// the caller may reuse smem for another tile right away.
//
// SYR2K: the K loop runs twice, first over op(A) x op(B), then over the same
// panels with the roles of A and B exchanged (A read with B's stride as the
// left operand, B with A's as the right one), accumulating both products into
// the same registers: alpha*(X Y^T + Y X^T) for the symmetric rank-2k update
// of Section 5.1 (M == N, both operands of one shape).  UPLO 1 (2) stores
// only the entries with m >= n (m <= n) of the tile.
//
// DEEP: two register staging sets, so each panel is fetched one and a half
// panels before it is packed (instead of half a panel).  The small tiles
// (one wave per SIMD, a short K loop per panel) otherwise wait out most of a
// global load's latency on every panel; their staging sets are small.
//
// KG > 1: the workgroup is KG groups of (BM/WM) * (BN/WN) waves; group q
// multiplies the panels p0 + q, p0 + q + KG, ... out of its own LDS buffers
// into its own accumulators, and at the end the groups' sums are added
// through LDS (group 0 first, then 1, ...) before group 0's epilogue.  A
// small tile then has KG waves per SIMD to hide latency with, without a
// second launch for a split K.  (GEMM only: SYR2K keeps KG = 1.)
template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, bool SYR2K = false, int UPLO = 0,
          bool DEEP = false, int KG = 1>
MG_DEVICE void sgemm_tile(const GemmArgs& g, int tm, int tn, float* smem)
{
    static_assert(KG == 1 || !SYR2K, "SYR2K runs one K group");
    constexpr int WAVES_N = BN / WN;
    constexpr int NT = (BM / WM) * WAVES_N * 64;   // threads of one K group
    constexpr int V = WM / 32;   // accumulator row blocks per wave
    constexpr int H = WN / 32;   // accumulator column blocks per wave
    static_assert(V == 1 || V == 2 || V == 4, "WM must be 32, 64 or 128");
    static_assert(H == 1 || H == 2 || H == 4, "WN must be 32, 64 or 128");
    static_assert(BK % 2 == 0, "BK must be a multiple of the MFMA depth");

    // K group of this wave (uniform across the wave) and its LDS buffers
    const int grp = KG > 1 ? int(threadIdx.x) / NT : 0;
    float* gsmem = smem + grp * (2 * BK * (BM + BN));
    float (*As)[BK * BM] = reinterpret_cast<float (*)[BK * BM]>(gsmem);
    float (*Bs)[BK * BN] = reinterpret_cast<float (*)[BK * BN]>(gsmem + 2 * BK * BM);

    const int tid = KG > 1 ? int(threadIdx.x) % NT : int(threadIdx.x);   // thread within the group
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm0 = (wave / WAVES_N) * WM;
    const int wn0 = (wave % WAVES_N) * WN;
    const int c = lane & 31;     // column of the MFMA operand / result
    const int h = lane >> 5;     // which k of the pair this lane supplies

    const int64_t m0 = int64_t(tm) * BM;
    const int64_t n0 = int64_t(tn) * BN;

    // Stored panels: A is M x K ('N') or K x M ('T'); B is K x N ('N') or N x K ('T').
    using LA = PanelLoader<TA ? BK : BM, TA ? BM : BK, NT>;
    using LB = PanelLoader<TB ? BN : BK, TB ? BK : BN, NT>;
    LA la[DEEP ? 2 : 1];
    LB lb[DEEP ? 2 : 1];
    const int64_t Ra = TA ? g.K : g.M, Ca = TA ? g.M : g.K;
    const int64_t Rb = TB ? g.N : g.K, Cb = TB ? g.K : g.N;

    // Panel p of the K loop: segment p / nk (SYR2K's second product swaps
    // the operands), k0 = (p % nk) * BK.
    const int nk = int((g.K + BK - 1) / BK);
    // set: the staging set (a compile-time constant, so the sets stay in
    // registers)
    auto fetch = [&](int p, auto set) {
        const bool swap = SYR2K && p >= nk;
        const int64_t k0 = int64_t(swap ? p - nk : p) * BK;
        const float* __restrict__ xa = swap ? g.B : g.A;
        const float* __restrict__ xb = swap ? g.A : g.B;
        const int64_t lxa = swap ? g.ldb : g.lda, lxb = swap ? g.lda : g.ldb;
        const bool va = swap ? g.vec_b : g.vec_a, vb = swap ? g.vec_a : g.vec_b;
        if (TA) la[set].load(xa, lxa, k0, m0, Ra, Ca, va, tid);
        else    la[set].load(xa, lxa, m0, k0, Ra, Ca, va, tid);
        if (TB) lb[set].load(xb, lxb, n0, k0, Rb, Cb, vb, tid);
        else    lb[set].load(xb, lxb, k0, n0, Rb, Cb, vb, tid);
    };
    auto pack = [&](int buf, auto set) {
        la[set].template store<TA, BM>(As[buf], tid);
        lb[set].template store<!TB, BN>(Bs[buf], tid);
    };
    using Set0 = std::integral_constant<int, 0>;
    using Set1 = std::integral_constant<int, DEEP ? 1 : 0>;

    floatx16 acc[V][H];
#pragma unroll
    for (int i = 0; i < V; ++i)
#pragma unroll
        for (int j = 0; j < H; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    // Panels [p0, p1) of the whole K loop.  A split SYR2K (gridDim.y > 1)
    // gives workgroup row s the range of k_chunk panels starting at s*k_chunk;
    // GEMM splits offset the operands instead (split_k_view) and run it all.
    int p0 = 0, p1 = SYR2K ? 2 * nk : nk;
    if (SYR2K && gridDim.y > 1) {
        p0 = int(blockIdx.y * g.k_chunk);
        p1 = min(p1, int(p0 + g.k_chunk));
    }
    // This group's panels: p0 + grp, then every KG-th.  With KG > 1 the
    // loop below indexes them by their position i = 0, 1, ... in the
    // group's sequence and the groups run the same number of iterations
    // (a group past its last panel only joins the barriers).
    p0 += grp;
    const int step = KG;
    // Panel p is staged in set ((p - p0) / KG) & 1 (DEEP) or set 0, and
    // multiplied from LDS buffer ((p - p0) / KG) & 1 of the group.
    if (p0 < p1) {
        fetch(p0, Set0{});
        pack(0, Set0{});
        if (DEEP && p0 + step < p1) fetch(p0 + step, Set1{});
    }
    __syncthreads();

    constexpr int STEPS = BK / 2;          // MFMA k-steps per panel
    constexpr int PACK_AT = STEPS / 2;     // the next panel is packed half-way
    // One panel: LDS buffer cur holds panel kt.  DEEP: fetch panel kt + 2
    // into set_cur (its panel kt went to LDS one iteration ago) and pack
    // panel kt + 1 from set_next; otherwise fetch panel kt + 1 into the one
    // set and pack it half-way.
    auto panel = [&](int kt, int cur, auto set_cur, auto set_next) {
        using SetNext = decltype(set_next);
        using SetCur = decltype(set_cur);
        if (KG > 1 && kt >= p1) {
            // this group has no panel left: only the barrier
            __syncthreads();
            return;
        }
        if (DEEP) {
            if (kt + 2 * step < p1) fetch(kt + 2 * step, SetCur{});
        } else {
            if (kt + step < p1) fetch(kt + step, SetCur{});
        }

        const float* a_rows = As[cur] + h * BM;
        const float* b_rows = Bs[cur] + h * BN;
        const int am = wm0 + V * c, bnn = wn0 + H * c;
        // Rows k = 2s and 2s+1 share their swizzle (it changes with k/4), so
        // the swizzle of a step is a compile-time constant.
        auto a_at = [&](int s) { return a_rows + 2 * s * BM + (am ^ panel_swizzle<BK>(2 * s)); };
        auto b_at = [&](int s) { return b_rows + 2 * s * BN + (bnn ^ panel_swizzle<BK>(2 * s)); };
        // Software pipeline: the fragments of step s+1 are read from LDS
        // before the MFMAs of step s are issued, into separate registers, so
        // LDS latency hides behind the matrix core.
        float a[V], b[H];
        lds_read<V>(a_at(0), a);
        lds_read<H>(b_at(0), b);
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            float an[V], bn[H];
            if (s + 1 < STEPS) {
                lds_read<V>(a_at(s + 1), an);
                lds_read<H>(b_at(s + 1), bn);
            }
            if (s == PACK_AT) {
                // Pack panel kt + 1 into the other LDS buffer (last read
                // before the previous barrier).  On the last panel this
                // rewrites stale data nobody reads.
                pack(cur ^ 1, SetNext{});
            }
#pragma unroll
            for (int i = 0; i < V; ++i)
#pragma unroll
                for (int j = 0; j < H; ++j)
                    acc[i][j] = mfma_f32_32x32x2(a[i], b[j], acc[i][j]);
            if (s + 1 < STEPS) {
#pragma unroll
                for (int i = 0; i < V; ++i) a[i] = an[i];
#pragma unroll
                for (int j = 0; j < H; ++j) b[j] = bn[j];
            }
        }
        __syncthreads();
    };
    if constexpr (KG > 1) {
        // every group runs the iterations of group 0, which has the most panels
        const int base = p0 - grp;
        const int iters = base < p1 ? (p1 - base + KG - 1) / KG : 0;
        if constexpr (DEEP) {
            for (int i = 0; i < iters; i += 2) {
                panel(p0 + i * step, 0, Set0{}, Set1{});
                if (i + 1 < iters) panel(p0 + (i + 1) * step, 1, Set1{}, Set0{});
            }
        } else {
            for (int i = 0; i < iters; ++i) panel(p0 + i * step, i & 1, Set0{}, Set0{});
        }
        // Add the groups' sums through LDS (free after the loop's last
        // barrier): group q > 0 stores its accumulators in turn, group 0
        // adds them, in the order q = 1, 2, ...
        float* red = smem;
        static_assert(BM * BN <= KG * 2 * BK * (BM + BN), "reduction fits the panel buffers");
        const int slot0 = ((wave * V * H) * 16) * 64 + lane;
#pragma unroll 1
        for (int q = 1; q < KG; ++q) {
            if (grp == q) {
#pragma unroll
                for (int i = 0; i < V; ++i)
#pragma unroll
                    for (int j = 0; j < H; ++j)
#pragma unroll
                        for (int r = 0; r < 16; ++r) red[slot0 + ((i * H + j) * 16 + r) * 64] = acc[i][j][r];
            }
            __syncthreads();
            if (grp == 0) {
#pragma unroll
                for (int i = 0; i < V; ++i)
#pragma unroll
                    for (int j = 0; j < H; ++j)
#pragma unroll
                        for (int r = 0; r < 16; ++r) acc[i][j][r] += red[slot0 + ((i * H + j) * 16 + r) * 64];
            }
            __syncthreads();
        }
        if (grp != 0) return;
    } else if constexpr (DEEP) {
        // unrolled by two so that the staging set of each panel is a
        // compile-time choice
        for (int kt = p0; kt < p1; kt += 2) {
            panel(kt, 0, Set0{}, Set1{});
            if (kt + 1 < p1) panel(kt + 1, 1, Set1{}, Set0{});
        }
    } else {
        for (int kt = p0; kt < p1; ++kt) panel(kt, (kt - p0) & 1, Set0{}, Set0{});
    }

    // Epilogue: C = alpha*acc + beta*C0, once per element.  C0 is read
    // through the pointer C is written through, so loads placed between the
    // stores could not be moved ahead of them and each would wait a whole
    // memory round trip; the C0 values of one accumulator block row (half of
    // it for the largest grids) are therefore all loaded first, then stored.
    const float alpha = g.alpha, beta = g.beta;
    const int64_t ncol = n0 + wn0 + H * c;   // first of this lane's H columns
    auto row_of = [&](int i, int r) { return m0 + wm0 + V * (8 * (r >> 2) + 4 * h + (r & 3)) + i; };
    // columns ncol .. ncol+H-1 all inside the stored triangle
    auto whole = [&](int64_t m) { return UPLO == 0 || (UPLO == 1 ? ncol + H - 1 <= m : ncol >= m); };
    // one 16-byte (H = 4) or 8-byte (H = 2) access per row: vec_c makes
    // C and ldc 16-byte aligned and ncol is a multiple of H
    auto vec_row = [&](int64_t m) { return (H == 4 || H == 2) && g.vec_c && ncol + H - 1 < g.N && whole(m); };
    auto inside = [&](int64_t m, int j) {
        return ncol + j < g.N && (UPLO == 0 || (UPLO == 1 ? ncol + j <= m : ncol + j >= m));
    };
    // rows per batch: half a block row for the largest accumulator grids,
    // whose registers leave no room for 16 x H loaded values and addresses
    constexpr int RB = V * H >= 16 ? 4 : 16;
#pragma unroll
    for (int i = 0; i < V; ++i) {
#pragma unroll
        for (int r0 = 0; r0 < 16; r0 += RB) {
            float c0[RB][H];
            if (beta != 0.f) {
                // Out-of-range rows and columns read a clamped in-range
                // element that is never stored (nor is anything outside the
                // triangle), so the loads need no branches.
                const bool vec = (H == 4 || H == 2) && g.vec_c && ncol + H - 1 < g.N;
#pragma unroll
                for (int rr = 0; rr < RB; ++rr) {
                    const int64_t m = row_of(i, r0 + rr);
                    const float* cp = g.C + (m < g.M ? m : g.M - 1) * g.ldc;
                    if (vec) {
                        if constexpr (H == 4) {
                            const floatx4 v = *reinterpret_cast<const floatx4*>(cp + ncol);
#pragma unroll
                            for (int j = 0; j < H; ++j) c0[rr][j] = v[j];
                        } else if constexpr (H == 2) {
                            const floatx2 v = *reinterpret_cast<const floatx2*>(cp + ncol);
#pragma unroll
                            for (int j = 0; j < H; ++j) c0[rr][j] = v[j];
                        }
                    } else {
#pragma unroll
                        for (int j = 0; j < H; ++j) c0[rr][j] = cp[ncol + j < g.N ? ncol + j : g.N - 1];
                    }
                }
            }
#pragma unroll
            for (int rr = 0; rr < RB; ++rr) {
                const int r = r0 + rr;
                const int64_t m = row_of(i, r);
                if (m >= g.M) continue;
                float* cp = g.C + m * g.ldc + ncol;
                float o[H];
#pragma unroll
                for (int j = 0; j < H; ++j)
                    o[j] = beta != 0.f ? __builtin_fmaf(alpha, acc[i][j][r], beta * c0[rr][j]) : alpha * acc[i][j][r];
                if (vec_row(m)) {
                    if constexpr (H == 4) {
                        const floatx4 v = {o[0], o[1], o[2], o[3]};
                        *reinterpret_cast<floatx4*>(cp) = v;
                    } else if constexpr (H == 2) {
                        const floatx2 v = {o[0], o[1]};
                        *reinterpret_cast<floatx2*>(cp) = v;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < H; ++j)
                        if (inside(m, j)) cp[j] = o[j];
                }
            }
        }
    }
}

}  // namespace mg
