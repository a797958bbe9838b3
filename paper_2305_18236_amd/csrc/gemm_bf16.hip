// BF16 and bf16x3 GEMM kernels and launchers: one workgroup per output tile
// of the scheme in tile_bf16.h, plus the stand-alone pack-stage conversion.
#include "tile_bf16.h"
#include "tile_bytes.h"
#include "kernels.h"

namespace mg {

template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, int TERMS>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64)
void gemm_bf16_kernel(GemmArgs args)
{
    __shared__ __attribute__((aligned(16))) uint16_t smem[bf16_lds_elems<BM, BN, BK, TERMS>()];
    GemmArgs g = args;
    split_k_view<TA, TB, false>(g);
    int tm, tn;
    tile_of(blockIdx.x, g.tiles_m, g.tiles_n, g.group_m, g.remap, tm, tn);
    bf16_tile<BM, BN, BK, WM, WN, TA, TB, TERMS>(g, tm, tn, smem);
}

// GEMM on operands pre-packed by bf16_pack_kernel (no conversion, no bounds
// checks on loads; the epilogue still clips to M x N).
template <int BM, int BN, int BK, int WM, int WN, int TERMS>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64)
void gemm_bf16_packed_kernel(GemmArgs args)
{
    __shared__ __attribute__((aligned(16))) uint16_t smem[bf16_lds_elems<BM, BN, BK, TERMS>()];
    GemmArgs g = args;
    split_k_view<false, true, true>(g);
    int tm, tn;
    tile_of(blockIdx.x, g.tiles_m, g.tiles_n, g.group_m, g.remap, tm, tn);
    bf16_tile<BM, BN, BK, WM, WN, false, true, TERMS, true>(g, tm, tn, smem);
}

// Direct form on pre-packed planes (direct_copy in tile_bytes.h): each K
// panel is one 128-byte row per row of op(A) and op(B)^T, copied from the
// planes straight into LDS while the previous panel is multiplied, with no
// register staging and no LDS write instructions.  Single-term planes hold
// 64 k per row; bf16x3's interleaved planes (launch_bf16_pack_interleaved)
// hold 32 k of both terms, hi in global chunks 0-3 and lo in 4-7.  The two
// buffers are separate arrays used in a fixed alternation, so the compiler
// can tell the copy into one from the reads of the other.  The planes are
// zero-padded to whole 256-row tiles and 128-deep K grains, so every copy is
// in bounds and the padding adds zeros.  Each 16-deep step issues its
// products in the order the staged kernel does (bf16x3: lo(A) hi(B),
// hi(A) lo(B), hi(A) hi(B)), so the results are bit-identical to it.
template <int BM, int BN, int WM, int WN, int TERMS>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64)
void gemm_bf16_direct_kernel(GemmArgs args)
{
    constexpr int BK = TERMS == 3 ? 32 : 64;  // k per 128-byte panel row
    constexpr int KBYTES = 128 / BK;          // bytes per k in a plane row
    constexpr int STEPS = BK / 16;
    constexpr int WAVES_N = BN / WN;
    constexpr int NW = (BM / WM) * WAVES_N;
    constexpr int V = WM / 32, H = WN / 32;

    __shared__ __attribute__((aligned(1024))) uint8_t A0[BM * 128];
    __shared__ __attribute__((aligned(1024))) uint8_t A1[BM * 128];
    __shared__ __attribute__((aligned(1024))) uint8_t B0[BN * 128];
    __shared__ __attribute__((aligned(1024))) uint8_t B1[BN * 128];

    GemmArgs g = args;
    int64_t kbyte0 = 0;
    if (gridDim.y > 1) {
        // split K: workgroup row s multiplies the range [s k_chunk, ...) and
        // stores its unscaled partial product (reduced afterwards)
        const int64_t k0 = int64_t(blockIdx.y) * g.k_chunk;
        g.K = min(g.k_chunk, g.K - k0);
        kbyte0 = KBYTES * k0;
        g.C = g.part + int64_t(blockIdx.y) * g.part_stride;
        g.ldc = g.ldp;
        g.alpha = 1.f;
        g.beta = 0.f;
    }
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / WAVES_N) * WM, wn0 = (wave % WAVES_N) * WN;
    const int c = lane & 31, h = lane >> 5;

    int tm, tn;
    tile_of(blockIdx.x, g.tiles_m, g.tiles_n, g.group_m, g.remap, tm, tn);
    const int64_t m0 = int64_t(tm) * BM, n0 = int64_t(tn) * BN;
    const uint8_t* __restrict__ qa =
        reinterpret_cast<const uint8_t*>(reinterpret_cast<const uint16_t*>(g.A) + m0 * g.lda) + kbyte0;
    const uint8_t* __restrict__ qb =
        reinterpret_cast<const uint8_t*>(reinterpret_cast<const uint16_t*>(g.B) + n0 * g.ldb) + kbyte0;
    const uint32_t lda32 = uint32_t(2 * g.lda), ldb32 = uint32_t(2 * g.ldb);

    floatx16 acc[V][H];
#pragma unroll
    for (int i = 0; i < V; ++i)
#pragma unroll
        for (int j = 0; j < H; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    auto copy_panel = [&](uint8_t* LA, uint8_t* LB, int kp) {
        direct_copy<BM, NW>(qa, lda32, uint32_t(kp) * 128u, LA, wave, lane);
        direct_copy<BN, NW>(qb, ldb32, uint32_t(kp) * 128u, LB, wave, lane);
    };
    auto chunk = [&](const uint8_t* L, int row, int g) { return __builtin_bit_cast(bf16x8, direct_chunk(L, row, g)); };
    auto panel = [&](const uint8_t* LA, const uint8_t* LB) {
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            // lane (c, h) supplies k 16s + 8h .. +7 of row c: global chunk
            // 2s + h (bf16x3: hi there, lo in chunk 4 + 2s + h)
            if constexpr (TERMS == 3) {
                bf16x8 ah[V], al[V], bh[H], bl[H];
#pragma unroll
                for (int j = 0; j < H; ++j) {
                    bh[j] = chunk(LB, wn0 + 32 * j + c, 2 * s + h);
                    bl[j] = chunk(LB, wn0 + 32 * j + c, 4 + 2 * s + h);
                }
#pragma unroll
                for (int i = 0; i < V; ++i) {
                    ah[i] = chunk(LA, wm0 + 32 * i + c, 2 * s + h);
                    al[i] = chunk(LA, wm0 + 32 * i + c, 4 + 2 * s + h);
                }
#pragma unroll
                for (int i = 0; i < V; ++i)
#pragma unroll
                    for (int j = 0; j < H; ++j) acc[i][j] = mfma16<3>(al[i], bh[j], acc[i][j]);
#pragma unroll
                for (int i = 0; i < V; ++i)
#pragma unroll
                    for (int j = 0; j < H; ++j) acc[i][j] = mfma16<3>(ah[i], bl[j], acc[i][j]);
#pragma unroll
                for (int i = 0; i < V; ++i)
#pragma unroll
                    for (int j = 0; j < H; ++j) acc[i][j] = mfma16<3>(ah[i], bh[j], acc[i][j]);
            } else {
                bf16x8 a[V], b[H];
#pragma unroll
                for (int i = 0; i < V; ++i) a[i] = chunk(LA, wm0 + 32 * i + c, 2 * s + h);
#pragma unroll
                for (int j = 0; j < H; ++j) b[j] = chunk(LB, wn0 + 32 * j + c, 2 * s + h);
#pragma unroll
                for (int i = 0; i < V; ++i)
#pragma unroll
                    for (int j = 0; j < H; ++j) acc[i][j] = mfma16<TERMS>(a[i], b[j], acc[i][j]);
            }
        }
    };
    // all copies landed in LDS, then every wave past the barrier
    auto arrive = [&]() {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    };

    const int nk = int((g.K + BK - 1) / BK);
    if (nk > 0) {
        copy_panel(A0, B0, 0);
        arrive();
    }
    for (int kt = 0; kt < nk; kt += 2) {
        // panel kt in buffer 0; panel kt+1 is copied into buffer 1 meanwhile
        if (kt + 1 < nk) copy_panel(A1, B1, kt + 1);
        panel(A0, B0);
        arrive();
        if (kt + 1 < nk) {
            if (kt + 2 < nk) copy_panel(A0, B0, kt + 2);
            panel(A1, B1);
            arrive();
        }
    }

    const float alpha = g.alpha, beta = g.beta;
    store_acc_blocks<V, H>(g.C, g.ldc, g.M, g.N, m0 + wm0, n0 + wn0, h, c, beta != 0.f, acc,
                           [&](float a, float c0) { return beta != 0.f ? __builtin_fmaf(alpha, a, beta * c0) : alpha * a; });
}

template <int BM, int BN, int WM, int WN, int TERMS>
static hipError_t launch_bf16_direct(GemmArgs g, hipStream_t stream)
{
    constexpr int NT = (BM / WM) * (BN / WN) * 64;
    g.tiles_m = int((g.M + BM - 1) / BM);
    g.tiles_n = int((g.N + BN - 1) / BN);
    const dim3 grid(g.tiles_m * g.tiles_n, split_count(g)), block(NT);
    hipLaunchKernelGGL((gemm_bf16_direct_kernel<BM, BN, WM, WN, TERMS>), grid, block, 0, stream, g);
    return hipGetLastError();
}

template <int BM, int BN, int BK, int WM, int WN, int TERMS>
static hipError_t launch_bf16_cfg(bool ta, bool tb, GemmArgs g, hipStream_t stream, bool packed)
{
    constexpr int NT = (BM / WM) * (BN / WN) * 64;
    g.tiles_m = int((g.M + BM - 1) / BM);
    g.tiles_n = int((g.N + BN - 1) / BN);
    const dim3 grid(g.tiles_m * g.tiles_n, split_count(g)), block(NT);
    if (packed) hipLaunchKernelGGL((gemm_bf16_packed_kernel<BM, BN, BK, WM, WN, TERMS>), grid, block, 0, stream, g);
    else if (!ta && !tb) hipLaunchKernelGGL((gemm_bf16_kernel<BM, BN, BK, WM, WN, false, false, TERMS>), grid, block, 0, stream, g);
    else if (!ta && tb) hipLaunchKernelGGL((gemm_bf16_kernel<BM, BN, BK, WM, WN, false, true, TERMS>), grid, block, 0, stream, g);
    else if (ta && !tb) hipLaunchKernelGGL((gemm_bf16_kernel<BM, BN, BK, WM, WN, true, false, TERMS>), grid, block, 0, stream, g);
    else hipLaunchKernelGGL((gemm_bf16_kernel<BM, BN, BK, WM, WN, true, true, TERMS>), grid, block, 0, stream, g);
    return hipGetLastError();
}

const SgemmConfig kBf16Configs[] = {
    // id, BM, BN, BK, WM, WN
    {0, 256, 256, 32, 128, 128},
    {1, 256, 256, 32, 128, 64},
    {2, 128, 128, 32, 64, 64},
    {3, 256, 128, 32, 128, 64},
    {4, 64, 64, 32, 32, 32},
    {5, 128, 64, 32, 64, 32},
    // configuration 1's tiles with panels copied straight into LDS, on
    // pre-packed planes (bf16x3: the interleaved ones); without the planes
    // it runs as configuration 1
    {6, 256, 256, 64, 128, 64},
    // configuration 2's tiles with panels copied straight into LDS, on
    // pre-packed planes (64 KiB of LDS: two workgroups per compute unit, so
    // one's epilogue overlaps the other's K loop when K is short); without
    // the planes it runs as configuration 2
    {7, 128, 128, 64, 64, 64},
    // the 128 x 128 tile of configuration 2 over eight waves (64 x 32 or
    // 32 x 64 each): two waves per SIMD
    {8, 128, 128, 32, 64, 32},
    {9, 128, 128, 32, 32, 64},
    // configuration 7's panels copied straight into LDS, over eight 64 x 32
    // waves; without the planes it runs as configuration 8
    {10, 128, 128, 64, 64, 32},
    // configuration 6 over sixteen 64 x 64 waves; without the planes it runs
    // as configuration 1
    {11, 256, 256, 64, 64, 64},
};
const int kNumBf16Configs = sizeof(kBf16Configs) / sizeof(kBf16Configs[0]);

template <int TERMS>
static hipError_t launch_terms(int cfg, bool ta, bool tb, GemmArgs g, hipStream_t stream, bool packed)
{
    switch (cfg) {
    case 0: return launch_bf16_cfg<256, 256, 32, 128, 128, TERMS>(ta, tb, g, stream, packed);
    case 1: return launch_bf16_cfg<256, 256, 32, 128, 64, TERMS>(ta, tb, g, stream, packed);
    case 2: return launch_bf16_cfg<128, 128, 32, 64, 64, TERMS>(ta, tb, g, stream, packed);
    case 3: return launch_bf16_cfg<256, 128, 32, 128, 64, TERMS>(ta, tb, g, stream, packed);
    case 4: return launch_bf16_cfg<64, 64, 32, 32, 32, TERMS>(ta, tb, g, stream, packed);
    case 5: return launch_bf16_cfg<128, 64, 32, 64, 32, TERMS>(ta, tb, g, stream, packed);
    case 6:
        if (packed) return launch_bf16_direct<256, 256, 128, 64, TERMS>(g, stream);
        return launch_bf16_cfg<256, 256, 32, 128, 64, TERMS>(ta, tb, g, stream, packed);
    case 7:
        if (packed) return launch_bf16_direct<128, 128, 64, 64, TERMS>(g, stream);
        return launch_bf16_cfg<128, 128, 32, 64, 64, TERMS>(ta, tb, g, stream, packed);
    case 8: return launch_bf16_cfg<128, 128, 32, 64, 32, TERMS>(ta, tb, g, stream, packed);
    case 9: return launch_bf16_cfg<128, 128, 32, 32, 64, TERMS>(ta, tb, g, stream, packed);
    case 10:
        if (packed) return launch_bf16_direct<128, 128, 64, 32, TERMS>(g, stream);
        return launch_bf16_cfg<128, 128, 32, 64, 32, TERMS>(ta, tb, g, stream, packed);
    case 11:
        if (packed) return launch_bf16_direct<256, 256, 64, 64, TERMS>(g, stream);
        return launch_bf16_cfg<256, 256, 32, 128, 64, TERMS>(ta, tb, g, stream, packed);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gemm_bf16(int terms, int cfg, bool ta, bool tb, GemmArgs g, hipStream_t stream, bool packed)
{
    switch (terms) {
    case 1: return launch_terms<1>(cfg, ta, tb, g, stream, packed);
    case 3: return launch_terms<3>(cfg, ta, tb, g, stream, packed);
    case 16: return launch_terms<16>(cfg, ta, tb, g, stream, packed);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Pre-pack of one operand for the BF16 paths: the logical R x Kd matrix
// op(X) (stored R x Kd when T is false, Kd x R when true) is rounded (TERMS 1:
// bf16, 16: fp16) or split into hi/lo (TERMS 3) once and written as
// k-contiguous 16-bit rows
// hi[Rp][ldq] (and lo[Rp][ldq]), zero outside R x Kd.  One workgroup of 256
// threads per 128 x 128 tile; the tile goes through LDS so that both stored
// layouts write whole 16-byte row chunks.
constexpr int PT = 128;          // pack tile
constexpr int PROW = PT + 8;     // LDS row of the pack tile (bf16), T == false

// T == true: unpadded 128-element rows whose sixteen 16-byte chunks are
// permuted by an XOR with (r >> 2) % 16, so that the 8-byte writes of a
// half-wave (32 rows four apart) meet at most two to a bank and the 16-byte
// reads of the write-out not at all (padded and unswizzled, the writes meet
// eight to a bank).  Returns the element offset of element k of row r.
MG_DEVICE int pt_swizzle(int r, int k) { return 8 * (((k >> 3) ^ (r >> 2)) & 15) + (k & 7); }

// IL (bf16x3 only): one plane whose rows interleave the two terms per 32 k,
// hi(k0 .. k0+31) then lo(k0 .. k0+31), so that a 32-deep panel of both
// terms is one 128-byte row (row stride ldq = 2 Kp elements; `lo` unused).
template <bool T, int TERMS, bool IL = false>
__global__ __launch_bounds__(256) void bf16_pack_kernel(const float* __restrict__ X, int64_t ldx, int64_t R,
                                                        int64_t Kd, int vec, uint16_t* __restrict__ hi,
                                                        uint16_t* __restrict__ lo, int64_t ldq)
{
    static_assert(!IL || TERMS == 3, "interleaving needs two terms");
    constexpr int ROW = T ? PT : PROW;
    __shared__ __attribute__((aligned(16))) uint16_t th[PT * ROW];
    __shared__ __attribute__((aligned(16))) uint16_t tl[TERMS == 3 ? PT * ROW : 8];
    const int tid = threadIdx.x;
    // blockIdx.x runs along the stored rows (over k tiles when T is false,
    // over row tiles of op(X) when T is true), so that consecutive workgroups
    // read neighbouring pieces of the same stored rows (measured: the other
    // order makes either pack about 20 % slower)
    const int64_t k0 = int64_t(T ? blockIdx.y : blockIdx.x) * PT, r0 = int64_t(T ? blockIdx.x : blockIdx.y) * PT;
    const int64_t sr0 = T ? k0 : r0, sc0 = T ? r0 : k0;      // stored tile origin
    const int64_t SRn = T ? Kd : R, SCn = T ? R : Kd;         // stored valid extent
    // 16 chunks of 4 floats per thread.  T == false: chunk s is stored row
    // id / 32, stored columns 4*(id % 32) .. +3, id = tid + 256*s.  T == true:
    // chunks 4b .. 4b+3 are the 4 x 4 block of stored rows 4*(id / 32) .. +3
    // (four k) and stored columns 4*(id % 32) .. +3 (four logical rows),
    // id = tid + 256*b, so each logical row's four k become one 8-byte write.
    auto stored_row = [&](int s) { return T ? 4 * ((tid + 256 * (s >> 2)) / 32) + (s & 3) : (tid + 256 * s) / 32; };
    auto stored_col = [&](int s) { return T ? 4 * ((tid + 256 * (s >> 2)) % 32) : 4 * ((tid + 256 * s) % 32); };
    floatx4 v[16];
    if (vec && sr0 + PT <= SRn && sc0 + PT <= SCn) {          // wave-uniform: interior tile
        const float* __restrict__ base = X + sr0 * ldx + sc0;
        const uint32_t ld32 = uint32_t(ldx);
#pragma unroll
        for (int s = 0; s < 16; ++s) v[s] = load16(base, (uint32_t(stored_row(s)) * ld32 + uint32_t(stored_col(s))) * 4u);
    } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) v[s] = fetch4_guarded(X, ldx, sr0 + stored_row(s), sc0 + stored_col(s), SRn, SCn, vec);
    }
    auto convert = [&](floatx4 x, uint32_t (&h)[2], uint32_t (&l)[2]) {
        if constexpr (TERMS == 3) split4(x, h, l);
        else convert4<TERMS>(x, h);
    };
    if (!T) {
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            // stored row = logical row, columns = k .. k+3
            uint32_t h[2], l[2];
            convert(v[s], h, l);
            const int off = stored_row(s) * PROW + stored_col(s);
            *reinterpret_cast<uint2*>(&th[off]) = make_uint2(h[0], h[1]);
            if (TERMS == 3) *reinterpret_cast<uint2*>(&tl[off]) = make_uint2(l[0], l[1]);
        }
    } else {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int id = tid + 256 * b;
            const int kk = 4 * (id / 32);            // first k of the block
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int r = 4 * (id % 32) + c;     // logical row
                const floatx4 x = {v[4 * b][c], v[4 * b + 1][c], v[4 * b + 2][c], v[4 * b + 3][c]};
                uint32_t h[2], l[2];
                convert(x, h, l);
                const int off = r * PT + pt_swizzle(r, kk);
                *reinterpret_cast<uint2*>(&th[off]) = make_uint2(h[0], h[1]);
                if (TERMS == 3) *reinterpret_cast<uint2*>(&tl[off]) = make_uint2(l[0], l[1]);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int id = tid + 256 * s;
        const int r = id / 16, c = 8 * (id % 16);
        const int off = T ? r * PT + pt_swizzle(r, c) : r * PROW + c;
        if constexpr (IL) {
            // k = k0 + c .. +7 lies inside one 32-k group (c % 8 == 0)
            const int64_t k = k0 + c;
            uint16_t* dst = hi + (r0 + r) * ldq + 64 * (k >> 5) + (k & 31);
            *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<const uint4*>(&th[off]);
            *reinterpret_cast<uint4*>(dst + 32) = *reinterpret_cast<const uint4*>(&tl[off]);
        } else {
            *reinterpret_cast<uint4*>(hi + (r0 + r) * ldq + k0 + c) = *reinterpret_cast<const uint4*>(&th[off]);
            if (TERMS == 3)
                *reinterpret_cast<uint4*>(lo + (r0 + r) * ldq + k0 + c) = *reinterpret_cast<const uint4*>(&tl[off]);
        }
    }
}

hipError_t launch_bf16_pack(bool trans, int terms, const float* X, int64_t ldx, int64_t R, int64_t Kd,
                            bool vec, uint16_t* hi, uint16_t* lo, int64_t ldq, int64_t Rp, int64_t Kp,
                            hipStream_t stream)
{
    const dim3 grid(unsigned(trans ? Rp / PT : Kp / PT), unsigned(trans ? Kp / PT : Rp / PT)), block(256);
    switch (terms) {
    case 3:
        if (trans) hipLaunchKernelGGL((bf16_pack_kernel<true, 3>), grid, block, 0, stream, X, ldx, R, Kd, int(vec), hi, lo, ldq);
        else hipLaunchKernelGGL((bf16_pack_kernel<false, 3>), grid, block, 0, stream, X, ldx, R, Kd, int(vec), hi, lo, ldq);
        break;
    case 1:
        if (trans) hipLaunchKernelGGL((bf16_pack_kernel<true, 1>), grid, block, 0, stream, X, ldx, R, Kd, int(vec), hi, lo, ldq);
        else hipLaunchKernelGGL((bf16_pack_kernel<false, 1>), grid, block, 0, stream, X, ldx, R, Kd, int(vec), hi, lo, ldq);
        break;
    case 16:
        if (trans) hipLaunchKernelGGL((bf16_pack_kernel<true, 16>), grid, block, 0, stream, X, ldx, R, Kd, int(vec), hi, lo, ldq);
        else hipLaunchKernelGGL((bf16_pack_kernel<false, 16>), grid, block, 0, stream, X, ldx, R, Kd, int(vec), hi, lo, ldq);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// bf16x3 pack into one plane per operand with the two terms interleaved per
// 32 k (row stride ldq = 2 Kp elements).
hipError_t launch_bf16_pack_interleaved(bool trans, const float* X, int64_t ldx, int64_t R, int64_t Kd, bool vec,
                                        uint16_t* q, int64_t ldq, int64_t Rp, int64_t Kp, hipStream_t stream)
{
    const dim3 grid(unsigned(trans ? Rp / PT : Kp / PT), unsigned(trans ? Kp / PT : Rp / PT)), block(256);
    if (trans) hipLaunchKernelGGL((bf16_pack_kernel<true, 3, true>), grid, block, 0, stream, X, ldx, R, Kd, int(vec), q, nullptr, ldq);
    else hipLaunchKernelGGL((bf16_pack_kernel<false, 3, true>), grid, block, 0, stream, X, ldx, R, Kd, int(vec), q, nullptr, ldq);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The pack stage's conversion on its own, for bit-exact checks: hi = bf16(x),
// lo = bf16(x - hi) (lo is written only when lo != nullptr).
__global__ __launch_bounds__(256) void bf16_split_kernel(const float* __restrict__ x, int64_t n,
                                                         uint16_t* __restrict__ hi, uint16_t* __restrict__ lo)
{
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
         t += int64_t(gridDim.x) * blockDim.x) {
        const float v = x[t];
        const uint32_t h = pack_bf16x2(v, 0.f);
        hi[t] = uint16_t(h & 0xffffu);
        if (lo) {
            const float hf = __builtin_bit_cast(float, h << 16);
            lo[t] = uint16_t(pack_bf16x2(v - hf, 0.f) & 0xffffu);
        }
    }
}

hipError_t launch_bf16_split(const float* x, int64_t n, uint16_t* hi, uint16_t* lo, hipStream_t stream)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(bf16_split_kernel, dim3(unsigned(blocks)), dim3(256), 0, stream, x, n, hi, lo);
    return hipGetLastError();
}

}  // namespace mg
