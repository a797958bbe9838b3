// FP8 path: OCP E4M3 operands with one power-of-two FP32 scale per 128 x 128
// tile, FP32 accumulation, on the scaled FP8 matrix cores of gfx950
// (v_mfma_scale_f32_32x32x64_f8f6f4).
//
// Two stages, following Algorithm 1 of Kuzma et al. (SPE 2023):
//
// 1. Pack (fp8_pack_kernel).  Where the paper packs each block of A and B
//    into a buffer in main memory in the micro-kernel's access order
//    (Section 3.1), this stage packs all of op(A) (M x K) and op(B)^T (N x K)
//    once into a caller-provided HBM workspace, quantised: for every
//    128 x 128 tile, amax -> s = the smallest power of two with
//    amax <= 448*s, q = E4M3(x / s) (x / s is exact: s is a power of two, and
//    |x / s| <= 448 so no value saturates).  Rows are k-contiguous, rows are
//    padded to a multiple of 256 and K to a multiple of 128 with zeros, so the
//    GEMM needs no bounds checks on its loads.  The scale is kept as its
//    E8M0 byte (exponent + 127).  One FP8 rank-4 update per 8-bit element
//    group is Table 1's 8-bit row; gfx950's instruction is rank-64.
//
// 2. GEMM (gemm_fp8_kernel).  Workgroup tiles, an in-kernel loop over
//    128-deep K-panels (one scale block per panel), packed panels copied into
//    LDS with 16-byte loads, and a wave micro-kernel whose accumulators live
//    for the whole K loop.  A wave's 32-row (32-column) MFMA block lies in one
//    128-row tile of op(A) (op(B)^T), and each 64-deep K step lies in one
//    128-deep scale block, so every lane of the wave passes the same scale
//    byte to the scaled MFMA, which multiplies the block product by
//    2^(ea-127) * 2^(eb-127) exactly before accumulating.
//
// Packed layout (also documented in include/mgemm.h):
//   q:      Rp x Kp bytes, row r holds E4M3 codes of op(X)[r][0..Kp)
//   scales: (Rp/128) x (Kp/128) E8M0 bytes, row-major
//   Rp = roundup(R, 256), Kp = roundup(K, 128).
#include "common.h"
#include "kernels.h"
#include "tile_bytes.h"
#include "epilogue.h"

namespace mg {

constexpr int QT = 128;       // quantisation tile
constexpr int QROW = 128 + 16; // LDS row of the transpose buffer (bytes)

MG_DEVICE float wave_max(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    return v;
}

// Smallest E with amax <= 448 * 2^E (E = 0 for amax == 0), clamped to the
// E8M0 range; returned as the E8M0 byte E + 127.
MG_DEVICE int scale_byte(float amax)
{
    if (!(amax > 0.f)) return 127;
    int e;
    const float f = frexpf(amax, &e);   // amax = f * 2^e, f in [0.5, 1); 448 = 0.875 * 2^9
    int E = (f <= 0.875f) ? e - 9 : e - 8;
    if (E < -127) E = -127;
    if (E > 127) E = 127;
    return E + 127;
}

// Byte offset, within LDS row r of the transposing pack's tile, of byte k of
// the row: the row's eight 16-byte chunks are permuted by an XOR with
// ((r >> 2) + (r >> 5)) % 8, so that the 4-byte writes of a wave (32 rows
// four apart, two k words) and the 16-byte reads of the write-out meet at
// most two to a bank (unswizzled, the writes meet eight to a bank).
MG_DEVICE int qt_swizzle(int r, int k) { return 16 * (((k >> 4) ^ ((r >> 2) + (r >> 5))) & 7) + (k & 15); }

// One workgroup of 256 threads per 128 x 128 tile of the logical R x Kd matrix
// op(X).  T == false: X stored R x Kd (k contiguous); T == true: stored Kd x R.
template <bool T>
__global__ __launch_bounds__(256) void fp8_pack_kernel(const float* __restrict__ X, int64_t ldx,
                                                       int64_t R, int64_t Kd, int vec,
                                                       uint8_t* __restrict__ q, int64_t ldq,
                                                       uint8_t* __restrict__ sc, int64_t lds)
{
    __shared__ __attribute__((aligned(16))) uint8_t tile[QT * QROW];
    __shared__ float wmax[4];
    const int tid = threadIdx.x;
    // blockIdx.x runs along the stored rows (over k tiles when T is false,
    // over row tiles of op(X) when T is true), so that consecutive workgroups
    // read neighbouring pieces of the same stored rows (measured: the other
    // order makes either pack about 20 % slower)
    const int kt = T ? blockIdx.y : blockIdx.x, rt = T ? blockIdx.x : blockIdx.y;
    const int64_t k0 = int64_t(kt) * QT;
    const int64_t r0 = int64_t(rt) * QT;

    // 16 chunks of 4 floats per thread.  T == false: chunk s is stored row
    // id / 32, stored columns 4*(id % 32) .. +3, id = tid + 256*s.  T == true:
    // chunks 4b .. 4b+3 are the 4 x 4 block of stored rows 4*(id / 32) .. +3
    // (four k) and stored columns 4*(id % 32) .. +3 (four logical rows),
    // id = tid + 256*b, so each logical row's four k become one 4-byte word.
    // Either way 32 lanes read 512 consecutive bytes of one stored row.
    auto stored_row = [&](int s) { return T ? 4 * ((tid + 256 * (s >> 2)) / 32) + (s & 3) : (tid + 256 * s) / 32; };
    auto stored_col = [&](int s) { return T ? 4 * ((tid + 256 * (s >> 2)) % 32) : 4 * ((tid + 256 * s) % 32); };
    floatx4 v[16];
    // stored tile origin and valid extent
    const int64_t sr0 = T ? k0 : r0, sc0 = T ? r0 : k0;
    const int64_t SRn = T ? Kd : R, SCn = T ? R : Kd;
    if (vec && sr0 + QT <= SRn && sc0 + QT <= SCn) {   // wave-uniform: interior tile
        const float* __restrict__ base = X + sr0 * ldx + sc0;
#pragma unroll
        for (int s = 0; s < 16; ++s) v[s] = *reinterpret_cast<const floatx4*>(base + stored_row(s) * ldx + stored_col(s));
    } else {
#pragma unroll
        for (int s = 0; s < 16; ++s) v[s] = fetch4_guarded(X, ldx, sr0 + stored_row(s), sc0 + stored_col(s), SRn, SCn, vec);
    }
    float amax = 0.f;
#pragma unroll
    for (int s = 0; s < 16; ++s)
        amax = fmaxf(amax, fmaxf(fmaxf(fabsf(v[s][0]), fabsf(v[s][1])),
                                 fmaxf(fabsf(v[s][2]), fabsf(v[s][3]))));
    amax = wave_max(amax);
    if ((tid & 63) == 0) wmax[tid >> 6] = amax;
    __syncthreads();
    amax = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    const int sbyte = scale_byte(amax);
    const float inv = __builtin_bit_cast(float, uint32_t(254 - sbyte) << 23);   // 2^-(sbyte-127)

    if (!T) {
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            // stored row = logical row r, columns = k .. k+3
            int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[s][0] * inv, v[s][1] * inv, 0, false);
            w = __builtin_amdgcn_cvt_pk_fp8_f32(v[s][2] * inv, v[s][3] * inv, w, true);
            *reinterpret_cast<uint32_t*>(&tile[stored_row(s) * QROW + stored_col(s)]) = uint32_t(w);
        }
    } else {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int id = tid + 256 * b;
            const int kk = 4 * (id / 32);            // first k of the block
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int r = 4 * (id % 32) + c;     // logical row
                int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * b][c] * inv, v[4 * b + 1][c] * inv, 0, false);
                w = __builtin_amdgcn_cvt_pk_fp8_f32(v[4 * b + 2][c] * inv, v[4 * b + 3][c] * inv, w, true);
                *reinterpret_cast<uint32_t*>(&tile[r * QROW + qt_swizzle(r, kk)]) = uint32_t(w);
            }
        }
    }
    __syncthreads();
    // Write the tile out: 128 rows x 128 bytes as 16-byte chunks.
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int id = tid + 256 * s;
        const int r = id / 8, c = 16 * (id % 8);
        const int lc = T ? qt_swizzle(r, c) : c;
        *reinterpret_cast<uint4*>(q + (r0 + r) * ldq + k0 + c) = *reinterpret_cast<const uint4*>(&tile[r * QROW + lc]);
    }
    if (tid == 0) sc[rt * lds + kt] = uint8_t(sbyte);
}

hipError_t launch_fp8_pack(bool trans, const float* X, int64_t ldx, int64_t R, int64_t Kd, bool vec,
                           uint8_t* q, int64_t ldq, uint8_t* sc, int64_t lds, int64_t Rp, int64_t Kp,
                           hipStream_t stream)
{
    const dim3 grid(unsigned(trans ? Rp / QT : Kp / QT), unsigned(trans ? Kp / QT : Rp / QT)), block(256);
    if (trans) hipLaunchKernelGGL(fp8_pack_kernel<true>, grid, block, 0, stream, X, ldx, R, Kd, int(vec), q, ldq, sc, lds);
    else hipLaunchKernelGGL(fp8_pack_kernel<false>, grid, block, 0, stream, X, ldx, R, Kd, int(vec), q, ldq, sc, lds);
    return hipGetLastError();
}

// INTERLEAVE: two register staging sets, so the panel packed during panel
// kt (panel kt+1) was fetched a whole panel earlier and its LDS writes are
// spread between panel kt's matrix instructions instead of forming a burst
// before the barrier (the same scheme as the INT8 kernel); otherwise the next
// panel's fetch is issued at the top of a panel and packed after its MFMAs.
template <int BM, int BN, int WM, int WN, bool INTERLEAVE>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64)
void gemm_fp8_kernel(Fp8Args g)
{
    constexpr int BK = 128;                 // one scale block per K-panel
    constexpr int STEPS = BK / 64;
    constexpr int LDR = BK + 16;            // bytes per packed LDS row (padded)
    constexpr int WAVES_N = BN / WN;
    constexpr int NT = (BM / WM) * WAVES_N * 64;
    constexpr int V = WM / 32, H = WN / 32;

    __shared__ __attribute__((aligned(16))) uint8_t As[2][BM * LDR];
    __shared__ __attribute__((aligned(16))) uint8_t Bs[2][BN * LDR];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / WAVES_N) * WM, wn0 = (wave % WAVES_N) * WN;
    const int c = lane & 31, h = lane >> 5;

    int tm, tn;
    tile_of(blockIdx.x, g.tiles_m, g.tiles_n, g.group_m, g.remap, tm, tn);
    const int64_t m0 = int64_t(tm) * BM, n0 = int64_t(tn) * BN;

    using PA = BytePanel<BM, NT, LDR>;
    using PB = BytePanel<BN, NT, LDR>;

    floatx16 acc[V][H];
#pragma unroll
    for (int i = 0; i < V; ++i)
#pragma unroll
        for (int j = 0; j < H; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int nk = int(g.Kp / BK);
    // Scale rows of this wave's MFMA blocks (wave-uniform).
    int srow_a[V], srow_b[H];
#pragma unroll
    for (int i = 0; i < V; ++i)
        srow_a[i] = __builtin_amdgcn_readfirstlane(int((m0 + wm0 + 32 * i) / 128 * g.lds));
#pragma unroll
    for (int j = 0; j < H; ++j)
        srow_b[j] = __builtin_amdgcn_readfirstlane(int((n0 + wn0 + 32 * j) / 128 * g.lds));

    // E8M0 scale bytes of the current panel (sa, sb) and of the next (sa_n, sb_n)
    int sa[V], sb[H], sa_n[V], sb_n[H];
#pragma unroll
    for (int i = 0; i < V; ++i) sa[i] = g.sA[srow_a[i]];
#pragma unroll
    for (int j = 0; j < H; ++j) sb[j] = g.sB[srow_b[j]];

    auto next_scales = [&](int kn) {
#pragma unroll
        for (int i = 0; i < V; ++i) sa_n[i] = g.sA[srow_a[i] + kn];
#pragma unroll
        for (int j = 0; j < H; ++j) sb_n[j] = g.sB[srow_b[j] + kn];
    };
    auto take_scales = [&]() {
#pragma unroll
        for (int i = 0; i < V; ++i) sa[i] = sa_n[i];
#pragma unroll
        for (int j = 0; j < H; ++j) sb[j] = sb_n[j];
    };
    // Step s of the panel in LDS buffer `cur`; after it, the chunks of the
    // staged panel (if any) that fall to this step are written to LDS `dst`.
    auto step = [&](int cur, int s, const PA* stage_a, const PB* stage_b, int dst) {
        const int koff = 64 * s + 32 * h;
        intx8 a[V], b[H];
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const uint8_t* p = &As[cur][(wm0 + 32 * i + c) * LDR + koff];
            const uint4 lo = *reinterpret_cast<const uint4*>(p);
            const uint4 hi = *reinterpret_cast<const uint4*>(p + 16);
            a[i] = intx8{int(lo.x), int(lo.y), int(lo.z), int(lo.w), int(hi.x), int(hi.y), int(hi.z), int(hi.w)};
        }
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const uint8_t* p = &Bs[cur][(wn0 + 32 * j + c) * LDR + koff];
            const uint4 lo = *reinterpret_cast<const uint4*>(p);
            const uint4 hi = *reinterpret_cast<const uint4*>(p + 16);
            b[j] = intx8{int(lo.x), int(lo.y), int(lo.z), int(lo.w), int(hi.x), int(hi.y), int(hi.z), int(hi.w)};
        }
#pragma unroll
        for (int i = 0; i < V; ++i)
#pragma unroll
            for (int j = 0; j < H; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                    a[i], b[j], acc[i][j], 0, 0, 0, sa[i], 0, sb[j]);
        if (stage_a) {
#pragma unroll
            for (int q = s; q < PA::PER; q += STEPS) stage_a->store_chunk(As[dst], tid, q);
#pragma unroll
            for (int q = s; q < PB::PER; q += STEPS) stage_b->store_chunk(Bs[dst], tid, q);
        }
    };

    if constexpr (!INTERLEAVE) {
        PA pa;
        PB pb;
        pa.load(g.qA, g.ldq, m0, 0, tid);
        pb.load(g.qB, g.ldq, n0, 0, tid);
        pa.store(As[0], tid);
        pb.store(Bs[0], tid);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            // Everything in one basic block, with the fetch of the next panel
            // and its scale bytes issued before the MFMAs: the last panel
            // re-fetches itself (inside the packed operands) and packs into
            // the buffer nobody reads any more.
            const int kn = kt + 1 < nk ? kt + 1 : kt;
            pa.load(g.qA, g.ldq, m0, int64_t(kn) * BK, tid);
            pb.load(g.qB, g.ldq, n0, int64_t(kn) * BK, tid);
            next_scales(kn);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s = 0; s < STEPS; ++s) step(cur, s, nullptr, nullptr, 0);
            // keep the pack, which waits for the loads above, after the MFMAs
            __builtin_amdgcn_sched_barrier(0);
            pa.store(As[cur ^ 1], tid);
            pb.store(Bs[cur ^ 1], tid);
            take_scales();
            __syncthreads();
        }
    } else {
        // staging set 0 / 1 holds the panel bound for LDS buffer 0 / 1
        PA pa0, pa1;
        PB pb0, pb1;
        pa0.load(g.qA, g.ldq, m0, 0, tid);
        pb0.load(g.qB, g.ldq, n0, 0, tid);
        const int k1 = nk > 1 ? 1 : 0;
        pa1.load(g.qA, g.ldq, m0, int64_t(k1) * BK, tid);
        pb1.load(g.qB, g.ldq, n0, int64_t(k1) * BK, tid);
        pa0.store(As[0], tid);
        pb0.store(Bs[0], tid);
        __syncthreads();
        for (int kt = 0; kt < nk; kt += 2) {
            {   // panel kt in LDS 0; panel kt+1 in staging 1 goes to LDS 1
                const int kn = kt + 2 < nk ? kt + 2 : nk - 1;
                pa0.load(g.qA, g.ldq, m0, int64_t(kn) * BK, tid);
                pb0.load(g.qB, g.ldq, n0, int64_t(kn) * BK, tid);
                next_scales(kt + 1 < nk ? kt + 1 : kt);
#pragma unroll
                for (int s = 0; s < STEPS; ++s) step(0, s, &pa1, &pb1, 1);
                take_scales();
                __syncthreads();
            }
            if (kt + 1 < nk) {   // panel kt+1 in LDS 1; panel kt+2 in staging 0 goes to LDS 0
                const int kn = kt + 3 < nk ? kt + 3 : nk - 1;
                pa1.load(g.qA, g.ldq, m0, int64_t(kn) * BK, tid);
                pb1.load(g.qB, g.ldq, n0, int64_t(kn) * BK, tid);
                next_scales(kt + 2 < nk ? kt + 2 : kt + 1);
#pragma unroll
                for (int s = 0; s < STEPS; ++s) step(1, s, &pa0, &pb0, 0);
                take_scales();
                __syncthreads();
            }
        }
    }

    const float alpha = g.alpha, beta = g.beta;
    store_acc_blocks<V, H>(g.C, g.ldc, g.M, g.N, m0 + wm0, n0 + wn0, h, c, beta != 0.f, acc,
                           [&](float a, float c0) { return beta != 0.f ? __builtin_fmaf(alpha, a, beta * c0) : alpha * a; });
}

template <int BM, int BN, int WM, int WN, bool INTERLEAVE>
static hipError_t launch_fp8_cfg(Fp8Args g, hipStream_t stream)
{
    constexpr int NT = (BM / WM) * (BN / WN) * 64;
    g.tiles_m = int((g.M + BM - 1) / BM);
    g.tiles_n = int((g.N + BN - 1) / BN);
    hipLaunchKernelGGL((gemm_fp8_kernel<BM, BN, WM, WN, INTERLEAVE>), dim3(g.tiles_m * g.tiles_n), dim3(NT), 0,
                       stream, g);
    return hipGetLastError();
}

// Direct form (direct_copy in tile_bytes.h): the next panel is copied from
// global memory straight into LDS while the current one is multiplied, with
// no register staging and no LDS write instructions.  The two buffers are
// separate arrays used in a fixed alternation, so the compiler can tell the
// copy into one from the reads of the other.
//
// MIDBAR: the barrier that hands a buffer from its readers to the next copy
// sits before the panel's LAST k-step instead of after it.  That step's
// fragments are already in registers when the waves meet, so their matrix
// instructions issue as soon as the barrier releases, interleaved with the
// reads of the next panel's first step; every other step likewise reads the
// fragments of the step after it while its own matrix instructions issue.
// Without MIDBAR each panel ends with the barrier, and the next panel's
// first matrix instruction waits for its fragment reads.  The products
// accumulate in the same order either way (bit-identical results).
// Measured at 8192^3 (GEMM only): 128 x 128 tiles 1829 -> 1943 TFLOP/s with
// MIDBAR (configuration 9 against 8); 256 x 256 tiles 2395 -> 2308, slower
// (its registers are then full), so those keep the barrier at the end.
template <int BM, int BN, int WM, int WN, bool MIDBAR>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64)
void gemm_fp8_direct_kernel(Fp8Args g)
{
    constexpr int BK = 128;                 // one scale block per K-panel
    constexpr int STEPS = BK / 64;
    constexpr int WAVES_N = BN / WN;
    constexpr int NW = (BM / WM) * WAVES_N;
    constexpr int V = WM / 32, H = WN / 32;

    __shared__ __attribute__((aligned(1024))) uint8_t A0[BM * BK];
    __shared__ __attribute__((aligned(1024))) uint8_t A1[BM * BK];
    __shared__ __attribute__((aligned(1024))) uint8_t B0[BN * BK];
    __shared__ __attribute__((aligned(1024))) uint8_t B1[BN * BK];

    const int tid = threadIdx.x;
    // wave is uniform across the wave: kept in a scalar register, so the
    // LDS destinations of the direct copies need no vector registers
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm0 = (wave / WAVES_N) * WM, wn0 = (wave % WAVES_N) * WN;
    const int c = lane & 31, h = lane >> 5;

    int tm, tn;
    tile_of(blockIdx.x, g.tiles_m, g.tiles_n, g.group_m, g.remap, tm, tn);
    const int64_t m0 = int64_t(tm) * BM, n0 = int64_t(tn) * BN;

    floatx16 acc[V][H];
#pragma unroll
    for (int i = 0; i < V; ++i)
#pragma unroll
        for (int j = 0; j < H; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int nk = int(g.Kp / BK);
    int srow_a[V], srow_b[H];
#pragma unroll
    for (int i = 0; i < V; ++i)
        srow_a[i] = __builtin_amdgcn_readfirstlane(int((m0 + wm0 + 32 * i) / 128 * g.lds));
#pragma unroll
    for (int j = 0; j < H; ++j)
        srow_b[j] = __builtin_amdgcn_readfirstlane(int((n0 + wn0 + 32 * j) / 128 * g.lds));
    int sa[V], sb[H], sa_n[V], sb_n[H];
#pragma unroll
    for (int i = 0; i < V; ++i) sa[i] = g.sA[srow_a[i]];
#pragma unroll
    for (int j = 0; j < H; ++j) sb[j] = g.sB[srow_b[j]];
    auto next_scales = [&](int kn) {
#pragma unroll
        for (int i = 0; i < V; ++i) sa_n[i] = g.sA[srow_a[i] + kn];
#pragma unroll
        for (int j = 0; j < H; ++j) sb_n[j] = g.sB[srow_b[j] + kn];
    };
    auto take_scales = [&]() {
#pragma unroll
        for (int i = 0; i < V; ++i) sa[i] = sa_n[i];
#pragma unroll
        for (int j = 0; j < H; ++j) sb[j] = sb_n[j];
    };

    const uint8_t* __restrict__ qa = g.qA + m0 * g.ldq;
    const uint8_t* __restrict__ qb = g.qB + n0 * g.ldq;
    const uint32_t ld32 = uint32_t(g.ldq);
    auto copy_panel = [&](uint8_t* LA, uint8_t* LB, int kp) {
        direct_copy<BM, NW>(qa, ld32, uint32_t(kp) * BK, LA, wave, lane);
        direct_copy<BN, NW>(qb, ld32, uint32_t(kp) * BK, LB, wave, lane);
    };
    auto frag = [&](const uint8_t* L, int row, int s) {
        const int g0 = 4 * s + 2 * h;        // global chunks g0, g0 + 1 of the row
        const uint4 lo = direct_chunk(L, row, g0), hi = direct_chunk(L, row, g0 + 1);
        return intx8{int(lo.x), int(lo.y), int(lo.z), int(lo.w), int(hi.x), int(hi.y), int(hi.z), int(hi.w)};
    };
    auto products = [&](const intx8 (&a)[V], const intx8 (&b)[H]) {
#pragma unroll
        for (int i = 0; i < V; ++i)
#pragma unroll
            for (int j = 0; j < H; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                    a[i], b[j], acc[i][j], 0, 0, 0, sa[i], 0, sb[j]);
    };
    // all copies landed in LDS, then every wave past the barrier
    auto arrive = [&]() {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    };

    if constexpr (!MIDBAR) {
        auto panel = [&](const uint8_t* LA, const uint8_t* LB) {
#pragma unroll
            for (int s = 0; s < STEPS; ++s) {
                intx8 a[V], b[H];
#pragma unroll
                for (int i = 0; i < V; ++i) a[i] = frag(LA, wm0 + 32 * i + c, s);
#pragma unroll
                for (int j = 0; j < H; ++j) b[j] = frag(LB, wn0 + 32 * j + c, s);
                products(a, b);
            }
        };
        copy_panel(A0, B0, 0);
        arrive();
        for (int kt = 0; kt < nk; kt += 2) {
            // panel kt in buffer 0; panel kt+1 is copied into buffer 1 meanwhile
            if (kt + 1 < nk) copy_panel(A1, B1, kt + 1);
            next_scales(kt + 1 < nk ? kt + 1 : kt);
            panel(A0, B0);
            take_scales();
            arrive();
            if (kt + 1 < nk) {
                if (kt + 2 < nk) copy_panel(A0, B0, kt + 2);
                next_scales(kt + 2 < nk ? kt + 2 : kt + 1);
                panel(A1, B1);
                take_scales();
                arrive();
            }
        }
    } else {
        // Fragments of the step being multiplied (ca, cb).  The next step's
        // are read while its products issue: its B fragments into nb first,
        // then each A fragment into ca[i] right after the last product that
        // reads ca[i] (so only B needs a second set of registers).  The reads
        // are unconditional: after the last panel they fetch stale LDS
        // contents that are never multiplied.
        intx8 ca[V], cb[H], nb[H];
        auto step = [&](const uint8_t* LA, const uint8_t* LB, int s_next) {
#pragma unroll
            for (int j = 0; j < H; ++j) nb[j] = frag(LB, wn0 + 32 * j + c, s_next);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < V; ++i) {
#pragma unroll
                for (int j = 0; j < H; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                        ca[i], cb[j], acc[i][j], 0, 0, 0, sa[i], 0, sb[j]);
                // the refill of ca[i] stays after the products that read it
                __builtin_amdgcn_sched_barrier(0);
                ca[i] = frag(LA, wm0 + 32 * i + c, s_next);
            }
#pragma unroll
            for (int j = 0; j < H; ++j) cb[j] = nb[j];
        };
        // Panel kt sits in (LA, LB) with its step 0 in ca/cb; the panel after
        // it (if any) is being copied into (XA, XB).  On return the next
        // panel's step 0 is in ca/cb and the copy of panel kt + 2 into
        // (LA, LB) is in flight.
        auto panel = [&](int kt, uint8_t* LA, uint8_t* LB, const uint8_t* XA, const uint8_t* XB) {
#pragma unroll
            for (int s = 0; s + 1 < STEPS; ++s) step(LA, LB, s + 1);
            // every wave's reads of (LA, LB) and copies into (XA, XB) done
            arrive();
            if (kt + 2 < nk) copy_panel(LA, LB, kt + 2);
            next_scales(kt + 1 < nk ? kt + 1 : kt);
            step(XA, XB, 0);
            take_scales();
        };
        copy_panel(A0, B0, 0);
        arrive();
        if (nk > 1) copy_panel(A1, B1, 1);
#pragma unroll
        for (int i = 0; i < V; ++i) ca[i] = frag(A0, wm0 + 32 * i + c, 0);
#pragma unroll
        for (int j = 0; j < H; ++j) cb[j] = frag(B0, wn0 + 32 * j + c, 0);
        for (int kt = 0; kt < nk; kt += 2) {
            panel(kt, A0, B0, A1, B1);
            if (kt + 1 < nk) panel(kt + 1, A1, B1, A0, B0);
        }
    }

    const float alpha = g.alpha, beta = g.beta;
    store_acc_blocks<V, H>(g.C, g.ldc, g.M, g.N, m0 + wm0, n0 + wn0, h, c, beta != 0.f, acc,
                           [&](float a, float c0) { return beta != 0.f ? __builtin_fmaf(alpha, a, beta * c0) : alpha * a; });
}

template <int BM, int BN, int WM, int WN, bool MIDBAR>
static hipError_t launch_fp8_direct(Fp8Args g, hipStream_t stream)
{
    constexpr int NT = (BM / WM) * (BN / WN) * 64;
    g.tiles_m = int((g.M + BM - 1) / BM);
    g.tiles_n = int((g.N + BN - 1) / BN);
    hipLaunchKernelGGL((gemm_fp8_direct_kernel<BM, BN, WM, WN, MIDBAR>), dim3(g.tiles_m * g.tiles_n), dim3(NT), 0,
                       stream, g);
    return hipGetLastError();
}

const SgemmConfig kFp8Configs[] = {
    // id, BM, BN, BK, WM, WN
    {0, 256, 256, 128, 128, 128},
    {1, 256, 128, 128, 128, 64},
    {2, 128, 128, 128, 64, 64},
    {3, 64, 64, 128, 32, 32},
    {4, 256, 256, 128, 128, 64},
    {5, 256, 256, 128, 128, 64},   // packs interleaved with the matrix work
    {6, 128, 128, 128, 64, 64},    // packs interleaved with the matrix work
    {7, 256, 256, 128, 128, 64},   // panels copied straight into LDS
    {8, 128, 128, 128, 64, 64},    // panels copied straight into LDS
    {9, 128, 128, 128, 64, 64},    // as 8, barrier before each panel's last step
    {10, 128, 128, 128, 64, 32},   // as 8 over eight 64 x 32 waves
    {11, 256, 256, 128, 64, 64},   // as 7 over sixteen 64 x 64 waves
};
const int kNumFp8Configs = sizeof(kFp8Configs) / sizeof(kFp8Configs[0]);

hipError_t launch_gemm_fp8(int cfg, Fp8Args g, hipStream_t stream)
{
    switch (cfg) {
    case 0: return launch_fp8_cfg<256, 256, 128, 128, false>(g, stream);
    case 1: return launch_fp8_cfg<256, 128, 128, 64, false>(g, stream);
    case 2: return launch_fp8_cfg<128, 128, 64, 64, false>(g, stream);
    case 3: return launch_fp8_cfg<64, 64, 32, 32, false>(g, stream);
    case 4: return launch_fp8_cfg<256, 256, 128, 64, false>(g, stream);
    case 5: return launch_fp8_cfg<256, 256, 128, 64, true>(g, stream);
    case 6: return launch_fp8_cfg<128, 128, 64, 64, true>(g, stream);
    case 7: return launch_fp8_direct<256, 256, 128, 64, false>(g, stream);
    case 8: return launch_fp8_direct<128, 128, 64, 64, false>(g, stream);
    case 9: return launch_fp8_direct<128, 128, 64, 64, true>(g, stream);
    case 10: return launch_fp8_direct<128, 128, 64, 32, false>(g, stream);
    case 11: return launch_fp8_direct<256, 256, 64, 64, false>(g, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mg
