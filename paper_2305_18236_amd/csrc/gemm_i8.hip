// INT8 path: 8-bit integer operands with exact 32-bit integer accumulation on
// the integer matrix cores of gfx950 (v_mfma_i32_32x32x32_i8), the 8-bit
// integer row of the paper's Table 1 (there a rank-4 update per instruction;
// here rank 32).
//
// Two stages, the same layering as the FP8 path (gemm_fp8.hip):
//
// 1. Pack (i8_pack_kernel): op(A) (M x K) and op(B)^T (N x K) are copied once
//    into a workspace as k-contiguous rows, rows padded to a multiple of 256
//    and K to a multiple of 128 with zeros (zeros add nothing to the sums), so
//    the GEMM needs no bounds checks on its loads.  A source that is already
//    k-contiguous (A stored M x K, B stored N x K) is copied; the other
//    layouts are transposed through LDS.
// 2. GEMM (gemm_i8_kernel): workgroup tiles, an in-kernel loop over 128-deep
//    K panels copied into LDS, and a wave micro-kernel whose int32
//    accumulators live for the whole K loop.  The epilogue computes
//    alpha*acc + beta*C0 modulo 2^32 (two's complement); C0 is not read when
//    beta == 0.  With K <= 131071 no partial sum leaves the int32 range
//    (|a*b| <= 2^14), so the accumulation itself is exact.
//
// MFMA 32x32x32 i8 operand layout: lane l supplies 16 consecutive k of op(A)
// row l%32 and the same 16 k of op(B) column l%32 (k block l/32); result
// register r of lane l is C[8*(r/4) + 4*(l/32) + r%4][l%32].
#include "common.h"
#include "kernels.h"
#include "tile_bytes.h"
#include "epilogue.h"

namespace mg {

typedef int intx4 __attribute__((ext_vector_type(4)));
typedef int intx16 __attribute__((ext_vector_type(16)));

constexpr int IT = 128;          // pack tile (rows x bytes)
constexpr int IROW = IT + 16;    // LDS row of the pack tile (bytes), T == false

// T == true: unpadded 128-byte rows whose eight 16-byte chunks are permuted
// by an XOR with (r >> 4) % 8, so that the 4-byte writes of a wave (eight
// rows sixteen apart, eight k words) meet at most two to a bank and the
// 16-byte reads of the write-out not at all (padded and unswizzled, the
// writes meet eight to a bank).  Returns the byte offset of byte k of row r.
MG_DEVICE int it_swizzle(int r, int k) { return 16 * (((k >> 4) ^ (r >> 4)) & 7) + (k & 15); }

// One workgroup of 256 threads per 128 x 128 tile of the logical R x Kd
// matrix op(X).  T == false: X stored R x Kd (k contiguous); T == true:
// stored Kd x R.  vec: 16-byte aligned X with ldx % 16 == 0.
template <bool T>
__global__ __launch_bounds__(256) void i8_pack_kernel(const int8_t* __restrict__ X, int64_t ldx, int64_t R,
                                                      int64_t Kd, int vec, int8_t* __restrict__ q, int64_t ldq)
{
    constexpr int ROW = T ? IT : IROW;
    __shared__ __attribute__((aligned(16))) uint8_t tile[IT * ROW];
    const int tid = threadIdx.x;
    // blockIdx.x runs along the stored rows (over k tiles when T is false,
    // over row tiles of op(X) when T is true), so that consecutive workgroups
    // read neighbouring pieces of the same stored rows (measured: the other
    // order makes either pack about 20 % slower)
    const int64_t k0 = int64_t(T ? blockIdx.y : blockIdx.x) * IT, r0 = int64_t(T ? blockIdx.x : blockIdx.y) * IT;
    const int64_t sr0 = T ? k0 : r0, sc0 = T ? r0 : k0;      // stored tile origin
    const int64_t SRn = T ? Kd : R, SCn = T ? R : Kd;         // stored valid extent

    // 4 chunks of 16 stored bytes per thread.  T == false: chunk s is stored
    // row id / 8, stored columns 16*(id % 8) .. +15, id = tid + 256*s.
    // T == true: the 4 x 16 block of stored rows 4*(tid / 8) .. +3 (four k)
    // and stored columns 16*(tid % 8) .. +15 (sixteen logical rows), chunk s
    // being stored row 4*(tid / 8) + s, so each logical row's four k become
    // one 4-byte word.  Either way 8 lanes read one 128-byte stored row.
    auto stored_row = [&](int s) { return T ? 4 * (tid / 8) + s : (tid + 256 * s) / 8; };
    auto stored_col = [&](int s) { return T ? 16 * (tid % 8) : 16 * ((tid + 256 * s) % 8); };
    uint4 v[4];
    if (vec && sr0 + IT <= SRn && sc0 + IT <= SCn) {          // wave-uniform: interior tile
        const int8_t* __restrict__ base = X + sr0 * ldx + sc0;
        const uint32_t ld32 = uint32_t(ldx);
#pragma unroll
        for (int s = 0; s < 4; ++s) v[s] = load16u(base, uint32_t(stored_row(s)) * ld32 + uint32_t(stored_col(s)));
    } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int64_t gr = sr0 + stored_row(s), gc = sc0 + stored_col(s);
            uint8_t b[16];
#pragma unroll
            for (int e = 0; e < 16; ++e)
                b[e] = (gr < SRn && gc + e < SCn) ? uint8_t(X[gr * ldx + gc + e]) : uint8_t(0);
            uint32_t w[4];
#pragma unroll
            for (int d = 0; d < 4; ++d)
                w[d] = uint32_t(b[4 * d]) | (uint32_t(b[4 * d + 1]) << 8) | (uint32_t(b[4 * d + 2]) << 16) |
                       (uint32_t(b[4 * d + 3]) << 24);
            v[s] = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
    if (!T) {
#pragma unroll
        for (int s = 0; s < 4; ++s)   // stored row = logical row, columns = k .. k+15
            *reinterpret_cast<uint4*>(&tile[stored_row(s) * IROW + stored_col(s)]) = v[s];
    } else {
        const int kk = 4 * (tid / 8);                  // first k of the block
        const uint32_t w[4][4] = {{v[0].x, v[0].y, v[0].z, v[0].w}, {v[1].x, v[1].y, v[1].z, v[1].w},
                                  {v[2].x, v[2].y, v[2].z, v[2].w}, {v[3].x, v[3].y, v[3].z, v[3].w}};
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int r = 16 * (tid % 8) + c;          // logical row
            const int sh = 8 * (c & 3);
            const uint32_t word = ((w[0][c >> 2] >> sh) & 0xffu) | (((w[1][c >> 2] >> sh) & 0xffu) << 8) |
                                  (((w[2][c >> 2] >> sh) & 0xffu) << 16) | (((w[3][c >> 2] >> sh) & 0xffu) << 24);
            *reinterpret_cast<uint32_t*>(&tile[r * IT + it_swizzle(r, kk)]) = word;
        }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int id = tid + 256 * s;
        const int r = id / 8, c = 16 * (id % 8);
        const int off = T ? r * IT + it_swizzle(r, c) : r * IROW + c;
        *reinterpret_cast<uint4*>(q + (r0 + r) * ldq + k0 + c) = *reinterpret_cast<const uint4*>(&tile[off]);
    }
}

hipError_t launch_i8_pack(bool trans, const int8_t* X, int64_t ldx, int64_t R, int64_t Kd, bool vec, int8_t* q,
                          int64_t ldq, int64_t Rp, int64_t Kp, hipStream_t stream)
{
    const dim3 grid(unsigned(trans ? Rp / IT : Kp / IT), unsigned(trans ? Kp / IT : Rp / IT)), block(256);
    if (trans) hipLaunchKernelGGL(i8_pack_kernel<true>, grid, block, 0, stream, X, ldx, R, Kd, int(vec), q, ldq);
    else hipLaunchKernelGGL(i8_pack_kernel<false>, grid, block, 0, stream, X, ldx, R, Kd, int(vec), q, ldq);
    return hipGetLastError();
}

// INTERLEAVE: two register staging sets, so the panel packed during panel
// kt (panel kt+1) was fetched a whole panel earlier and its LDS writes can be
// spread between panel kt's matrix instructions instead of forming a burst
// before the barrier; otherwise the next panel's fetch is issued at the top of
// a panel and packed after its MFMAs.
template <int BM, int BN, int WM, int WN, bool INTERLEAVE>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64)
void gemm_i8_kernel(I8Args g)
{
    constexpr int BK = 128;
    constexpr int STEPS = BK / 32;
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
    const uint8_t* qA = reinterpret_cast<const uint8_t*>(g.qA);
    const uint8_t* qB = reinterpret_cast<const uint8_t*>(g.qB);

    intx16 acc[V][H];
#pragma unroll
    for (int i = 0; i < V; ++i)
#pragma unroll
        for (int j = 0; j < H; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

    using PA = BytePanel<BM, NT, LDR>;
    using PB = BytePanel<BN, NT, LDR>;
    // Step s of the panel in LDS buffer `cur`; after it, the chunks of the
    // staged panel (if any) that fall to this step are written to LDS `dst`.
    auto step = [&](int cur, int s, const PA* sa, const PB* sb, int dst) {
        const int koff = 32 * s + 16 * h;
        intx4 a[V], b[H];
#pragma unroll
        for (int i = 0; i < V; ++i)
            a[i] = *reinterpret_cast<const intx4*>(&As[cur][(wm0 + 32 * i + c) * LDR + koff]);
#pragma unroll
        for (int j = 0; j < H; ++j)
            b[j] = *reinterpret_cast<const intx4*>(&Bs[cur][(wn0 + 32 * j + c) * LDR + koff]);
#pragma unroll
        for (int i = 0; i < V; ++i)
#pragma unroll
            for (int j = 0; j < H; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i][j], 0, 0, 0);
        if (sa) {
#pragma unroll
            for (int q = s; q < PA::PER; q += STEPS) sa->store_chunk(As[dst], tid, q);
#pragma unroll
            for (int q = s; q < PB::PER; q += STEPS) sb->store_chunk(Bs[dst], tid, q);
        }
    };

    const int nk = int(g.Kp / BK);
    if constexpr (!INTERLEAVE) {
        PA pa;
        PB pb;
        pa.load(qA, g.ldq, m0, 0, tid);
        pb.load(qB, g.ldq, n0, 0, tid);
        pa.store(As[0], tid);
        pb.store(Bs[0], tid);
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            // One basic block per panel with the next panel's fetch issued
            // before the MFMAs (the last panel re-fetches itself and packs
            // into the buffer nobody reads any more).
            const int kn = kt + 1 < nk ? kt + 1 : kt;
            pa.load(qA, g.ldq, m0, int64_t(kn) * BK, tid);
            pb.load(qB, g.ldq, n0, int64_t(kn) * BK, tid);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s = 0; s < STEPS; ++s) step(cur, s, nullptr, nullptr, 0);
            // keep the pack, which waits for the loads above, after the MFMAs
            __builtin_amdgcn_sched_barrier(0);
            pa.store(As[cur ^ 1], tid);
            pb.store(Bs[cur ^ 1], tid);
            __syncthreads();
        }
    } else {
        // staging set 0 / 1 holds the panel bound for LDS buffer 0 / 1
        PA pa0, pa1;
        PB pb0, pb1;
        pa0.load(qA, g.ldq, m0, 0, tid);
        pb0.load(qB, g.ldq, n0, 0, tid);
        const int k1 = nk > 1 ? 1 : 0;
        pa1.load(qA, g.ldq, m0, int64_t(k1) * BK, tid);
        pb1.load(qB, g.ldq, n0, int64_t(k1) * BK, tid);
        pa0.store(As[0], tid);
        pb0.store(Bs[0], tid);
        __syncthreads();
        for (int kt = 0; kt < nk; kt += 2) {
            {   // panel kt in LDS 0; panel kt+1 in staging 1 goes to LDS 1
                const int kn = kt + 2 < nk ? kt + 2 : nk - 1;
                pa0.load(qA, g.ldq, m0, int64_t(kn) * BK, tid);
                pb0.load(qB, g.ldq, n0, int64_t(kn) * BK, tid);
#pragma unroll
                for (int s = 0; s < STEPS; ++s) step(0, s, &pa1, &pb1, 1);
                __syncthreads();
            }
            if (kt + 1 < nk) {   // panel kt+1 in LDS 1; panel kt+2 in staging 0 goes to LDS 0
                const int kn = kt + 3 < nk ? kt + 3 : nk - 1;
                pa1.load(qA, g.ldq, m0, int64_t(kn) * BK, tid);
                pb1.load(qB, g.ldq, n0, int64_t(kn) * BK, tid);
#pragma unroll
                for (int s = 0; s < STEPS; ++s) step(1, s, &pa0, &pb0, 0);
                __syncthreads();
            }
        }
    }

    // C = alpha*acc + beta*C0 modulo 2^32 (unsigned arithmetic wraps).
    const uint32_t alpha = uint32_t(g.alpha), beta = uint32_t(g.beta);
    store_acc_blocks<V, H>(g.C, g.ldc, g.M, g.N, m0 + wm0, n0 + wn0, h, c, beta != 0u, acc,
                           [&](int32_t a, int32_t c0) { return int32_t(alpha * uint32_t(a) + beta * uint32_t(c0)); });
}

// C = beta * C modulo 2^32 (beta == 0 writes zeros without reading C): the
// quick return for alpha == 0 or K == 0.
__global__ __launch_bounds__(256) void scale_c_i32_kernel(int32_t* C, int64_t M, int64_t N, int64_t ldc,
                                                          int32_t beta)
{
    const int64_t total = M * N;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = t / N, j = t % N;
        int32_t* p = C + i * ldc + j;
        *p = (beta == 0) ? 0 : int32_t(uint32_t(beta) * uint32_t(*p));
    }
}

hipError_t launch_scale_c_i32(int32_t* C, int64_t M, int64_t N, int64_t ldc, int32_t beta, hipStream_t stream)
{
    int64_t blocks = (M * N + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(scale_c_i32_kernel, dim3(unsigned(blocks)), dim3(256), 0, stream, C, M, N, ldc, beta);
    return hipGetLastError();
}

// Direct form (direct_copy in tile_bytes.h): the next panel is copied from
// global memory straight into LDS while the current one is multiplied, with
// no register staging and no LDS write instructions.  The two buffers are
// separate arrays used in a fixed alternation, so the compiler can tell the
// copy into one from the reads of the other.
template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64)
void gemm_i8_direct_kernel(I8Args g)
{
    constexpr int BK = 128;
    constexpr int STEPS = BK / 32;
    constexpr int WAVES_N = BN / WN;
    constexpr int NW = (BM / WM) * WAVES_N;
    constexpr int V = WM / 32, H = WN / 32;

    __shared__ __attribute__((aligned(1024))) uint8_t A0[BM * BK];
    __shared__ __attribute__((aligned(1024))) uint8_t A1[BM * BK];
    __shared__ __attribute__((aligned(1024))) uint8_t B0[BN * BK];
    __shared__ __attribute__((aligned(1024))) uint8_t B1[BN * BK];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / WAVES_N) * WM, wn0 = (wave % WAVES_N) * WN;
    const int c = lane & 31, h = lane >> 5;

    int tm, tn;
    tile_of(blockIdx.x, g.tiles_m, g.tiles_n, g.group_m, g.remap, tm, tn);
    const int64_t m0 = int64_t(tm) * BM, n0 = int64_t(tn) * BN;
    const uint8_t* __restrict__ qa = reinterpret_cast<const uint8_t*>(g.qA) + m0 * g.ldq;
    const uint8_t* __restrict__ qb = reinterpret_cast<const uint8_t*>(g.qB) + n0 * g.ldq;
    const uint32_t ld32 = uint32_t(g.ldq);

    intx16 acc[V][H];
#pragma unroll
    for (int i = 0; i < V; ++i)
#pragma unroll
        for (int j = 0; j < H; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

    auto copy_panel = [&](uint8_t* LA, uint8_t* LB, int kp) {
        direct_copy<BM, NW>(qa, ld32, uint32_t(kp) * BK, LA, wave, lane);
        direct_copy<BN, NW>(qb, ld32, uint32_t(kp) * BK, LB, wave, lane);
    };
    auto panel = [&](const uint8_t* LA, const uint8_t* LB) {
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            // lane (c, h) supplies 16 k of row c: global chunk 2s + h
            intx4 a[V], b[H];
#pragma unroll
            for (int i = 0; i < V; ++i) a[i] = __builtin_bit_cast(intx4, direct_chunk(LA, wm0 + 32 * i + c, 2 * s + h));
#pragma unroll
            for (int j = 0; j < H; ++j) b[j] = __builtin_bit_cast(intx4, direct_chunk(LB, wn0 + 32 * j + c, 2 * s + h));
#pragma unroll
            for (int i = 0; i < V; ++i)
#pragma unroll
                for (int j = 0; j < H; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    };
    // all copies landed in LDS, then every wave past the barrier
    auto arrive = [&]() {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    };

    const int nk = int(g.Kp / BK);
    copy_panel(A0, B0, 0);
    arrive();
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

    // C = alpha*acc + beta*C0 modulo 2^32 (unsigned arithmetic wraps).
    const uint32_t alpha = uint32_t(g.alpha), beta = uint32_t(g.beta);
    store_acc_blocks<V, H>(g.C, g.ldc, g.M, g.N, m0 + wm0, n0 + wn0, h, c, beta != 0u, acc,
                           [&](int32_t a, int32_t c0) { return int32_t(alpha * uint32_t(a) + beta * uint32_t(c0)); });
}

template <int BM, int BN, int WM, int WN>
static hipError_t launch_i8_direct(I8Args g, hipStream_t stream)
{
    constexpr int NT = (BM / WM) * (BN / WN) * 64;
    g.tiles_m = int((g.M + BM - 1) / BM);
    g.tiles_n = int((g.N + BN - 1) / BN);
    hipLaunchKernelGGL((gemm_i8_direct_kernel<BM, BN, WM, WN>), dim3(g.tiles_m * g.tiles_n), dim3(NT), 0, stream, g);
    return hipGetLastError();
}

template <int BM, int BN, int WM, int WN, bool INTERLEAVE>
static hipError_t launch_i8_cfg(I8Args g, hipStream_t stream)
{
    constexpr int NT = (BM / WM) * (BN / WN) * 64;
    g.tiles_m = int((g.M + BM - 1) / BM);
    g.tiles_n = int((g.N + BN - 1) / BN);
    hipLaunchKernelGGL((gemm_i8_kernel<BM, BN, WM, WN, INTERLEAVE>), dim3(g.tiles_m * g.tiles_n), dim3(NT), 0, stream,
                       g);
    return hipGetLastError();
}

const SgemmConfig kI8Configs[] = {
    // id, BM, BN, BK, WM, WN
    {0, 256, 256, 128, 128, 64},
    {1, 128, 128, 128, 64, 64},
    {2, 64, 64, 128, 32, 32},
    {3, 256, 256, 128, 128, 64},   // packs interleaved with the matrix work
    {4, 128, 128, 128, 64, 64},    // packs interleaved with the matrix work
    {5, 256, 256, 128, 128, 64},   // panels copied straight into LDS
    {6, 128, 128, 128, 64, 32},    // panels copied straight into LDS, eight 64 x 32 waves
    {7, 256, 256, 128, 64, 64},    // as 5 over sixteen 64 x 64 waves
};
const int kNumI8Configs = sizeof(kI8Configs) / sizeof(kI8Configs[0]);

hipError_t launch_gemm_i8(int cfg, I8Args g, hipStream_t stream)
{
    switch (cfg) {
    case 0: return launch_i8_cfg<256, 256, 128, 64, false>(g, stream);
    case 1: return launch_i8_cfg<128, 128, 64, 64, false>(g, stream);
    case 2: return launch_i8_cfg<64, 64, 32, 32, false>(g, stream);
    case 3: return launch_i8_cfg<256, 256, 128, 64, true>(g, stream);
    case 4: return launch_i8_cfg<128, 128, 64, 64, true>(g, stream);
    case 5: return launch_i8_direct<256, 256, 128, 64>(g, stream);
    case 6: return launch_i8_direct<128, 128, 64, 32>(g, stream);
    case 7: return launch_i8_direct<256, 256, 64, 64>(g, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mg
