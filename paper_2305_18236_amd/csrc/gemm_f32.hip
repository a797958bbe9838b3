// FP32 GEMM kernels and launchers: one workgroup per output tile of the
// layered FP32 scheme in tile_f32.h.
#include "tile_f32.h"
#include "kernels.h"

namespace mg {

template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, bool DEEP, int KG>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64 * KG)
void sgemm_mfma_kernel(GemmArgs args)
{
    __shared__ __attribute__((aligned(16))) float smem[sgemm_lds_floats<BM, BN, BK, KG>()];
    GemmArgs g = args;
    split_k_view<TA, TB, false>(g);
    int tm, tn;
    tile_of(blockIdx.x, g.tiles_m, g.tiles_n, g.group_m, g.remap, tm, tn);
    sgemm_tile<BM, BN, BK, WM, WN, TA, TB, false, 0, DEEP, KG>(g, tm, tn, smem);
}

// ---------------------------------------------------------------------------
// Host-side launchers, one per tile configuration.

template <int BM, int BN, int BK, int WM, int WN, bool DEEP = false, int KG = 1>
static hipError_t launch_sgemm_cfg(bool ta, bool tb, GemmArgs g, hipStream_t stream)
{
    constexpr int NT = (BM / WM) * (BN / WN) * 64 * KG;
    g.tiles_m = int((g.M + BM - 1) / BM);
    g.tiles_n = int((g.N + BN - 1) / BN);
    const dim3 grid(g.tiles_m * g.tiles_n, split_count(g)), block(NT);
    if (!ta && !tb) hipLaunchKernelGGL((sgemm_mfma_kernel<BM, BN, BK, WM, WN, false, false, DEEP, KG>), grid, block, 0, stream, g);
    else if (!ta && tb) hipLaunchKernelGGL((sgemm_mfma_kernel<BM, BN, BK, WM, WN, false, true, DEEP, KG>), grid, block, 0, stream, g);
    else if (ta && !tb) hipLaunchKernelGGL((sgemm_mfma_kernel<BM, BN, BK, WM, WN, true, false, DEEP, KG>), grid, block, 0, stream, g);
    else hipLaunchKernelGGL((sgemm_mfma_kernel<BM, BN, BK, WM, WN, true, true, DEEP, KG>), grid, block, 0, stream, g);
    return hipGetLastError();
}

const SgemmConfig kSgemmConfigs[] = {
    // id, BM, BN, BK, WM, WN
    {0, 128, 128, 32, 64, 64},
    {1, 256, 256, 16, 128, 128},
    {2, 256, 128, 32, 128, 64},
    {3, 64, 64, 32, 32, 32},
    {4, 128, 64, 32, 64, 32},
    {5, 256, 256, 16, 128, 64},
    {6, 256, 256, 32, 128, 64},
    {7, 256, 256, 32, 128, 128},
    // no packing ("Tiling"): operands loaded straight into registers, BK is
    // the K chunk of one register fetch (tile_direct.h)
    {8, 64, 64, 8, 32, 32, 1},
    {9, 128, 128, 8, 64, 64, 1},
    // vector-ALU micro-kernel (tile_valu.h): packed panels, 8 x 8 outputs per
    // thread with scalar FP32 FMAs; WM x WN is one wave's share of the tile
    {10, 128, 128, 8, 32, 128, 0, 1},
    {11, 128, 128, 16, 32, 128, 0, 1},
    // as 3, 4 and 0, each panel fetched one and a half panels ahead (two
    // register staging sets)
    {12, 64, 64, 32, 32, 32},
    {13, 128, 64, 32, 64, 32},
    {14, 128, 128, 32, 64, 64},
    // as 12 and 13 with two K groups of waves in the workgroup (each group
    // every other panel, sums added through LDS): two waves per SIMD
    {15, 64, 64, 32, 32, 32},
    {16, 128, 64, 32, 64, 32},
    // as 5 with two register staging sets
    {17, 256, 256, 16, 128, 64},
    // 128 x 128 tiles of eight waves (64 x 32 or 32 x 64 each) with two
    // register staging sets: two waves per SIMD where configuration 0 and
    // 14 (four 64 x 64 waves) have one
    {18, 128, 128, 32, 64, 32},
    {19, 128, 128, 32, 32, 64},
    // the 128 x 64 tile over eight 32 x 32 waves with two staging sets
    {20, 128, 64, 32, 32, 32},
};
const int kNumSgemmConfigs = sizeof(kSgemmConfigs) / sizeof(kSgemmConfigs[0]);

hipError_t launch_sgemm(int cfg, bool ta, bool tb, GemmArgs g, hipStream_t stream)
{
    switch (cfg) {
    case 0: return launch_sgemm_cfg<128, 128, 32, 64, 64>(ta, tb, g, stream);
    case 1: return launch_sgemm_cfg<256, 256, 16, 128, 128>(ta, tb, g, stream);
    case 2: return launch_sgemm_cfg<256, 128, 32, 128, 64>(ta, tb, g, stream);
    case 3: return launch_sgemm_cfg<64, 64, 32, 32, 32>(ta, tb, g, stream);
    case 4: return launch_sgemm_cfg<128, 64, 32, 64, 32>(ta, tb, g, stream);
    case 5: return launch_sgemm_cfg<256, 256, 16, 128, 64>(ta, tb, g, stream);
    case 6: return launch_sgemm_cfg<256, 256, 32, 128, 64>(ta, tb, g, stream);
    case 7: return launch_sgemm_cfg<256, 256, 32, 128, 128>(ta, tb, g, stream);
    case 8:
    case 9: return launch_sgemm_direct(cfg, ta, tb, g, stream);
    case 10:
    case 11: return launch_sgemm_valu(cfg, ta, tb, g, stream);
    case 12: return launch_sgemm_cfg<64, 64, 32, 32, 32, true>(ta, tb, g, stream);
    case 13: return launch_sgemm_cfg<128, 64, 32, 64, 32, true>(ta, tb, g, stream);
    case 14: return launch_sgemm_cfg<128, 128, 32, 64, 64, true>(ta, tb, g, stream);
    case 15: return launch_sgemm_cfg<64, 64, 32, 32, 32, true, 2>(ta, tb, g, stream);
    case 16: return launch_sgemm_cfg<128, 64, 32, 64, 32, true, 2>(ta, tb, g, stream);
    case 17: return launch_sgemm_cfg<256, 256, 16, 128, 64, true>(ta, tb, g, stream);
    case 18: return launch_sgemm_cfg<128, 128, 32, 64, 32, true>(ta, tb, g, stream);
    case 19: return launch_sgemm_cfg<128, 128, 32, 32, 64, true>(ta, tb, g, stream);
    case 20: return launch_sgemm_cfg<128, 64, 32, 32, 32, true>(ta, tb, g, stream);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// C = beta * C (beta == 0 writes zeros without reading C): the BLAS quick
// return for alpha == 0 or K == 0.
__global__ __launch_bounds__(256) void scale_c_kernel(float* C, int64_t M, int64_t N, int64_t ldc, float beta)
{
    const int64_t total = M * N;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = t / N, j = t % N;
        float* p = C + i * ldc + j;
        *p = (beta == 0.f) ? 0.f : beta * *p;
    }
}

// ---------------------------------------------------------------------------
// Split-K reduction: C = alpha * (P_0 + P_1 + ... + P_{S-1}) + beta * C0, the
// partials summed in order of s (so results do not depend on scheduling) and
// the epilogue formula of the tile kernels applied to the sum.  Each thread
// handles four consecutive columns of one row per step.
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const float* __restrict__ part, int64_t ldp,
                                                            int64_t stride, int S, float* C, int64_t ldc,
                                                            int64_t M, int64_t N, float alpha, float beta,
                                                            int vec_c)
{
    const int64_t n4 = (N + 3) / 4;
    const int64_t total = M * n4;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t i = t / n4, j = (t - i * n4) * 4;
        const float* p = part + i * ldp + j;
        floatx4 acc = *reinterpret_cast<const floatx4*>(p);
        for (int s = 1; s < S; ++s) {
            const floatx4 x = *reinterpret_cast<const floatx4*>(p + s * stride);
            acc[0] += x[0]; acc[1] += x[1]; acc[2] += x[2]; acc[3] += x[3];
        }
        float* c = C + i * ldc + j;
        if (vec_c && j + 3 < N) {
            floatx4 o = {alpha * acc[0], alpha * acc[1], alpha * acc[2], alpha * acc[3]};
            if (beta != 0.f) {
                const floatx4 c0 = *reinterpret_cast<const floatx4*>(c);
                o[0] = __builtin_fmaf(alpha, acc[0], beta * c0[0]);
                o[1] = __builtin_fmaf(alpha, acc[1], beta * c0[1]);
                o[2] = __builtin_fmaf(alpha, acc[2], beta * c0[2]);
                o[3] = __builtin_fmaf(alpha, acc[3], beta * c0[3]);
            }
            *reinterpret_cast<floatx4*>(c) = o;
        } else {
            for (int e = 0; e < 4 && j + e < N; ++e) {
                float o = alpha * acc[e];
                if (beta != 0.f) o = __builtin_fmaf(alpha, acc[e], beta * c[e]);
                c[e] = o;
            }
        }
    }
}

hipError_t launch_splitk_reduce(const GemmArgs& g, int splits, float* C, int64_t ldc, hipStream_t stream)
{
    const int64_t total = g.M * ((g.N + 3) / 4);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    const int vec_c = (reinterpret_cast<uintptr_t>(C) & 15) == 0 && ldc % 4 == 0;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(unsigned(blocks)), dim3(256), 0, stream, g.part, g.ldp,
                       g.part_stride, splits, C, ldc, g.M, g.N, g.alpha, g.beta, vec_c);
    return hipGetLastError();
}

hipError_t launch_scale_c(float* C, int64_t M, int64_t N, int64_t ldc, float beta, hipStream_t stream)
{
    const int64_t total = M * N;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(scale_c_kernel, dim3(unsigned(blocks)), dim3(256), 0, stream, C, M, N, ldc, beta);
    return hipGetLastError();
}

}  // namespace mg
