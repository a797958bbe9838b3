// FP32 GEMM kernels and launchers: one workgroup per output tile of the
// layered FP32 scheme in tile_f32.h.
#include "tile_f32.h"
#include "kernels.h"

namespace mg {

template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64)
void sgemm_mfma_kernel(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) float smem[sgemm_lds_floats<BM, BN, BK>()];
    int tm, tn;
    tile_of(blockIdx.x, g.tiles_m, g.tiles_n, g.group_m, tm, tn);
    sgemm_tile<BM, BN, BK, WM, WN, TA, TB>(g, tm, tn, smem);
}

// ---------------------------------------------------------------------------
// Host-side launchers, one per tile configuration.

template <int BM, int BN, int BK, int WM, int WN>
static hipError_t launch_sgemm_cfg(bool ta, bool tb, GemmArgs g, hipStream_t stream)
{
    constexpr int NT = (BM / WM) * (BN / WN) * 64;
    g.tiles_m = int((g.M + BM - 1) / BM);
    g.tiles_n = int((g.N + BN - 1) / BN);
    const dim3 grid(g.tiles_m * g.tiles_n), block(NT);
    if (!ta && !tb) hipLaunchKernelGGL((sgemm_mfma_kernel<BM, BN, BK, WM, WN, false, false>), grid, block, 0, stream, g);
    else if (!ta && tb) hipLaunchKernelGGL((sgemm_mfma_kernel<BM, BN, BK, WM, WN, false, true>), grid, block, 0, stream, g);
    else if (ta && !tb) hipLaunchKernelGGL((sgemm_mfma_kernel<BM, BN, BK, WM, WN, true, false>), grid, block, 0, stream, g);
    else hipLaunchKernelGGL((sgemm_mfma_kernel<BM, BN, BK, WM, WN, true, true>), grid, block, 0, stream, g);
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

hipError_t launch_scale_c(float* C, int64_t M, int64_t N, int64_t ldc, float beta, hipStream_t stream)
{
    const int64_t total = M * N;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(scale_c_kernel, dim3(unsigned(blocks)), dim3(256), 0, stream, C, M, N, ldc, beta);
    return hipGetLastError();
}

}  // namespace mg
