// BF16 and bf16x3 GEMM kernels and launchers: one workgroup per output tile
// of the scheme in tile_bf16.h, plus the stand-alone pack-stage conversion.
#include "tile_bf16.h"
#include "kernels.h"

namespace mg {

template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, int TERMS>
__global__ __launch_bounds__((BM / WM) * (BN / WN) * 64)
void gemm_bf16_kernel(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t smem[bf16_lds_elems<BM, BN, BK, TERMS>()];
    int tm, tn;
    tile_of(blockIdx.x, g.tiles_m, g.tiles_n, g.group_m, tm, tn);
    bf16_tile<BM, BN, BK, WM, WN, TA, TB, TERMS>(g, tm, tn, smem);
}

template <int BM, int BN, int BK, int WM, int WN, int TERMS>
static hipError_t launch_bf16_cfg(bool ta, bool tb, GemmArgs g, hipStream_t stream)
{
    constexpr int NT = (BM / WM) * (BN / WN) * 64;
    g.tiles_m = int((g.M + BM - 1) / BM);
    g.tiles_n = int((g.N + BN - 1) / BN);
    const dim3 grid(g.tiles_m * g.tiles_n), block(NT);
    if (!ta && !tb) hipLaunchKernelGGL((gemm_bf16_kernel<BM, BN, BK, WM, WN, false, false, TERMS>), grid, block, 0, stream, g);
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
};
const int kNumBf16Configs = sizeof(kBf16Configs) / sizeof(kBf16Configs[0]);

template <int TERMS>
static hipError_t launch_terms(int cfg, bool ta, bool tb, GemmArgs g, hipStream_t stream)
{
    switch (cfg) {
    case 0: return launch_bf16_cfg<256, 256, 32, 128, 128, TERMS>(ta, tb, g, stream);
    case 1: return launch_bf16_cfg<256, 256, 32, 128, 64, TERMS>(ta, tb, g, stream);
    case 2: return launch_bf16_cfg<128, 128, 32, 64, 64, TERMS>(ta, tb, g, stream);
    case 3: return launch_bf16_cfg<256, 128, 32, 128, 64, TERMS>(ta, tb, g, stream);
    case 4: return launch_bf16_cfg<64, 64, 32, 32, 32, TERMS>(ta, tb, g, stream);
    case 5: return launch_bf16_cfg<128, 64, 32, 64, 32, TERMS>(ta, tb, g, stream);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gemm_bf16(int terms, int cfg, bool ta, bool tb, GemmArgs g, hipStream_t stream)
{
    return terms == 3 ? launch_terms<3>(cfg, ta, tb, g, stream) : launch_terms<1>(cfg, ta, tb, g, stream);
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
