// FP32 GEMM without packing ("Tiling"): kernels and launchers for the
// direct-load tile of tile_direct.h.  Selected through the FP32 configuration
// table like every other tile shape.
#include "tile_direct.h"
#include "kernels.h"

namespace mg {

template <int WAVES_M, int WAVES_N, int WM, int WN, bool TA, bool TB>
__global__ __launch_bounds__(WAVES_M * WAVES_N * 64)
void sgemm_direct_kernel(GemmArgs args)
{
    GemmArgs g = args;
    split_k_view<TA, TB, false>(g);
    int tm, tn;
    tile_of(blockIdx.x, g.tiles_m, g.tiles_n, g.group_m, g.remap, tm, tn);
    direct_tile<WAVES_M, WAVES_N, WM, WN, TA, TB>(g, tm, tn);
}

template <int WAVES_M, int WAVES_N, int WM, int WN>
static hipError_t launch_direct_cfg(bool ta, bool tb, GemmArgs g, hipStream_t stream)
{
    constexpr int BM = WAVES_M * WM, BN = WAVES_N * WN;
    g.tiles_m = int((g.M + BM - 1) / BM);
    g.tiles_n = int((g.N + BN - 1) / BN);
    const dim3 grid(g.tiles_m * g.tiles_n, split_count(g)), block(WAVES_M * WAVES_N * 64);
    if (!ta && !tb) hipLaunchKernelGGL((sgemm_direct_kernel<WAVES_M, WAVES_N, WM, WN, false, false>), grid, block, 0, stream, g);
    else if (!ta && tb) hipLaunchKernelGGL((sgemm_direct_kernel<WAVES_M, WAVES_N, WM, WN, false, true>), grid, block, 0, stream, g);
    else if (ta && !tb) hipLaunchKernelGGL((sgemm_direct_kernel<WAVES_M, WAVES_N, WM, WN, true, false>), grid, block, 0, stream, g);
    else hipLaunchKernelGGL((sgemm_direct_kernel<WAVES_M, WAVES_N, WM, WN, true, true>), grid, block, 0, stream, g);
    return hipGetLastError();
}

hipError_t launch_sgemm_direct(int cfg, bool ta, bool tb, GemmArgs g, hipStream_t stream)
{
    switch (cfg) {
    case 8: return launch_direct_cfg<2, 2, 32, 32>(ta, tb, g, stream);
    case 9: return launch_direct_cfg<2, 2, 64, 64>(ta, tb, g, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mg
