// FP32 GEMM with the vector-ALU micro-kernel of tile_valu.h (the generic
// lowering, compared against the matrix-core one).  Selected through the FP32
// configuration table.
#include "tile_valu.h"
#include "kernels.h"

namespace mg {

template <int BK, bool TA, bool TB>
__global__ __launch_bounds__(256) void sgemm_valu_kernel(GemmArgs args)
{
    __shared__ __attribute__((aligned(16))) float smem[sgemm_lds_floats<128, 128, BK>()];
    GemmArgs g = args;
    split_k_view<TA, TB, false>(g);
    int tm, tn;
    tile_of(blockIdx.x, g.tiles_m, g.tiles_n, g.group_m, g.remap, tm, tn);
    valu_tile<BK, TA, TB>(g, tm, tn, smem);
}

template <int BK>
static hipError_t launch_valu_cfg(bool ta, bool tb, GemmArgs g, hipStream_t stream)
{
    g.tiles_m = int((g.M + 127) / 128);
    g.tiles_n = int((g.N + 127) / 128);
    const dim3 grid(g.tiles_m * g.tiles_n, split_count(g)), block(256);
    if (!ta && !tb) hipLaunchKernelGGL((sgemm_valu_kernel<BK, false, false>), grid, block, 0, stream, g);
    else if (!ta && tb) hipLaunchKernelGGL((sgemm_valu_kernel<BK, false, true>), grid, block, 0, stream, g);
    else if (ta && !tb) hipLaunchKernelGGL((sgemm_valu_kernel<BK, true, false>), grid, block, 0, stream, g);
    else hipLaunchKernelGGL((sgemm_valu_kernel<BK, true, true>), grid, block, 0, stream, g);
    return hipGetLastError();
}

hipError_t launch_sgemm_valu(int cfg, bool ta, bool tb, GemmArgs g, hipStream_t stream)
{
    switch (cfg) {
    case 10: return launch_valu_cfg<8>(ta, tb, g, stream);
    case 11: return launch_valu_cfg<16>(ta, tb, g, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mg
