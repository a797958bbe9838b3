// SYR2K on the FP32 matrix cores: the paper's worked example of reusing the
// macro level for another BLAS kernel (Section 5.1).
//
//   C = alpha*A*B^T + alpha*B*A^T + beta*C   (trans 'N': A, B are N x K)
//   C = alpha*A^T*B + alpha*B^T*A + beta*C   (trans 'T': A, B are K x N)
//
// C is symmetric and only one triangle is computed and stored.  The paper's
// recipe: the block loops visit blocks of C, each block needs a normal and a
// transposed panel of both A and B, packed by the same packing routine, and
// two intrinsic calls update the block.  Here every workgroup owns one square
// tile of the stored triangle (tiles strictly outside it are never launched)
// and runs the FP32 tile of tile_f32.h with its SYR2K option: the K loop goes
// over the panels twice, the second time with A and B exchanged, so both
// products accumulate in the same registers and the epilogue writes
// alpha*(X Y^T + Y X^T) + beta*C once, masked to the triangle on diagonal
// tiles.  Transposition is absorbed by the pack as for GEMM.
#include "tile_f32.h"
#include "kernels.h"

namespace mg {

// Linear workgroup id -> tile (tm, tn) of the lower triangle (tm >= tn) of a
// T x T tile grid: row tm holds tm + 1 tiles.  The XCD remap of tile_of()
// comes first, so each XCD walks a contiguous range of the triangle.
MG_DEVICE void tri_tile_of(int pid, int T, int& tm, int& tn)
{
    const int total = T * (T + 1) / 2;
    constexpr int XCDS = 8;
    if (total % XCDS == 0) {
        const int per = total / XCDS;
        pid = (pid % XCDS) * per + pid / XCDS;
    }
    int r = int((sqrtf(8.f * float(pid) + 1.f) - 1.f) * 0.5f);
    while ((r + 1) * (r + 2) / 2 <= pid) ++r;   // fix rounding of the float root
    while (r * (r + 1) / 2 > pid) --r;
    tm = r;
    tn = pid - r * (r + 1) / 2;
}

// Split form (gridDim.y = S > 1): the 2 * ceil(K / BK) panels of a tile's
// K loop (both products) are cut into ranges of g.k_chunk panels; workgroup
// row s writes its unscaled partial tile to g.part + s * g.part_stride (row
// stride g.ldp) and syr2k_reduce_kernel sums the S partials of every
// triangle entry in order of s.  Used when the triangle has too few tiles
// to keep every compute unit busy through the last round of tiles.
template <int BT, int BK, int WM, int WN, bool TR, int UPLO>
__global__ __launch_bounds__((BT / WM) * (BT / WN) * 64)
void syr2k_kernel(GemmArgs args)
{
    __shared__ __attribute__((aligned(16))) float smem[sgemm_lds_floats<BT, BT, BK>()];
    GemmArgs g = args;
    if (gridDim.y > 1) {
        g.C = g.part + int64_t(blockIdx.y) * g.part_stride;
        g.ldc = g.ldp;
        g.alpha = 1.f;
        g.beta = 0.f;
        g.vec_c = 1;
    }
    int tm, tn;
    tri_tile_of(blockIdx.x, g.tiles_m, tm, tn);
    if (UPLO == 2) {   // upper triangle: the mirrored tile
        const int t = tm;
        tm = tn;
        tn = t;
    }
    // trans 'N': op(A) = X (stored N x K), op(B) = Y^T (Y stored N x K);
    // trans 'T': op(A) = X^T (stored K x N), op(B) = Y (stored K x N).
    // Two register staging sets (each panel fetched one and a half panels
    // before it is packed), as the GEMM's 256 x 256 tile.
    sgemm_tile<BT, BT, BK, WM, WN, TR, !TR, true, UPLO, true>(g, tm, tn, smem);
}

template <int BT, int BK, int WM, int WN>
static hipError_t launch_syr2k_cfg(bool lower, bool tr, int splits, GemmArgs g, hipStream_t stream)
{
    constexpr int NT = (BT / WM) * (BT / WN) * 64;
    const int T = int((g.N + BT - 1) / BT);
    g.tiles_m = g.tiles_n = T;
    const dim3 grid(unsigned(int64_t(T) * (T + 1) / 2), unsigned(splits > 1 ? splits : 1)), block(NT);
    if (lower && !tr) hipLaunchKernelGGL((syr2k_kernel<BT, BK, WM, WN, false, 1>), grid, block, 0, stream, g);
    else if (lower && tr) hipLaunchKernelGGL((syr2k_kernel<BT, BK, WM, WN, true, 1>), grid, block, 0, stream, g);
    else if (!tr) hipLaunchKernelGGL((syr2k_kernel<BT, BK, WM, WN, false, 2>), grid, block, 0, stream, g);
    else hipLaunchKernelGGL((syr2k_kernel<BT, BK, WM, WN, true, 2>), grid, block, 0, stream, g);
    return hipGetLastError();
}

bool syr2k_config_supported(int cfg) { return cfg == 0 || cfg == 3 || cfg == 5 || cfg == 18; }

int syr2k_panel_depth(int cfg) { return cfg == 5 ? 16 : 32; }

hipError_t launch_syr2k(int cfg, bool lower, bool tr, int splits, GemmArgs g, hipStream_t stream)
{
    switch (cfg) {
    case 0: return launch_syr2k_cfg<128, 32, 64, 64>(lower, tr, splits, g, stream);
    case 3: return launch_syr2k_cfg<64, 32, 32, 32>(lower, tr, splits, g, stream);
    case 5: return launch_syr2k_cfg<256, 16, 128, 64>(lower, tr, splits, g, stream);
    case 18: return launch_syr2k_cfg<128, 32, 64, 32>(lower, tr, splits, g, stream);
    default: return hipErrorInvalidValue;
    }
}

// C = alpha * (P_0 + ... + P_{S-1}) + beta * C0 on one triangle, partials
// summed in order of s.  One workgroup per matrix row (grid-stride); each
// thread takes four consecutive columns, with 16-byte accesses where all four
// lie in the triangle and C allows them (vec_c: C 16-byte aligned, ldc % 4 ==
// 0; the partials always do: 256-byte aligned base, ldp and the partial
// stride multiples of 4), element by element otherwise.
__global__ __launch_bounds__(256) void syr2k_reduce_kernel(const float* __restrict__ part, int64_t ldp,
                                                          int64_t stride, int S, float* C, int64_t N,
                                                          int64_t ldc, float alpha, float beta, int lower,
                                                          int vec_c)
{
    for (int64_t i = blockIdx.x; i < N; i += gridDim.x) {
        const int64_t j0 = lower ? 0 : i, j1 = lower ? i + 1 : N;
        for (int64_t q = (j0 & ~int64_t(3)) + 4 * int64_t(threadIdx.x); q < j1; q += 4 * int64_t(blockDim.x)) {
            const float* p = part + i * ldp + q;
            float* c = C + i * ldc + q;
            if (vec_c && q >= j0 && q + 3 < j1) {
                floatx4 acc = *reinterpret_cast<const floatx4*>(p);
                for (int s = 1; s < S; ++s) {
                    const floatx4 v = *reinterpret_cast<const floatx4*>(p + s * stride);
                    acc[0] += v[0]; acc[1] += v[1]; acc[2] += v[2]; acc[3] += v[3];
                }
                floatx4 o;
                if (beta != 0.f) {
                    const floatx4 c0 = *reinterpret_cast<const floatx4*>(c);
#pragma unroll
                    for (int e = 0; e < 4; ++e) o[e] = __builtin_fmaf(alpha, acc[e], beta * c0[e]);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) o[e] = alpha * acc[e];
                }
                *reinterpret_cast<floatx4*>(c) = o;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (q + e < j0 || q + e >= j1) continue;
                    float acc = p[e];
                    for (int s = 1; s < S; ++s) acc += p[s * stride + e];
                    c[e] = beta != 0.f ? __builtin_fmaf(alpha, acc, beta * c[e]) : alpha * acc;
                }
            }
        }
    }
}

hipError_t launch_syr2k_reduce(const GemmArgs& g, int splits, bool lower, hipStream_t stream)
{
    const int64_t blocks = g.N < 8192 ? g.N : 8192;
    hipLaunchKernelGGL(syr2k_reduce_kernel, dim3(unsigned(blocks > 0 ? blocks : 1)), dim3(256), 0, stream, g.part,
                       g.ldp, g.part_stride, splits, g.C, g.N, g.ldc, g.alpha, g.beta, int(lower), int(g.vec_c));
    return hipGetLastError();
}

// C = beta * C on one triangle (beta == 0 writes zeros without reading C):
// the quick return for alpha == 0 or K == 0.
__global__ __launch_bounds__(256) void scale_tri_kernel(float* C, int64_t N, int64_t ldc, float beta, int lower)
{
    for (int64_t i = blockIdx.x; i < N; i += gridDim.x) {
        const int64_t j0 = lower ? 0 : i, j1 = lower ? i + 1 : N;
        for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
            float* p = C + i * ldc + j;
            *p = (beta == 0.f) ? 0.f : beta * *p;
        }
    }
}

hipError_t launch_scale_tri(float* C, int64_t N, int64_t ldc, float beta, bool lower, hipStream_t stream)
{
    const int64_t blocks = N < 4096 ? N : 4096;
    hipLaunchKernelGGL(scale_tri_kernel, dim3(unsigned(blocks > 0 ? blocks : 1)), dim3(256), 0, stream, C, N, ldc,
                       beta, int(lower));
    return hipGetLastError();
}

}  // namespace mg
