// Shared device-side helpers of the mgemm kernels (gfx950 / CDNA4 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));

#define MG_DEVICE __device__ __forceinline__

namespace mg {

// Arguments of one GEMM, as the kernels see them.  Strides are row strides of
// the stored matrices in elements; trans flags say whether op(X) = X^T.
struct GemmArgs {
    const float* A;
    const float* B;
    float* C;
    int64_t M, N, K;
    int64_t lda, ldb, ldc;
    float alpha, beta;
    int tiles_m, tiles_n;
    int group_m;      // tile rows per raster group (L2 reuse of B panels)
    int remap;        // 1: give each XCD a contiguous range of tiles (see tile_of)
    // vec_a / vec_b: 16-byte loads allowed (16-byte aligned, ld % 4 == 0) and
    // in-panel byte offsets fit 32 bits (ld < 2^22 - 64), which lets interior
    // panels address through a uniform base plus a 32-bit per-lane offset.
    // vec_c: 16-byte aligned C with ldc % 4 == 0.
    int vec_a, vec_b, vec_c;
    // Pre-packed BF16 operands only: element offset from the hi plane of
    // op(A) (op(B)^T) to its lo plane.
    int64_t plane_a, plane_b;
    // Split-K (launched with gridDim.y > 1): workgroup row s of the grid
    // multiplies the K range [s*k_chunk, min(K, (s+1)*k_chunk)) and stores its
    // unscaled partial product at part + s*part_stride (row stride ldp, a
    // multiple of 4, 16-byte aligned); splitk_reduce_kernel then sums the
    // partials in order of s and applies alpha and beta.
    float* part;
    int64_t k_chunk, ldp, part_stride;
};

// The GEMM one workgroup of a split-K launch computes (see GemmArgs::part).
// PACKED: A and B are k-contiguous bf16 rows (the pre-packed planes).
template <bool TA, bool TB, bool PACKED>
MG_DEVICE void split_k_view(GemmArgs& g)
{
    if (gridDim.y == 1) return;
    const int64_t k0 = int64_t(blockIdx.y) * g.k_chunk;
    g.K = min(g.k_chunk, g.K - k0);
    if (PACKED) {
        g.A = reinterpret_cast<const float*>(reinterpret_cast<const uint16_t*>(g.A) + k0);
        g.B = reinterpret_cast<const float*>(reinterpret_cast<const uint16_t*>(g.B) + k0);
    } else {
        g.A += TA ? k0 * g.lda : k0;
        g.B += TB ? k0 : k0 * g.ldb;
    }
    g.C = g.part + int64_t(blockIdx.y) * g.part_stride;
    g.ldc = g.ldp;
    g.alpha = 1.f;
    g.beta = 0.f;
    g.vec_c = 1;
}

// Arguments of the FP8 GEMM on packed operands (see gemm_fp8.hip).
struct Fp8Args {
    const uint8_t* qA;   // Mp x Kp E4M3 codes of op(A), row stride ldq
    const uint8_t* qB;   // Np x Kp E4M3 codes of op(B)^T, row stride ldq
    const uint8_t* sA;   // (Mp/128) x (Kp/128) E8M0 scale bytes, row stride lds
    const uint8_t* sB;   // (Np/128) x (Kp/128)
    float* C;
    int64_t M, N, Kp;
    int64_t ldq, lds, ldc;
    float alpha, beta;
    int tiles_m, tiles_n, group_m, remap;
};

// Map a linear workgroup id to an output tile (tm, tn): a raster that walks
// groups of `group_m` tile rows column by column, so that tiles running at
// the same time share A row panels and B column panels.
//
// Hardware hands consecutive workgroup ids to the 8 XCDs round-robin.  With
// `remap` set the ids are first permuted so that each XCD owns a contiguous
// range of the raster (its resident tiles then form one compact block per
// XCD); without it each XCD takes every eighth tile of the raster.
MG_DEVICE void tile_of(int pid, int tiles_m, int tiles_n, int group_m, int remap, int& tm, int& tn)
{
    const int total = tiles_m * tiles_n;
    constexpr int XCDS = 8;
    if (remap && total % XCDS == 0) {
        const int per = total / XCDS;
        pid = (pid % XCDS) * per + pid / XCDS;
    }
    const int in_group = group_m * tiles_n;
    const int g = pid / in_group;
    const int first_m = g * group_m;
    const int rows = min(tiles_m - first_m, group_m);
    const int local = pid - g * in_group;
    tm = first_m + local % rows;
    tn = local / rows;
}

// Guarded 16-byte fetch of stored columns gc .. gc+3 of stored row gr of a
// matrix with R x Cn valid entries (row stride ld); out-of-range elements read
// 0.  Used only on edge panels: its per-lane branches serialise the loads.
MG_DEVICE floatx4 fetch4_guarded(const float* __restrict__ src, int64_t ld, int64_t gr, int64_t gc,
                                 int64_t R, int64_t Cn, bool vec)
{
    floatx4 x = {0.f, 0.f, 0.f, 0.f};
    if (gr < R) {
        const float* p = src + gr * ld + gc;
        if (vec && gc + 3 < Cn) {
            x = *reinterpret_cast<const floatx4*>(p);
        } else {
            if (gc + 0 < Cn) x[0] = p[0];
            if (gc + 1 < Cn) x[1] = p[1];
            if (gc + 2 < Cn) x[2] = p[2];
            if (gc + 3 < Cn) x[3] = p[3];
        }
    }
    return x;
}

// 16-byte load at a uniform base plus a 32-bit per-lane BYTE offset: the
// form the global_load ... saddr instructions take (one VGPR per address).
MG_DEVICE floatx4 load16(const float* __restrict__ base, uint32_t byte_off)
{
    return *reinterpret_cast<const floatx4*>(reinterpret_cast<const char*>(base) + byte_off);
}

MG_DEVICE uint4 load16u(const void* __restrict__ base, uint32_t byte_off)
{
    return *reinterpret_cast<const uint4*>(reinterpret_cast<const char*>(base) + byte_off);
}

MG_DEVICE floatx16 mfma_f32_32x32x2(float a, float b, floatx16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

}  // namespace mg
