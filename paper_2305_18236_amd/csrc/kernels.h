// Internal (C++ linkage) interface between the C-ABI host layer and the
// kernel translation units.  Not part of the public header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace mg {

struct SgemmConfig {
    int id, bm, bn, bk, wm, wn;
    int direct;   // 1: operands loaded straight into registers (no LDS packing)
    int valu;     // 1: vector-ALU FMA micro-kernel instead of the matrix cores
};

extern const SgemmConfig kSgemmConfigs[];
extern const int kNumSgemmConfigs;

hipError_t launch_sgemm(int cfg, bool ta, bool tb, GemmArgs g, hipStream_t stream);
hipError_t launch_sgemm_direct(int cfg, bool ta, bool tb, GemmArgs g, hipStream_t stream);
hipError_t launch_sgemm_valu(int cfg, bool ta, bool tb, GemmArgs g, hipStream_t stream);
extern const SgemmConfig kBf16Configs[];
extern const int kNumBf16Configs;

// terms == 1: plain BF16; terms == 3: bf16x3 split.  packed: g.A / g.B are
// the hi planes written by launch_bf16_pack (plane_a / plane_b to the lo
// planes), or, for bf16x3 with configuration 6, the interleaved planes
// written by launch_bf16_pack_interleaved (row stride lda / ldb = 2 Kp).
hipError_t launch_gemm_bf16(int terms, int cfg, bool ta, bool tb, GemmArgs g, hipStream_t stream,
                            bool packed = false);
hipError_t launch_bf16_pack(bool trans, int terms, const float* X, int64_t ldx, int64_t R, int64_t Kd,
                            bool vec, uint16_t* hi, uint16_t* lo, int64_t ldq, int64_t Rp, int64_t Kp,
                            hipStream_t stream);
hipError_t launch_bf16_pack_interleaved(bool trans, const float* X, int64_t ldx, int64_t R, int64_t Kd, bool vec,
                                        uint16_t* q, int64_t ldq, int64_t Rp, int64_t Kp, hipStream_t stream);
hipError_t launch_bf16_split(const float* x, int64_t n, uint16_t* hi, uint16_t* lo, hipStream_t stream);

extern const SgemmConfig kFp8Configs[];
extern const int kNumFp8Configs;

hipError_t launch_fp8_pack(bool trans, const float* X, int64_t ldx, int64_t R, int64_t Kd, bool vec,
                           uint8_t* q, int64_t ldq, uint8_t* sc, int64_t lds, int64_t Rp, int64_t Kp,
                           hipStream_t stream);
hipError_t launch_gemm_fp8(int cfg, Fp8Args g, hipStream_t stream);

// One problem of a batched launch, as the persistent kernel reads it.
struct BatchProblem {
    GemmArgs g;           // operands, sizes, strides, alpha/beta, tile grid, vector flags
    int64_t tile_begin;   // first work item (tile) of this problem
    int variant;          // tile variant of the path's batched set
    int ta, tb;           // op(A) = A^T, op(B) = B^T
    int pad_;
};

// Tile variants of the persistent batched kernels, as configuration ids of
// the single-GEMM tables: FP32 {64x64, 128x128}; BF16 paths {64x64, 128x64,
// 128x128}.  All run 256 threads.  (A third FP32 variant would push the
// persistent kernel past 256 registers per lane.)
constexpr int kSgemmBatchedVariants = 2;
constexpr int kBf16BatchedVariants = 3;
extern const int kSgemmBatchedCfg[kSgemmBatchedVariants];
extern const int kBf16BatchedCfg[kBf16BatchedVariants];

// counter: a device word holding 0 at launch (the work-list cursor).
// stamps: nullptr, or 2 * grid words that receive each workgroup's start and
// end wall-clock times.
hipError_t launch_gemm_batched(int path, const BatchProblem* dev_problems, int count,
                               int64_t total_tiles, int grid, unsigned long long* counter,
                               unsigned long long* stamps, hipStream_t stream);
int batched_blocks_per_cu(int path);

hipError_t launch_scale_c(float* C, int64_t M, int64_t N, int64_t ldc, float beta, hipStream_t stream);

// SYR2K on one triangle (see gemm_syr2k.hip); g.M == g.N, cfg a square FP32
// configuration accepted by syr2k_config_supported().
// splits > 1: the 2 * ceil(K / BK) panels of every tile's K loop are cut into
// `splits` ranges of g.k_chunk panels (splits == ceil(panels / k_chunk)),
// each writing a partial tile to g.part (g.ldp, g.part_stride), summed by
// launch_syr2k_reduce into g.C with g.alpha / g.beta.
bool syr2k_config_supported(int cfg);
int syr2k_panel_depth(int cfg);
hipError_t launch_syr2k(int cfg, bool lower, bool tr, int splits, GemmArgs g, hipStream_t stream);
hipError_t launch_syr2k_reduce(const GemmArgs& g, int splits, bool lower, hipStream_t stream);
hipError_t launch_scale_tri(float* C, int64_t N, int64_t ldc, float beta, bool lower, hipStream_t stream);

// INT8 GEMM on packed operands (see gemm_i8.hip).
struct I8Args {
    const int8_t* qA;    // Mp x Kp int8 rows of op(A), row stride ldq
    const int8_t* qB;    // Np x Kp int8 rows of op(B)^T, row stride ldq
    int32_t* C;
    int64_t M, N, Kp;
    int64_t ldq, ldc;
    int32_t alpha, beta;
    int tiles_m, tiles_n, group_m, remap;
};
extern const SgemmConfig kI8Configs[];
extern const int kNumI8Configs;
hipError_t launch_i8_pack(bool trans, const int8_t* X, int64_t ldx, int64_t R, int64_t Kd, bool vec, int8_t* q,
                          int64_t ldq, int64_t Rp, int64_t Kp, hipStream_t stream);
hipError_t launch_gemm_i8(int cfg, I8Args g, hipStream_t stream);
hipError_t launch_scale_c_i32(int32_t* C, int64_t M, int64_t N, int64_t ldc, int32_t beta, hipStream_t stream);

// Number of K ranges of a split-K launch described by g (1: no split).
inline unsigned split_count(const GemmArgs& g)
{
    return g.k_chunk > 0 ? unsigned((g.K + g.k_chunk - 1) / g.k_chunk) : 1u;
}

// Average shader clock (MHz) of a few compute units over `wall_ticks` of the
// constant-rate wall clock (wall_hz ticks per second), measured by a probe
// launched on `stream` behind the work already queued there; waits for the
// stream.
hipError_t measure_sclk(hipStream_t stream, int64_t wall_ticks, double wall_hz, double* mhz);

// Sums the `splits` partials of g.part into C with g.alpha / g.beta.
hipError_t launch_splitk_reduce(const GemmArgs& g, int splits, float* C, int64_t ldc, hipStream_t stream);

}  // namespace mg
