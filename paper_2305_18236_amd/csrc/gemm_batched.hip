// Uneven batched GEMM in one persistent launch.
//
// Every problem of the batch is cut into output tiles of its own variant
// (tile shape chosen per problem by the tuning table or the default rule),
// the tiles of all problems form one work list, and a grid sized to fill the
// GPU once takes the items from that list one at a time through an atomic
// counter: whichever workgroup finishes first takes the next item.  The host
// orders the problems by the cost of one of their tiles, largest first, so
// this is greedy longest-processing-time-first scheduling, and the short
// tiles at the end fill the gaps the long ones leave.
//
// Each tile runs the same layered tile code as the single-GEMM kernels
// (tile_f32.h, tile_bf16.h): the blocked, packed, MFMA micro-kernel scheme of
// Algorithm 1 of Kuzma et al. (SPE 2023), with one LDS buffer sized for the
// largest variant shared by all of them.
#include "tile_f32.h"
#include "tile_bf16.h"
#include "kernels.h"

namespace mg {

const int kSgemmBatchedCfg[kSgemmBatchedVariants] = {3, 0};
const int kBf16BatchedCfg[kBf16BatchedVariants] = {4, 5, 2};

// Index of the problem owning work item `item`: the last p with
// tile_begin <= item (problems with no tiles are skipped by the search).
MG_DEVICE int owner(const BatchProblem* __restrict__ P, int count, int64_t item)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P[mid].tile_begin <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int BM, int BN, int BK, int WM, int WN>
MG_DEVICE void f32_variant(const BatchProblem& p, int tm, int tn, float* smem)
{
    if (p.ta) {
        if (p.tb) sgemm_tile<BM, BN, BK, WM, WN, true, true>(p.g, tm, tn, smem);
        else sgemm_tile<BM, BN, BK, WM, WN, true, false>(p.g, tm, tn, smem);
    } else {
        if (p.tb) sgemm_tile<BM, BN, BK, WM, WN, false, true>(p.g, tm, tn, smem);
        else sgemm_tile<BM, BN, BK, WM, WN, false, false>(p.g, tm, tn, smem);
    }
}

// Two waves per SIMD: the register budget stays at 256 per lane, so two
// workgroups share a CU and one's epilogue overlaps the other's K loop.
// The next work item for the whole workgroup: thread 0 takes it from the
// counter and hands it to the others through the first 8 bytes of the panel
// buffer.  That buffer is free here: every tile ends its K loop with a
// workgroup barrier after its last LDS access (its epilogue touches no LDS),
// and the second barrier keeps the next tile's packing from overwriting the
// slot before every thread has read it.  (A separate __shared__ word would
// push the bf16x3 kernel's LDS past half a CU and halve its occupancy.)
MG_DEVICE int64_t next_item(unsigned long long* counter, void* smem)
{
    int64_t* slot = static_cast<int64_t*>(smem);
    if (threadIdx.x == 0) *slot = int64_t(atomicAdd(counter, 1ull));
    __syncthreads();
    const int64_t item = *slot;
    __syncthreads();
    return item;
}

// Optional timing of the launch: workgroup b writes the constant-rate wall
// clock at its start to stamps[2b] and after its last item to stamps[2b + 1]
// (one 8-byte vector store each, from thread 0), so the caller can measure
// how long workgroups idle at the end while the last tiles finish.
MG_DEVICE void stamp(unsigned long long* stamps, int which)
{
    if (stamps != nullptr && threadIdx.x == 0) stamps[2 * int64_t(blockIdx.x) + which] = wall_clock64();
}

__global__ __launch_bounds__(256, 2) void sgemm_batched_kernel(const BatchProblem* __restrict__ P, int count,
                                                             int64_t total_tiles, unsigned long long* counter,
                                                             unsigned long long* stamps)
{
    __shared__ __attribute__((aligned(16))) float smem[sgemm_lds_floats<128, 128, 32>()];
    stamp(stamps, 0);
    for (int64_t item = next_item(counter, smem); item < total_tiles; item = next_item(counter, smem)) {
        const BatchProblem& p = P[owner(P, count, item)];
        const int64_t local = item - p.tile_begin;
        const int tm = int(local / p.g.tiles_n), tn = int(local % p.g.tiles_n);
        if (p.variant == 0) f32_variant<64, 64, 32, 32, 32>(p, tm, tn, smem);
        else f32_variant<128, 128, 32, 64, 64>(p, tm, tn, smem);
    }
    stamp(stamps, 1);
}

template <int BM, int BN, int BK, int WM, int WN, int TERMS>
MG_DEVICE void bf16_variant(const BatchProblem& p, int tm, int tn, uint16_t* smem)
{
    if (p.ta) {
        if (p.tb) bf16_tile<BM, BN, BK, WM, WN, true, true, TERMS>(p.g, tm, tn, smem);
        else bf16_tile<BM, BN, BK, WM, WN, true, false, TERMS>(p.g, tm, tn, smem);
    } else {
        if (p.tb) bf16_tile<BM, BN, BK, WM, WN, false, true, TERMS>(p.g, tm, tn, smem);
        else bf16_tile<BM, BN, BK, WM, WN, false, false, TERMS>(p.g, tm, tn, smem);
    }
}

template <int TERMS>
__global__ __launch_bounds__(256, 2) void bf16_batched_kernel(const BatchProblem* __restrict__ P, int count,
                                                            int64_t total_tiles, unsigned long long* counter,
                                                            unsigned long long* stamps)
{
    __shared__ __attribute__((aligned(16))) uint16_t smem[bf16_lds_elems<128, 128, 32, TERMS>()];
    stamp(stamps, 0);
    for (int64_t item = next_item(counter, smem); item < total_tiles; item = next_item(counter, smem)) {
        const BatchProblem& p = P[owner(P, count, item)];
        const int64_t local = item - p.tile_begin;
        const int tm = int(local / p.g.tiles_n), tn = int(local % p.g.tiles_n);
        switch (p.variant) {
        case 0: bf16_variant<64, 64, 32, 32, 32, TERMS>(p, tm, tn, smem); break;
        case 1: bf16_variant<128, 64, 32, 64, 32, TERMS>(p, tm, tn, smem); break;
        default: bf16_variant<128, 128, 32, 64, 64, TERMS>(p, tm, tn, smem); break;
        }
    }
    stamp(stamps, 1);
}

static const void* batched_kernel(int path)
{
    switch (path) {
    case 0: return reinterpret_cast<const void*>(&sgemm_batched_kernel);
    case 1: return reinterpret_cast<const void*>(&bf16_batched_kernel<3>);
    case 2: return reinterpret_cast<const void*>(&bf16_batched_kernel<1>);
    case 4: return reinterpret_cast<const void*>(&bf16_batched_kernel<16>);
    default: return nullptr;
    }
}

int batched_blocks_per_cu(int path)
{
    const void* k = batched_kernel(path);
    if (!k) return 0;
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, 256, 0) != hipSuccess || blocks < 1)
        blocks = 1;
    return blocks;
}

hipError_t launch_gemm_batched(int path, const BatchProblem* dev_problems, int count,
                               int64_t total_tiles, int grid, unsigned long long* counter,
                               unsigned long long* stamps, hipStream_t stream)
{
    const dim3 g(grid), b(256);
    switch (path) {
    case 0: hipLaunchKernelGGL(sgemm_batched_kernel, g, b, 0, stream, dev_problems, count, total_tiles, counter, stamps); break;
    case 1: hipLaunchKernelGGL(bf16_batched_kernel<3>, g, b, 0, stream, dev_problems, count, total_tiles, counter, stamps); break;
    case 2: hipLaunchKernelGGL(bf16_batched_kernel<1>, g, b, 0, stream, dev_problems, count, total_tiles, counter, stamps); break;
    case 4: hipLaunchKernelGGL(bf16_batched_kernel<16>, g, b, 0, stream, dev_problems, count, total_tiles, counter, stamps); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mg
