#pragma once
// Staging of one panel of a pre-packed 8-bit operand (FP8 codes or int8
// values): ROWS rows of a 128-deep K panel, k-contiguous in global memory
// (row stride ldq bytes, zero-padded so no bounds checks are needed), copied
// through registers into LDS rows of LDR bytes.  Eight lanes copy one
// 128-byte row with 16-byte accesses.
#include "common.h"

namespace mg {

template <int ROWS, int NT, int LDR>
struct BytePanel {
    static constexpr int CHUNKS = ROWS * 128 / 16;
    static constexpr int PER = CHUNKS / NT;
    static_assert(CHUNKS % NT == 0, "panels must split evenly");
    uint4 v[PER];

    MG_DEVICE void load(const uint8_t* __restrict__ q, int64_t ldq, int64_t row0, int64_t k0, int tid)
    {
        const uint8_t* __restrict__ base = q + row0 * ldq + k0;
        const uint32_t ld32 = uint32_t(ldq);
#pragma unroll
        for (int s = 0; s < PER; ++s) {
            const uint32_t id = tid + s * NT;
            v[s] = load16u(base, (id / 8) * ld32 + 16 * (id % 8));
        }
    }

    MG_DEVICE void store(uint8_t* lds, int tid) const
    {
#pragma unroll
        for (int s = 0; s < PER; ++s) store_chunk(lds, tid, s);
    }

    // One of the PER 16-byte chunks, so that a caller can spread the LDS
    // writes of a panel between its matrix instructions.
    MG_DEVICE void store_chunk(uint8_t* lds, int tid, int s) const
    {
        const int id = tid + s * NT;
        *reinterpret_cast<uint4*>(&lds[(id / 8) * LDR + 16 * (id % 8)]) = v[s];
    }
};

}  // namespace mg
