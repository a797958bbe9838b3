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

// Direct form of the byte panels: packed 128-byte k rows copied from global
// memory straight into LDS (global_load_lds_dwordx4: each lane's 16 bytes land
// at the wave's LDS base + 16 * lane), with no register staging and no LDS
// write instructions.  LDS rows are unpadded; since the copy cannot scatter,
// the bank-conflict-free layout is made by choosing the source instead: LDS
// chunk c of row r holds global chunk c ^ direct_swz(r), so 16 consecutive
// rows read at one k fall on 16 distinct 16-byte bank groups.
MG_DEVICE int direct_swz(int r) { return (r >> 1) & 7; }

// Copy ROWS rows of 128 bytes (row stride ld32 from q, k offset k0) into
// `lds`; copy j of wave w fills LDS chunks (j*NW + w)*64 .. +63.
template <int ROWS, int NW>
MG_DEVICE void direct_copy(const uint8_t* __restrict__ q, uint32_t ld32, uint32_t k0, uint8_t* lds, int wave,
                           int lane)
{
    constexpr int J = ROWS * 8 / (NW * 64);
    static_assert(ROWS * 8 % (NW * 64) == 0, "panels must split evenly");
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int slot = (j * NW + wave) * 64 + lane, r = slot >> 3;
        const uint32_t off = uint32_t(r) * ld32 + k0 + 16u * uint32_t((slot & 7) ^ direct_swz(r));
        __builtin_amdgcn_global_load_lds(q + off, lds + (j * NW + wave) * 1024, 16, 0, 0);
    }
}

// The 16 bytes of global chunk g (k bytes 16g .. 16g+15) of LDS row `row`.
MG_DEVICE uint4 direct_chunk(const uint8_t* lds, int row, int g)
{
    return *reinterpret_cast<const uint4*>(lds + row * 128 + 16 * (g ^ direct_swz(row)));
}

}  // namespace mg
