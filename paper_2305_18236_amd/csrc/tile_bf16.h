#pragma once
// GEMM on the 16-bit matrix cores of gfx950 (v_mfma_f32_32x32x16_bf16 and
// v_mfma_f32_32x32x16_f16) with FP32 inputs, outputs and accumulation.  The
// TERMS parameter selects the arithmetic:
//
//   TERMS == 1  (plain BF16): each operand is rounded to bfloat16 (nearest,
//               ties to even) while it is packed into LDS.
//   TERMS == 3  (bf16x3 split): each operand x is split while packing into
//               hi = bf16(x) and lo = bf16(x - hi) (x - hi is exact in FP32),
//               and the micro-kernel accumulates hi*hi + hi*lo + lo*hi in FP32;
//               the dropped lo*lo term is below 2^-16 |a||b|.
//   TERMS == 16 (FP16): each operand is rounded to IEEE binary16 (nearest,
//               ties to even; beyond 65504 it overflows to infinity) and the
//               FP16 matrix instruction multiplies them (Table 1's 16-bit
//               float row, like BF16).
//
// Layers follow Algorithm 1 of Kuzma et al. (SPE 2023) as in the FP32 kernel
// (workgroup tiles for the i/j block loops, an in-kernel K-panel loop, packing
// of op(A) and op(B) panels into LDS, a wave micro-kernel that keeps its
// accumulators for the whole K loop).  Here the packing step also carries the
// data-type conversion, the way Section 3's packing chooses the element layout
// the target's matrix instruction wants: the rank-16 BF16 update reads eight
// consecutive k of one row per lane (the 16-bit rank-n layout of Section 3.3,
// scaled to the MFMA's depth), so both panels are packed k-contiguous:
// row mn of a panel holds op(X)[mn][k0 .. k0+BK) as bf16, padded by PAD
// elements so that the 16-byte fragment reads of consecutive rows fall in
// different LDS banks.
//
// MFMA 32x32x16 bf16 operand layout: lane l supplies eight k values of
// op(A) row l%32 and the same eight k values of op(B) column l%32 (k block
// l/32); result register r of lane l is C[8*(r/4) + 4*(l/32) + r%4][l%32].
#include "common.h"
#include "epilogue.h"

namespace mg {

// Round two floats to bf16 (hardware RNE) and return them packed.
MG_DEVICE uint32_t pack_bf16x2(float a, float b)
{
    typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
    bf16x2_t v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
}

// Split four floats: hi = bf16(x), lo = bf16(x - float(hi)).
MG_DEVICE void split4(floatx4 x, uint32_t (&hi)[2], uint32_t (&lo)[2])
{
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const float x0 = x[2 * p], x1 = x[2 * p + 1];
        const uint32_t h = pack_bf16x2(x0, x1);
        const float h0 = __builtin_bit_cast(float, h << 16);
        const float h1 = __builtin_bit_cast(float, h & 0xffff0000u);
        hi[p] = h;
        lo[p] = pack_bf16x2(x0 - h0, x1 - h1);
    }
}

MG_DEVICE void round4(floatx4 x, uint32_t (&hi)[2])
{
    hi[0] = pack_bf16x2(x[0], x[1]);
    hi[1] = pack_bf16x2(x[2], x[3]);
}

// Round two floats to binary16 (hardware RNE) and return them packed.
MG_DEVICE uint32_t pack_f16x2(float a, float b)
{
    typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
    f16x2_t v = {(_Float16)a, (_Float16)b};
    return __builtin_bit_cast(uint32_t, v);
}

// The single-term conversion of kind TERMS (1: bf16, 16: fp16).
template <int TERMS>
MG_DEVICE void convert4(floatx4 x, uint32_t (&hi)[2])
{
    if constexpr (TERMS == 16) {
        hi[0] = pack_f16x2(x[0], x[1]);
        hi[1] = pack_f16x2(x[2], x[3]);
    } else {
        round4(x, hi);
    }
}

// One rank-16 update of a 32 x 32 FP32 accumulator by the 16-bit matrix
// instruction of kind TERMS (both operands hold eight 16-bit values per lane).
template <int TERMS>
MG_DEVICE floatx16 mfma16(bf16x8 a, bf16x8 b, floatx16 c)
{
    if constexpr (TERMS == 16) {
        typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, a), __builtin_bit_cast(f16x8_t, b),
                                                      c, 0, 0, 0);
    } else {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
}

// One operand panel: ROWS (m or n) x BK (k), FP32 in global memory, packed
// into LDS as bf16 rows of LDR = BK + PAD elements.
//   KSRC: the stored matrix is k-contiguous (A 'N', B 'T'); a chunk is four
//         consecutive k of one row and becomes one 8-byte LDS write per term.
//   else: the stored matrix is mn-contiguous (A 'T', B 'N'); a block is four
//         k rows x four mn columns, fetched as four 16-byte loads and
//         transposed in registers into four 8-byte LDS writes per term.
// Lane order of the pack (LDS rows are LDR = BK + 8 bf16 = 80 bytes for
// BK = 32; 64 banks of 4 bytes):
//   KSRC: eight lanes cover one row's BK values (one 128-byte global line);
//         the row of lane group rr is row_perm(rr), which puts rows
//         0, 4, 8, 12 in one 32-lane write so their 64-byte pieces start at
//         bank offsets 0, 16, 32, 48 (row stride 20 dwords) and never collide;
//   else: lanes run over the BK/4 k-blocks first, then over mn-blocks, so one
//         8-byte write instruction stores 8 k-blocks of 4 rows spaced 4 apart:
//         dword 80*mb + 2*kb mod 64 is distinct for every lane.
MG_DEVICE int row_perm(int rr) { return (rr & ~15) | ((rr & 3) << 2) | ((rr >> 2) & 3); }

template <int ROWS, int BK, int LDR, int NT, bool KSRC, int TERMS>
struct BfPanel {
    static_assert(ROWS % 16 == 0, "row permutation works on groups of 16 rows");
    static constexpr int CHUNKS = ROWS * BK / 4;    // 16-byte chunks (KSRC)
    static constexpr int BLOCKS = ROWS * BK / 16;   // 4x4 blocks (mn-contiguous source)
    static constexpr int PER = KSRC ? (CHUNKS + NT - 1) / NT : (BLOCKS + NT - 1) / NT;
    static constexpr int LOADS = KSRC ? PER : 4 * PER;
    floatx4 v[LOADS];

    // mn0: first row (m or n) of the panel; k0: first k.  R x Cn: valid extent
    // of the stored matrix.
    MG_DEVICE void load(const float* __restrict__ src, int64_t ld, int64_t mn0, int64_t k0,
                        int64_t R, int64_t Cn, bool vec, int tid)
    {
        // stored-panel origin and extent: KSRC rows are mn, columns k; else rows k, columns mn
        const int64_t r0 = KSRC ? mn0 : k0, c0 = KSRC ? k0 : mn0;
        const int SR = KSRC ? ROWS : BK, SC = KSRC ? BK : ROWS;
        // Wave-uniform test: interior panels take the branch-free path, so all
        // their loads are in flight at once; edge panels take the guarded path.
        if (vec && r0 + SR <= R && c0 + SC <= Cn) {
            // uniform base + 32-bit per-lane offset (vec guarantees it fits)
            const float* __restrict__ base = src + r0 * ld + c0;
            const uint32_t ld32 = uint32_t(ld);
            if (KSRC) {
#pragma unroll
                for (int s = 0; s < PER; ++s) {
                    const int q = tid + s * NT;
                    if (CHUNKS % NT != 0 && q >= CHUNKS) break;
                    const uint32_t r = row_perm(q / (BK / 4)), c = (q % (BK / 4)) * 4;
                    v[s] = load16(base, (r * ld32 + c) * 4u);
                }
            } else {
#pragma unroll
                for (int b = 0; b < PER; ++b) {
                    const int q = tid + b * NT;
                    if (BLOCKS % NT != 0 && q >= BLOCKS) break;
                    const uint32_t kb = q % (BK / 4), mb = q / (BK / 4);
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        v[4 * b + e] = load16(base, ((4 * kb + e) * ld32 + 4 * mb) * 4u);
                }
            }
        } else {
            if (KSRC) {
#pragma unroll
                for (int s = 0; s < PER; ++s) {
                    const int q = tid + s * NT;
                    if (CHUNKS % NT != 0 && q >= CHUNKS) break;
                    const int r = row_perm(q / (BK / 4)), c = (q % (BK / 4)) * 4;
                    v[s] = fetch4_guarded(src, ld, mn0 + r, k0 + c, R, Cn, vec);
                }
            } else {
#pragma unroll
                for (int b = 0; b < PER; ++b) {
                    const int q = tid + b * NT;
                    if (BLOCKS % NT != 0 && q >= BLOCKS) break;
                    const int kb = q % (BK / 4), mb = q / (BK / 4);
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        v[4 * b + e] = fetch4_guarded(src, ld, k0 + 4 * kb + e, mn0 + 4 * mb, R, Cn, vec);
                }
            }
        }
    }

    MG_DEVICE void store(uint16_t* hi_lds, uint16_t* lo_lds, int tid) const
    {
        if (KSRC) {
#pragma unroll
            for (int s = 0; s < PER; ++s) {
                const int q = tid + s * NT;
                if (CHUNKS % NT != 0 && q >= CHUNKS) break;
                const int r = row_perm(q / (BK / 4)), c = (q % (BK / 4)) * 4;
                put(hi_lds, lo_lds, r * LDR + c, v[s]);
            }
        } else {
#pragma unroll
            for (int b = 0; b < PER; ++b) {
                const int q = tid + b * NT;
                if (BLOCKS % NT != 0 && q >= BLOCKS) break;
                const int kb = q % (BK / 4), mb = q / (BK / 4);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const floatx4 col = {v[4 * b + 0][t], v[4 * b + 1][t], v[4 * b + 2][t], v[4 * b + 3][t]};
                    put(hi_lds, lo_lds, (4 * mb + t) * LDR + 4 * kb, col);
                }
            }
        }
    }

    MG_DEVICE static void put(uint16_t* hi_lds, uint16_t* lo_lds, int off, floatx4 x)
    {
        uint32_t h[2], l[2];
        if constexpr (TERMS == 3) {
            split4(x, h, l);
            *reinterpret_cast<uint2*>(lo_lds + off) = make_uint2(l[0], l[1]);
        } else {
            convert4<TERMS>(x, h);
        }
        *reinterpret_cast<uint2*>(hi_lds + off) = make_uint2(h[0], h[1]);
    }
};

// Padding of a packed bf16 row (elements) and the LDS a configuration needs.
constexpr int BF16_PAD = 8;
template <int BM, int BN, int BK, int TERMS>
constexpr int bf16_lds_elems() { return 2 * (TERMS == 3 ? 2 : 1) * (BM + BN) * (BK + BF16_PAD); }

// One BM x BN output tile (tm, tn), computed by the whole workgroup.  smem:
// bf16_lds_elems() 16-bit elements of LDS, 16-byte aligned.  Ends with a
// workgroup barrier after the last LDS read.
// One operand panel read from PRE-PACKED bf16 planes (bf16_pack_kernel): rows
// of ld bf16 (k-contiguous, zero-padded), hi plane at `hi`, lo plane at
// hi + plane.  The pack to LDS is a plain 16-byte copy; lanes take four
// 16-byte chunks of one row, rows in row_perm order, so a 16-lane write
// covers rows 0, 4, 8, 12 at bank offsets 0, 16, 32, 48 (conflict-free).
template <int ROWS, int BK, int LDR, int NT, int TERMS>
struct BfPackedPanel {
    static constexpr int CPR = BK / 8;          // 16-byte chunks per row and plane
    static constexpr int CHUNKS = ROWS * CPR;
    static constexpr int PER = (CHUNKS + NT - 1) / NT;
    static constexpr int NL = (TERMS == 3) ? 2 : 1;
    static_assert(ROWS % 16 == 0, "row permutation works on groups of 16 rows");
    uint4 v[NL][PER];

    MG_DEVICE void load(const uint16_t* __restrict__ hi, int64_t plane, int64_t ld, int64_t mn0,
                        int64_t k0, int tid)
    {
        const uint16_t* __restrict__ base = hi + mn0 * ld + k0;
        const uint32_t ld32 = uint32_t(ld);
#pragma unroll
        for (int s = 0; s < PER; ++s) {
            const int q = tid + s * NT;
            if (CHUNKS % NT != 0 && q >= CHUNKS) break;
            const uint32_t r = row_perm(q / CPR), c = (q % CPR) * 8;
            const uint32_t off = (r * ld32 + c) * 2u;
            v[0][s] = load16u(base, off);
            if (TERMS == 3) v[NL - 1][s] = load16u(base + plane, off);
        }
    }

    MG_DEVICE void store(uint16_t* hi_lds, uint16_t* lo_lds, int tid) const
    {
#pragma unroll
        for (int s = 0; s < PER; ++s) store_chunk(hi_lds, lo_lds, tid, s);
    }

    // One of the PER chunks, so that a caller can spread a panel's LDS writes
    // between its matrix instructions.
    MG_DEVICE void store_chunk(uint16_t* hi_lds, uint16_t* lo_lds, int tid, int s) const
    {
        const int q = tid + s * NT;
        if (CHUNKS % NT != 0 && q >= CHUNKS) return;
        const int r = row_perm(q / CPR), c = (q % CPR) * 8;
        *reinterpret_cast<uint4*>(hi_lds + r * LDR + c) = v[0][s];
        if (TERMS == 3) *reinterpret_cast<uint4*>(lo_lds + r * LDR + c) = v[NL - 1][s];
    }
};

template <bool PACKED, int ROWS, int BK, int LDR, int NT, bool KSRC, int TERMS>
struct BfLoaderSel {
    using type = BfPanel<ROWS, BK, LDR, NT, KSRC, TERMS>;
};
template <int ROWS, int BK, int LDR, int NT, bool KSRC, int TERMS>
struct BfLoaderSel<true, ROWS, BK, LDR, NT, KSRC, TERMS> {
    using type = BfPackedPanel<ROWS, BK, LDR, NT, TERMS>;
};

// PACKED: g.A / g.B point at the hi planes of pre-packed op(A) / op(B)^T
// (bf16, row stride lda / ldb, zero-padded to whole tiles and panels), TA/TB
// are ignored and no bounds checks are needed on the loads.
template <int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, int TERMS, bool PACKED = false>
MG_DEVICE void bf16_tile(const GemmArgs& g, int tm, int tn, uint16_t* smem)
{
    constexpr int WAVES_N = BN / WN;
    constexpr int NT = (BM / WM) * WAVES_N * 64;
    constexpr int V = WM / 32, H = WN / 32;
    constexpr int LDR = BK + BF16_PAD;       // bf16 elements per packed row
    constexpr int NL = (TERMS == 3) ? 2 : 1; // hi (and lo) panels
    static_assert(BK % 16 == 0, "BK must be a multiple of the MFMA depth (16)");
    static_assert((LDR * 2) % 16 == 0, "packed rows must keep 16-byte alignment");

    uint16_t (*As)[NL][BM * LDR] = reinterpret_cast<uint16_t (*)[NL][BM * LDR]>(smem);
    uint16_t (*Bs)[NL][BN * LDR] = reinterpret_cast<uint16_t (*)[NL][BN * LDR]>(smem + 2 * NL * BM * LDR);

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / WAVES_N) * WM, wn0 = (wave % WAVES_N) * WN;
    const int c = lane & 31, h = lane >> 5;

    const int64_t m0 = int64_t(tm) * BM, n0 = int64_t(tn) * BN;

    typename BfLoaderSel<PACKED, BM, BK, LDR, NT, !TA, TERMS>::type pa;
    typename BfLoaderSel<PACKED, BN, BK, LDR, NT, TB, TERMS>::type pb;
    // Stored extents: A is M x K ('N') or K x M ('T'); B is K x N ('N') or N x K ('T').
    const int64_t Ra = TA ? g.K : g.M, Ca = TA ? g.M : g.K;
    const int64_t Rb = TB ? g.N : g.K, Cb = TB ? g.K : g.N;
    (void)Ra; (void)Ca; (void)Rb; (void)Cb;

    auto fetch = [&](int64_t k0) {
        if constexpr (PACKED) {
            pa.load(reinterpret_cast<const uint16_t*>(g.A), g.plane_a, g.lda, m0, k0, tid);
            pb.load(reinterpret_cast<const uint16_t*>(g.B), g.plane_b, g.ldb, n0, k0, tid);
        } else {
            pa.load(g.A, g.lda, m0, k0, Ra, Ca, g.vec_a, tid);
            pb.load(g.B, g.ldb, n0, k0, Rb, Cb, g.vec_b, tid);
        }
    };
    auto pack = [&](int buf) {
        pa.store(As[buf][0], As[buf][NL - 1], tid);
        pb.store(Bs[buf][0], Bs[buf][NL - 1], tid);
    };

    floatx16 acc[V][H];
#pragma unroll
    for (int i = 0; i < V; ++i)
#pragma unroll
        for (int j = 0; j < H; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int nk = int((g.K + BK - 1) / BK);
    constexpr int STEPS = BK / 16;          // MFMA k-steps per panel

    // Fragment reads of one MFMA k-step from LDS buffer `cur`.  bf16x3 issues
    // B before A and the lo halves before the hi ones, in the order its three
    // MFMA groups consume them (lo(A)*hi(B), hi(A)*lo(B), hi(A)*hi(B)), so the
    // first group starts while the later fragments are still in flight.  The
    // single-term kinds, with half the fragment registers, read the next
    // step's fragments before issuing this step's MFMAs (software pipelining
    // across the panel's steps).
    auto read_step = [&](int cur, int s, bf16x8 (&xah)[V], bf16x8 (&xal)[V], bf16x8 (&xbh)[H],
                         bf16x8 (&xbl)[H]) {
        const int koff = 16 * s + 8 * h;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int off = (wn0 + 32 * j + c) * LDR + koff;
            xbh[j] = *reinterpret_cast<const bf16x8*>(&Bs[cur][0][off]);
        }
        if constexpr (TERMS == 3) {
#pragma unroll
            for (int i = 0; i < V; ++i) {
                const int off = (wm0 + 32 * i + c) * LDR + koff;
                xal[i] = *reinterpret_cast<const bf16x8*>(&As[cur][NL - 1][off]);
            }
#pragma unroll
            for (int j = 0; j < H; ++j) {
                const int off = (wn0 + 32 * j + c) * LDR + koff;
                xbl[j] = *reinterpret_cast<const bf16x8*>(&Bs[cur][NL - 1][off]);
            }
        }
#pragma unroll
        for (int i = 0; i < V; ++i) {
            const int off = (wm0 + 32 * i + c) * LDR + koff;
            xah[i] = *reinterpret_cast<const bf16x8*>(&As[cur][0][off]);
        }
    };
    auto mfma_step = [&](const bf16x8 (&ah)[V], const bf16x8 (&al)[V], const bf16x8 (&bh)[H],
                         const bf16x8 (&bl)[H]) {
        if (TERMS == 3) {
            // small terms first; consecutive instructions use different accumulators
#pragma unroll
            for (int i = 0; i < V; ++i)
#pragma unroll
                for (int j = 0; j < H; ++j)
                    acc[i][j] = mfma16<TERMS>(al[i], bh[j], acc[i][j]);
#pragma unroll
            for (int i = 0; i < V; ++i)
#pragma unroll
                for (int j = 0; j < H; ++j)
                    acc[i][j] = mfma16<TERMS>(ah[i], bl[j], acc[i][j]);
        }
#pragma unroll
        for (int i = 0; i < V; ++i)
#pragma unroll
            for (int j = 0; j < H; ++j)
                acc[i][j] = mfma16<TERMS>(ah[i], bh[j], acc[i][j]);
    };
    constexpr bool PIPE = TERMS != 3;
    // The MFMA work of the panel in LDS buffer `cur`; `after_step(s)` runs
    // after step s's matrix instructions are issued.
    auto panel = [&](int cur, auto&& after_step) {
        bf16x8 ah[V], bh[H], al[V], bl[H];
        if (PIPE) read_step(cur, 0, ah, al, bh, bl);
#pragma unroll
        for (int s = 0; s < STEPS; ++s) {
            bf16x8 nah[V], nbh[H], nal[V], nbl[H];
            if (!PIPE) read_step(cur, s, ah, al, bh, bl);
            else if (s + 1 < STEPS) read_step(cur, s + 1, nah, nal, nbh, nbl);
            mfma_step(ah, al, bh, bl);
            after_step(s);
            if (PIPE && s + 1 < STEPS) {
#pragma unroll
                for (int i = 0; i < V; ++i) ah[i] = nah[i];
#pragma unroll
                for (int j = 0; j < H; ++j) bh[j] = nbh[j];
            }
        }
    };

    if constexpr (PACKED && TERMS != 3 && WM * WN < 128 * 128) {
        // Pre-packed single-term operands: two register staging sets, so the
        // panel packed during panel kt (panel kt+1) was fetched a whole panel
        // earlier and its LDS writes are spread between panel kt's matrix
        // instructions instead of forming a burst before the barrier.  (Not
        // with 128 x 128 wave tiles, whose accumulators leave no room for the
        // second set.)
        using PA = typename BfLoaderSel<PACKED, BM, BK, LDR, NT, !TA, TERMS>::type;
        using PB = typename BfLoaderSel<PACKED, BN, BK, LDR, NT, TB, TERMS>::type;
        PA pa0, pa1;
        PB pb0, pb1;
        const uint16_t* qa = reinterpret_cast<const uint16_t*>(g.A);
        const uint16_t* qb = reinterpret_cast<const uint16_t*>(g.B);
        auto load = [&](PA& xa, PB& xb, int kp) {
            xa.load(qa, g.plane_a, g.lda, m0, int64_t(kp) * BK, tid);
            xb.load(qb, g.plane_b, g.ldb, n0, int64_t(kp) * BK, tid);
        };
        if (nk > 0) {
            load(pa0, pb0, 0);
            load(pa1, pb1, nk > 1 ? 1 : 0);
            pa0.store(As[0][0], As[0][NL - 1], tid);
            pb0.store(Bs[0][0], Bs[0][NL - 1], tid);
        }
        __syncthreads();
        for (int kt = 0; kt < nk; kt += 2) {
            // panel kt in LDS 0; panel kt+1 (staging 1) goes to LDS 1
            load(pa0, pb0, kt + 2 < nk ? kt + 2 : nk - 1);
            panel(0, [&](int s) {
#pragma unroll
                for (int q = s; q < PA::PER; q += STEPS) pa1.store_chunk(As[1][0], As[1][NL - 1], tid, q);
#pragma unroll
                for (int q = s; q < PB::PER; q += STEPS) pb1.store_chunk(Bs[1][0], Bs[1][NL - 1], tid, q);
            });
            __syncthreads();
            if (kt + 1 < nk) {
                // panel kt+1 in LDS 1; panel kt+2 (staging 0) goes to LDS 0
                load(pa1, pb1, kt + 3 < nk ? kt + 3 : nk - 1);
                panel(1, [&](int s) {
#pragma unroll
                    for (int q = s; q < PA::PER; q += STEPS) pa0.store_chunk(As[0][0], As[0][NL - 1], tid, q);
#pragma unroll
                    for (int q = s; q < PB::PER; q += STEPS) pb0.store_chunk(Bs[0][0], Bs[0][NL - 1], tid, q);
                });
                __syncthreads();
            }
        }
    } else {
        if (nk > 0) {
            fetch(0);
            pack(0);
        }
        __syncthreads();
        // The next panel is converted and packed after the last MFMA step:
        // packing half-way through the panel was measured slower here (the
        // conversion's registers then overlap the fragments').
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < nk) fetch(int64_t(kt + 1) * BK);
            panel(cur, [](int) {});
            // Keep the pack (which waits for this iteration's global loads)
            // after the MFMAs: the compiler may otherwise hoist the LDS writes
            // above them, since they target the other buffer.
            __builtin_amdgcn_sched_barrier(0);
            pack(cur ^ 1);   // the last panel rewrites stale data nobody reads
            __syncthreads();
        }
    }

    // Epilogue: C = alpha*acc + beta*C0 (C0 not read when beta == 0).
    const float alpha = g.alpha, beta = g.beta;
    store_acc_blocks<V, H>(g.C, g.ldc, g.M, g.N, m0 + wm0, n0 + wn0, h, c, beta != 0.f, acc,
                           [&](float a, float c0) { return beta != 0.f ? __builtin_fmaf(alpha, a, beta * c0) : alpha * a; });
}

}  // namespace mg
