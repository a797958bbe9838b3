"""The blocking model of Section 3.1 (Eq. 1-7), restated for one MI355X.

The paper derives its cache-blocking factors from the cache sizes (Eq. 1-4:
kc from L1, mc from L2, nc from L3), requires them to be multiples of the
register tile (Eq. 5-7) and leaves only the register tile mr x kr x nr to
tuning.  On the GPU every blocking level is a tile shape of a compiled kernel
(workgroup tile BM x BN, LDS panel depth BK, wave tile WM x WN), and the
memories play these roles:

  * LDS (160 KiB per compute unit) is the L1 of Eq. 1-2: it holds the
    double-buffered BM x BK and BK x BN panels a workgroup packs (Eq. 1), and
    the workgroups resident on one compute unit share it;
  * the register file (512 registers per lane on each SIMD) is the vector
    register file of Eq. 2: each wave keeps its WM x WN block of C there for
    the whole K loop, beside its operand fragments;
  * the L2 of an XCD (4 MiB, shared by its 32 compute units) and the 256 MiB
    Infinity Cache are the L2 and L3 of Eq. 3-4: the panels of the tiles
    running at once on an XCD are re-read from L2, and operands that fit the
    Infinity Cache are re-read from it instead of HBM;
  * Eq. 5-7 become BM % WM = BN % WN = 0 and BK a multiple of the matrix
    instruction's depth kr.

The GPU adds a constraint the paper's single core does not have: the tiles
(times the K ranges of a split) are the work items of 256 compute units, so
the number of rounds of workgroups and how full the last one is matter as
much as the tile's own efficiency.

`candidates()` applies these constraints to the compiled configurations of a
path and to K-range counts, ranks what survives with a simple time model, and
returns the few the autotuner then measures (the paper's "only mr, kr, nr need
tuning" does not carry over: here the model prunes, the measurement decides).
This module is host-side planning only; it computes no part of a GEMM.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

# MI355X (gfx950) facts used by the model.
CUS = 256
LDS_BYTES = 160 * 1024
VGPRS_PER_SIMD_LANE = 512
SIMDS_PER_CU = 4
MAX_WAVES_PER_SIMD = 8
L2_BYTES_PER_XCD = 4 << 20
CUS_PER_XCD = 32
MALL_BYTES = 256 << 20
HBM_BYTES_PER_S = 8.0e12

# Paths of mg_gemm (and the INT8 table, 5).
FP32, BF16X3, BF16, FP8, FP16, I8 = 0, 1, 2, 3, 4, 5
# Spec peak of the matrix instructions each path issues (TFLOP/s), and how
# many of them one useful multiply-add costs.
PEAK = {FP32: 157.3, BF16X3: 2516.6, BF16: 2516.6, FP16: 2516.6, FP8: 5033.2, I8: 5033.2}
ISSUED = {FP32: 1, BF16X3: 3, BF16: 1, FP16: 1, FP8: 1, I8: 1}
# depth of one matrix instruction (kr)
KR = {FP32: 2, BF16X3: 16, BF16: 16, FP16: 16, FP8: 64, I8: 32}
# bytes of one operand element as the GEMM kernel reads it (bf16x3: two
# 16-bit terms), and as it sits in LDS
OPERAND_BYTES = {FP32: 4, BF16X3: 4, BF16: 2, FP16: 2, FP8: 1, I8: 1}
# fraction of the spec peak a tile class sustains when every compute unit is
# busy (measured on MI355X at 8192^3-class sizes: FP32 256x256 88 %, 128x128
# 79 %, 64x64 77 %; the 16-bit and 8-bit kernels about half their peak)
SUSTAINED = {FP32: {256: 0.88, 128: 0.79, 64: 0.77}, BF16X3: {256: 0.52, 128: 0.42, 64: 0.30},
             BF16: {256: 0.50, 128: 0.40, 64: 0.28}, FP16: {256: 0.47, 128: 0.38, 64: 0.27},
             FP8: {256: 0.48, 128: 0.38, 64: 0.25}, I8: {256: 0.45, 128: 0.36, 64: 0.25}}
MIN_RANGE = 256          # shortest K range a split may leave (the library's kMinRange)
SPLIT_GRAIN = 128        # K ranges are whole multiples of this
SPLITS = (1, 2, 3, 4, 6, 8)
MAX_PAD = 1.5            # padded tile area over the problem's area


@dataclass(frozen=True)
class Config:
    path: int
    id: int
    bm: int
    bn: int
    bk: int
    wm: int
    wn: int
    packs: bool
    mfma: bool

    @property
    def waves(self) -> int:
        return (self.bm // self.wm) * (self.bn // self.wn)

    @property
    def lds_bytes(self) -> int:
        """Two stages of a BM x BK and a BK x BN panel (Eq. 1); unpacked
        configurations use no LDS.  The 16-bit direct-copy configurations
        (BK 64) hold 128-byte panel rows whatever the kind: 64 k of BF16 or
        FP16, or 32 k of bf16x3's two terms."""
        if not self.packs:
            return 0
        if self.path in (BF16X3, BF16, FP16) and self.bk == 64:
            return 2 * (self.bm + self.bn) * 128
        return 2 * (self.bm + self.bn) * self.bk * OPERAND_BYTES[self.path]

    @property
    def acc_registers(self) -> int:
        """FP32 accumulator registers per lane of one wave (C's block, Eq. 2)."""
        return self.wm * self.wn // 64

    def occupancy(self) -> int:
        """Workgroups one compute unit holds at once: LDS (Eq. 1), the
        register file (Eq. 2; accumulators plus 64 registers of fragments and
        addresses per wave, in whole waves per SIMD) and wave slots."""
        by_lds = LDS_BYTES // self.lds_bytes if self.lds_bytes else 8
        per_wave = self.acc_registers + 64
        waves_per_simd = max(1, min(MAX_WAVES_PER_SIMD, VGPRS_PER_SIMD_LANE // per_wave))
        by_regs = max(1, (waves_per_simd * SIMDS_PER_CU) // self.waves)
        return max(1, min(by_lds, by_regs))


def feasible(c: Config) -> list[str]:
    """The constraints a configuration violates (empty: admissible)."""
    bad = []
    if c.lds_bytes > LDS_BYTES:
        bad.append("Eq. 1: panels exceed LDS")
    if c.acc_registers + 16 > VGPRS_PER_SIMD_LANE:
        bad.append("Eq. 2: accumulators exceed the register file")
    if c.bm % c.wm or c.bn % c.wn:
        bad.append("Eq. 6-7: BM, BN not multiples of the wave tile")
    if c.mfma and c.bk % KR[c.path] and c.path in (FP32,):
        bad.append("Eq. 5: BK not a multiple of kr")
    if c.wm % 32 or c.wn % 32:
        bad.append("Eq. 6-7: wave tile not a multiple of the 32 x 32 instruction")
    return bad


def tiles(M: int, N: int, c: Config) -> int:
    return math.ceil(M / c.bm) * math.ceil(N / c.bn)


def effective_splits(K: int, s: int) -> int:
    """K ranges the library cuts for a requested count s (a range length of
    ceil(K / s) rounded up to a multiple of 128)."""
    if s < 2 or K < 2 * SPLIT_GRAIN:
        return 1
    chunk = math.ceil(math.ceil(K / s) / SPLIT_GRAIN) * SPLIT_GRAIN
    return math.ceil(K / chunk)


def l2_window_bytes(c: Config, occupancy: int, group_m: int = 4) -> int:
    """Bytes of the K panels that the tiles running at once on one XCD read
    per K step (Eq. 3-4): the raster walks group_m tile rows, so the XCD's
    32 x occupancy tiles span group_m row panels of A and the rest as column
    panels of B."""
    resident = CUS_PER_XCD * occupancy
    cols = max(1, resident // group_m)
    return (group_m * c.bm + cols * c.bn) * c.bk * OPERAND_BYTES[c.path] * 2


def model_us(c: Config, M: int, N: int, K: int, splits: int, beta_nonzero: bool = True) -> float:
    """Predicted time of one GEMM with configuration c and `splits` K ranges:
    the matrix work at the tile class's sustained rate, stretched by the
    rounds of workgroups over the compute units (a part-empty last round
    costs a full one), or the HBM traffic if that is longer (operands re-read
    from HBM unless they fit the Infinity Cache), plus the split's reduction
    (read every partial and C, write C once)."""
    cls = 256 if min(c.bm, c.bn) >= 256 else 128 if min(c.bm, c.bn) >= 128 else 64
    rate = PEAK[c.path] * 1e12 / ISSUED[c.path] * SUSTAINED[c.path][cls]
    if not c.mfma:
        rate *= 0.6
    occ = c.occupancy()
    items = tiles(M, N, c) * splits
    slots = CUS * occ
    rounds = math.ceil(items / slots)
    fill = items / (rounds * slots)
    padded = math.ceil(M / c.bm) * c.bm * math.ceil(N / c.bn) * c.bn
    t_mfma = 2.0 * padded * K / rate / max(fill, 1e-9)
    ob = OPERAND_BYTES[c.path] if c.path != BF16X3 else 4
    a_bytes, b_bytes = M * K * ob, K * N * ob
    if a_bytes + b_bytes <= MALL_BYTES:
        reads = a_bytes + b_bytes
    else:
        # re-reads of the operand that does not stay cached: A once per
        # column of tiles beyond what the MALL keeps, approximated as B kept
        reads = a_bytes + b_bytes * max(1.0, (a_bytes + b_bytes) / MALL_BYTES)
    c_bytes = 4.0 * M * N * (2 if beta_nonzero else 1)
    t_mem = (reads + c_bytes) / HBM_BYTES_PER_S
    t = max(t_mfma, t_mem)
    if splits > 1:
        t += 4.0 * (splits + 1) * M * N / HBM_BYTES_PER_S + 5e-6
    return t * 1e6


def candidates(configs: list[Config], M: int, N: int, K: int, keep: int = 12, allow_split: bool = True):
    """Admissible (configuration, K ranges) pairs for an M x N x K GEMM, best
    predicted first, at most `keep`: each admissible configuration offers its
    best predicted K-range count and its unsplit plan, so every tile shape
    is measured both ways."""
    scored = []
    for c in configs:
        # the vector-ALU micro-kernels exist for the engine comparison, and
        # unpacked tiles only pay below about 64^3 (the packing ablation)
        if feasible(c) or not c.mfma or (not c.packs and max(M, N, K) > 128):
            continue
        pad = math.ceil(M / c.bm) * c.bm * math.ceil(N / c.bn) * c.bn / float(M * N)
        if pad > MAX_PAD:
            continue
        splits = SPLITS if (allow_split and c.path not in (FP8, I8)) else (1,)
        opts = {}
        for s in splits:
            se = effective_splits(K, s)
            if se > 1 and K // se < MIN_RANGE:
                continue
            opts.setdefault(se, model_us(c, M, N, K, se))
        best_s = min(opts, key=opts.get)
        for se in {1, best_s}:
            scored.append((opts[se], c.id, se))
    if not scored:   # every tile pads too much: keep the smallest tiles unsplit
        small = min((c for c in configs if not feasible(c)), key=lambda c: c.bm * c.bn)
        return [(small.id, 1)]
    scored.sort()
    return [(cid, s) for _, cid, s in scored[:keep]]


def library_configs(native, path: int) -> list[Config]:
    """The compiled configurations of a path, as the library describes them."""
    out = []
    for i in range(native.mg_num_configs(path)):
        c = native.mg_config_info(path, i)
        out.append(Config(path, c["id"], c["bm"], c["bn"], c["bk"], c["wm"], c["wn"],
                          native.mg_config_packs(path, i) == 1, native.mg_config_uses_mfma(path, i) == 1))
    return out
