"""Host-side model of the direct-copy panel layout (tile_bytes.h) and of
bf16x3's interleaved planes (gemm_bf16.hip), checked on the CPU.

The direct kernels copy packed 128-byte rows from global memory into LDS with
an instruction that writes lane l's 16 bytes at the wave's LDS base + 16 l, so
the bank swizzle is made on the source side: copy j of wave w fills LDS chunk
slot s = (j NW + w) 64 + l, which is row s / 8, and it fetches global chunk
(s mod 8) XOR swz(row), swz(r) = (r >> 1) mod 8.  A fragment read of global
chunk g of row r then looks at LDS chunk g XOR swz(r).  These tests restate
that index algebra and check what the kernels rely on: every LDS chunk is
written exactly once, every fragment read finds the global chunk it asks
for, and 16 consecutive rows read at one chunk fall on 16 distinct 16-byte
bank groups.  The GPU parity tests check the kernels themselves.
"""
import numpy as np
import pytest


def swz(r):
    return (r >> 1) & 7


def direct_copy_model(panel, rows, nw):
    """LDS image (rows x 128 bytes) written by direct_copy<rows, nw> from a
    rows x 128 global panel."""
    lds = np.full(rows * 128, -1, dtype=np.int64)
    copies = rows * 8 // (nw * 64)
    assert rows * 8 % (nw * 64) == 0
    for w in range(nw):
        for j in range(copies):
            for lane in range(64):
                slot = (j * nw + w) * 64 + lane
                r = slot >> 3
                src = 16 * ((slot & 7) ^ swz(r))
                dst = (j * nw + w) * 1024 + 16 * lane
                assert np.all(lds[dst:dst + 16] == -1), "an LDS chunk written twice"
                lds[dst:dst + 16] = panel[r, src:src + 16]
    return lds


def direct_chunk_model(lds, row, g):
    off = row * 128 + 16 * (g ^ swz(row))
    return lds[off:off + 16]


@pytest.mark.parametrize("rows,nw", [(256, 8), (128, 4), (256, 4), (128, 8)])
def test_copy_then_fragment_reads_recover_the_global_panel(rows, nw):
    panel = np.arange(rows * 128, dtype=np.int64).reshape(rows, 128)
    lds = direct_copy_model(panel, rows, nw)
    assert np.all(lds >= 0)                        # every LDS byte written
    for r in range(rows):
        for g in range(8):
            assert np.array_equal(direct_chunk_model(lds, r, g), panel[r, 16 * g:16 * g + 16])


def test_sixteen_rows_at_one_chunk_hit_distinct_bank_groups():
    for r0 in range(0, 256, 16):
        for g in range(8):
            groups = {((r * 128 + 16 * (g ^ swz(r))) // 16) % 16 for r in range(r0, r0 + 16)}
            assert len(groups) == 16


def test_fragment_chunks_per_type():
    """The chunk each lane half reads per MFMA step covers a panel row exactly
    once: FP8 (two chunks per 64-deep step), INT8 / BF16 / FP16 (one chunk per
    step, 32 bytes of k per step), bf16x3 (hi chunk 2s + h, lo chunk 4 + 2s + h)."""
    fp8 = sorted(c for s in range(2) for h in range(2) for c in (4 * s + 2 * h, 4 * s + 2 * h + 1))
    one = sorted(2 * s + h for s in range(4) for h in range(2))
    x3 = sorted(c for s in range(2) for h in range(2) for c in (2 * s + h, 4 + 2 * s + h))
    assert fp8 == one == x3 == list(range(8))


def interleaved_index(k):
    """Element offsets of hi(k) and lo(k) in a bf16x3 interleaved row."""
    return 64 * (k >> 5) + (k & 31), 64 * (k >> 5) + (k & 31) + 32


@pytest.mark.parametrize("Kp", [128, 384, 8192])
def test_interleaved_planes_are_a_bijection_and_match_the_kernel_reads(Kp):
    hi = np.array([interleaved_index(k)[0] for k in range(Kp)])
    lo = np.array([interleaved_index(k)[1] for k in range(Kp)])
    both = np.concatenate([hi, lo])
    assert both.min() == 0 and both.max() == 2 * Kp - 1 and len(np.unique(both)) == 2 * Kp
    # the pack writes 8 consecutive k as one 16-byte chunk: they stay in one
    # 32-k group, so hi and lo of the chunk are contiguous
    for k0 in range(0, Kp, 8):
        assert np.array_equal(hi[k0:k0 + 8], hi[k0] + np.arange(8))
        assert np.array_equal(lo[k0:k0 + 8], lo[k0] + np.arange(8))
    # the kernel reads panel kp as the 128-byte row at element 64 kp: lane half
    # h of step s takes hi from chunk 2s + h and lo from chunk 4 + 2s + h, and
    # both must hold k = 32 kp + 16 s + 8 h .. +7
    for kp in range(Kp // 32):
        for s in range(2):
            for h in range(2):
                ks = 32 * kp + 16 * s + 8 * h + np.arange(8)
                assert np.array_equal(hi[ks], 64 * kp + 8 * (2 * s + h) + np.arange(8))
                assert np.array_equal(lo[ks], 64 * kp + 8 * (4 + 2 * s + h) + np.arange(8))


def test_split_k_ranges_start_on_whole_interleaved_rows():
    """Split K cuts K into ranges that are multiples of 128, so a range's
    first k sits at byte 4 k0 of a row, a whole number of 128-byte panels."""
    for k0 in range(0, 4096, 128):
        assert (4 * k0) % 128 == 0
        assert interleaved_index(k0)[0] * 2 == 4 * k0
