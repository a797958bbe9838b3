"""The blocking model (the Eq. 1-7 analogue of blocking.py) on the library's
compiled configurations: what it admits, what it prunes and why."""
import pytest

from paper_2305_18236_amd import blocking


@pytest.fixture(scope="module")
def native():
    from paper_2305_18236_amd import _native
    _native.lib()
    return _native


@pytest.mark.parametrize("path", [0, 1, 2, 3, 4, 5])
def test_every_compiled_configuration_satisfies_the_model(native, path):
    """The compiled tiles were chosen to fit: Eq. 1 (two panel stages within
    160 KiB of LDS), Eq. 2 (accumulators within the register file), Eq. 5-7
    (divisibility)."""
    for c in blocking.library_configs(native, path):
        assert blocking.feasible(c) == [], (c, blocking.feasible(c))
        assert c.lds_bytes <= blocking.LDS_BYTES
        assert c.occupancy() >= 1


def test_lds_bytes_of_known_configurations(native):
    cfg = {c.id: c for c in blocking.library_configs(native, 0)}
    assert cfg[5].lds_bytes == 2 * (256 + 256) * 16 * 4          # 64 KiB, FP32 256x256x16
    b3 = {c.id: c for c in blocking.library_configs(native, 1)}
    assert b3[6].lds_bytes == 128 * 1024                          # 128-byte rows, two stages
    assert b3[6].occupancy() == 1 and b3[7].occupancy() == 2


def test_violations_are_named():
    big = blocking.Config(0, 99, 512, 512, 64, 128, 128, True, True)     # 512 KiB of panels
    assert any("Eq. 1" in v for v in blocking.feasible(big))
    odd = blocking.Config(0, 98, 192, 128, 32, 128, 64, True, True)     # 192 % 128 != 0
    assert any("Eq. 6-7" in v for v in blocking.feasible(odd))
    regs = blocking.Config(0, 97, 512, 512, 8, 512, 512, True, True)    # 4096 accumulators per lane
    assert any("Eq. 2" in v for v in blocking.feasible(regs))


def test_effective_splits_match_the_library(native):
    for K in (256, 300, 1000, 1536, 4096, 8192):
        for s in (1, 2, 3, 4, 6, 8):
            assert native.mg_force_splits(0, s) == 0
            try:
                got = native.mg_split_count(0, 64, 64, K)
            finally:
                native.mg_force_splits(0, -1)
            assert got == blocking.effective_splits(K, s), (K, s)


def test_candidates_prune_padding_and_short_ranges(native):
    cfgs = blocking.library_configs(native, 0)
    # 96 x 96: 256 x 256 tiles would pad the area 7x; never offered
    for cid, s in blocking.candidates(cfgs, 96, 96, 4096):
        c = {c.id: c for c in cfgs}[cid]
        assert c.bm <= 128 and c.bn <= 128
    # K = 512: no split may leave ranges shorter than 256
    for cid, s in blocking.candidates(cfgs, 4096, 4096, 512):
        assert s == 1 or 512 // s >= blocking.MIN_RANGE
    # FP8 never splits; the vector-ALU kernels are never offered
    assert all(s == 1 for _, s in blocking.candidates(blocking.library_configs(native, 3), 1024, 1024, 8192))
    valu = {c.id for c in cfgs if not c.mfma}
    assert not valu & {cid for cid, _ in blocking.candidates(cfgs, 8192, 8192, 8192)}


def test_round_model_prefers_full_rounds(native):
    """The GPU-specific term: at equal work, a plan whose workgroups fill
    their rounds is predicted faster than one that leaves a last round
    nearly empty (3072^3 in 256 x 256 tiles: 144 tiles on 256 compute
    units, 56 % of one round, against 2304 tiles of 64 x 64, five per
    compute unit, filling 90 % of two rounds; measured 784 against 512 us)."""
    cfg = {c.id: c for c in blocking.library_configs(native, 0)}
    t_big = blocking.model_us(cfg[5], 3072, 3072, 3072, 1)       # 144 tiles: 56 % of one round
    t_small = blocking.model_us(cfg[3], 3072, 3072, 3072, 1)     # 2304 tiles, 5 per CU
    assert t_small < t_big
    # and at 8192^3 (1024 tiles, four whole rounds) the big tile wins
    assert blocking.model_us(cfg[5], 8192, 8192, 8192, 1) < blocking.model_us(cfg[3], 8192, 8192, 8192, 1)
