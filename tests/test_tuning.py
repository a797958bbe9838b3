"""Host-side checks of the tuning table and of batched-argument validation
(no device call is made by anything tested here)."""
import ctypes
import os

import pytest

from paper_2305_18236_amd import autotune


@pytest.fixture()
def native():
    from paper_2305_18236_amd import _native
    _native.lib()
    yield _native
    # restore the default table
    _native.mg_load_tuning(None)
    _native._load_default_tuning(_native.lib())


@pytest.fixture()
def rule(native):
    """The library with no tuning table: the built-in rule alone decides
    (the native fixture restores the committed table afterwards)."""
    native.mg_load_tuning(None)
    return native


def test_bucket_rule_matches_library(native, tmp_path):
    # a table that maps every (mb, nb, kb) of path 0 to a config derived from mb
    n = native.mg_num_configs(0)
    lines = [f"0 {mb} {nb} {kb} {mb % n}" for mb in range(21) for nb in (10,) for kb in (10,)]
    p = tmp_path / "t.txt"
    p.write_text("# test\n" + "\n".join(lines) + "\n")
    assert native.mg_load_tuning(str(p)) == 0
    for M in [1, 2, 3, 5, 6, 7, 11, 12, 13, 23, 24, 25, 95, 96, 97, 1000, 1536, 1535, 3000, 10 ** 6, 10 ** 9]:
        assert native.mg_tuned_config(0, M, 1024, 1024) == autotune.bucket(M) % n, M


def test_table_selection_order(native, tmp_path):
    p = tmp_path / "t.txt"
    p.write_text("0 8 8 8 3\n1 8 8 8 2\n")
    assert native.mg_load_tuning(str(p)) == 0
    assert native.mg_tuned_config(0, 256, 256, 256) == 3
    assert native.mg_tuned_config(1, 256, 256, 256) == 2
    # forced configuration wins over the table
    assert native.mg_force_config(0, 1) == 0
    try:
        assert native.mg_tuned_config(0, 256, 256, 256) == 1
    finally:
        native.mg_force_config(0, -1)
    # untuned buckets use the built-in rule: the same as with no table at all
    untuned = native.mg_tuned_config(0, 8192, 8192, 8192)
    native.mg_load_tuning(None)
    assert native.mg_tuned_config(0, 8192, 8192, 8192) == untuned


def test_batched_entries_do_not_steer_single_gemms(native, tmp_path):
    p = tmp_path / "t.txt"
    p.write_text("0 8 8 8 3 b\n1 8 8 8 4 b\n")
    assert native.mg_load_tuning(str(p)) == 0
    assert native.mg_batched_config(0, 256, 256, 256) == 3
    assert native.mg_batched_config(1, 256, 256, 256) == 4
    native.mg_load_tuning(None)
    untuned = native.mg_tuned_config(0, 256, 256, 256)
    assert native.mg_load_tuning(str(p)) == 0
    assert native.mg_tuned_config(0, 256, 256, 256) == untuned
    # an 's' entry steers single GEMMs, and the batched kernel when it is a batched variant
    p.write_text("0 8 8 8 3 s\n")
    assert native.mg_load_tuning(str(p)) == 0
    assert native.mg_tuned_config(0, 256, 256, 256) == 3
    assert native.mg_batched_config(0, 256, 256, 256) == 3


@pytest.mark.parametrize("text", ["0 8 8 8\n", "0 8 8 8 99\n", "7 8 8 8 0\n", "0 30 8 8 0\n", "x y z\n",
                                  "0 8 8 8 3 q\n", "0 8 8 8 3 bb\n"])
def test_malformed_table_rejected_and_previous_kept(native, tmp_path, text):
    good = tmp_path / "good.txt"
    good.write_text("0 8 8 8 3\n")
    assert native.mg_load_tuning(str(good)) == 0
    bad = tmp_path / "bad.txt"
    bad.write_text(text)
    assert native.mg_load_tuning(str(bad)) == -103
    assert native.mg_tuned_config(0, 256, 256, 256) == 3


def test_missing_table_file(native, tmp_path):
    assert native.mg_load_tuning(str(tmp_path / "nope.txt")) == -103


def test_committed_table_parses(native):
    path = native.TUNING_TABLE
    if not os.path.exists(path):
        pytest.skip("no tuning table committed")
    assert native.mg_load_tuning(path) == 0


def test_autotune_pruning():
    # 64 x 64 tiles never waste more than 4x area; 256 x 256 tiles on a 40 x 40 problem do
    assert autotune.padded_area_ratio(40, 40, 64, 64) <= 4.0
    assert autotune.padded_area_ratio(40, 40, 256, 256) > 4.0


FAKE = 0x1000


def _problem(native, **kw):
    a = dict(transA=b"N", transB=b"N", M=4, N=5, K=6, alpha=1.0, beta=0.0, A=FAKE, lda=6,
             B=FAKE, ldb=5, C=FAKE, ldc=5)
    a.update(kw)
    return native.mg_problem(a["transA"], a["transB"], a["M"], a["N"], a["K"], a["alpha"], a["beta"],
                             a["A"], a["lda"], a["B"], a["ldb"], a["C"], a["ldc"])


def test_batched_validation_reports_the_bad_problem(native):
    arr = (native.mg_problem * 4)(_problem(native), _problem(native), _problem(native, ldb=2),
                                  _problem(native, transA=b"Q"))
    st, bad = native.mg_gemm_batched(0, 4, arr, FAKE, 1 << 20, None)
    assert (st, bad) == (-10, 2)
    st, bad = native.mg_gemm_batched(0, -1, arr, FAKE, 1 << 20, None)
    assert st == -2
    st, bad = native.mg_gemm_batched(3, 4, arr, FAKE, 1 << 20, None)
    assert st == -101
    # valid problems but no workspace: rejected before any device call
    ok = (native.mg_problem * 2)(_problem(native), _problem(native))
    st, bad = native.mg_gemm_batched(0, 2, ok, None, 0, None)
    assert st == -100
    assert native.mg_gemm_batched_workspace_size(0, 2) > 0
    assert native.mg_gemm_batched_workspace_size(3, 2) == 0
    # an all-empty batch is a no-op
    empty = (native.mg_problem * 2)(_problem(native, M=0, A=None, C=None), _problem(native, N=0, B=None, C=None, ldb=1, ldc=1))
    st, bad = native.mg_gemm_batched(0, 2, empty, FAKE, 1 << 20, None)
    assert st == 0


def test_problem_struct_layout(native):
    # the C struct has natural alignment: char, char, pad, 3 x int64, 2 x float, 6 x (ptr/int64)
    assert ctypes.sizeof(native.mg_problem) == 8 + 24 + 8 + 48


def test_force_tile_order_validation(native):
    """The tile-order override takes remap 0/1 with group_m 1..64 on the six
    configuration tables, and -1 (any group) returns to the automatic order."""
    try:
        for path in range(6):
            assert native.mg_force_tile_order(path, 0, 1) == 0
            assert native.mg_force_tile_order(path, 1, 64) == 0
            assert native.mg_force_tile_order(path, -1, 0) == 0
        for remap, gm in ((2, 4), (-2, 4), (0, 0), (1, 65), (0, -3)):
            assert native.mg_force_tile_order(0, remap, gm) == -101
        assert native.mg_force_tile_order(6, 0, 4) == -101
        assert native.mg_force_tile_order(-1, 0, 4) == -101
    finally:
        for path in range(6):
            native.mg_force_tile_order(path, -1)


def test_split_plan_rules(rule):
    native = rule
    """Host-side split-K plan: ranges are multiples of 128 deep, K < 256 never
    splits, forcing is validated, and the workspace covers the partials."""
    try:
        assert native.mg_force_splits(0, 4) == 0
        assert native.mg_split_count(0, 64, 64, 1000) == 4      # ranges of 256
        assert native.mg_split_count(0, 64, 64, 300) == 3       # ranges of 128
        assert native.mg_split_count(0, 64, 64, 255) == 1       # too short to split
        assert native.mg_split_count(3, 64, 64, 4096) == 1      # FP8 never splits
        assert native.mg_gemm_workspace_size(0, "N", "N", 64, 66, 1000) == 4 * 64 * 68 * 4
        assert native.mg_force_splits(0, 1) == 0
        assert native.mg_split_count(0, 64, 64, 1000) == 1
        assert native.mg_gemm_workspace_size(0, "N", "N", 64, 66, 1000) == 0
        for bad in (0, -2, 17):
            assert native.mg_force_splits(0, bad) == -101
        assert native.mg_force_splits(7, 2) == -101
    finally:
        native.mg_force_splits(0, -1)
    # automatic rule: a problem with enough tiles for every compute unit never splits
    assert native.mg_split_count(0, 8192, 8192, 8192) == 1
    assert native.mg_gemm_workspace_size(0, "N", "N", 8192, 8192, 8192) == 0
    # one tile and a long K splits into ranges at least 256 deep
    s = native.mg_split_count(0, 64, 64, 4096)
    assert 2 <= s <= 16 and 4096 / s >= 256 - 128


def test_sixteen_bit_direct_copy_choice(rule):
    native = rule
    """16-bit problems large enough for pre-packed planes and for 256 x 256
    tiles take configuration 6 (the same tiles, panels copied straight into
    LDS); problems too small to pre-pack, or beyond the planes' K limit,
    keep configuration 1.  bf16x3 then asks for workspace for its
    interleaved planes."""
    # (BF16 and FP16 over sixteen waves: 11)
    for path in (1, 2, 4):
        assert native.mg_tuned_config(path, 8192, 8192, 8192) == (6 if path == 1 else 11)
        assert native.mg_tuned_config(path, 256, 8192, 8192) == 1          # M < 512: no planes
        assert native.mg_tuned_config(path, 8192, 8192, 2 ** 21 + 1) == 1  # beyond the planes' K limit
    # bf16x3 pre-splits only where both operands are re-read often enough
    # (or for the 128 x 128 direct tile, which 2048^3 takes unsplit)
    assert native.mg_tuned_config(1, 2048, 2048, 2048) == 10
    assert native.mg_tuned_config(1, 16384, 1024, 4096) == 1
    assert native.mg_tuned_config(1, 4096, 4096, 4096) == 6
    assert native.mg_tuned_config(1, 2048, 8192, 2048) == 6
    assert native.mg_tuned_config(1, 3072, 3072, 3072) == 6
    assert native.mg_tuned_config(1, 4096, 2048, 8192) == 6
    assert native.mg_tuned_config(1, 1024, 8192, 4096) == 1
    assert native.mg_tuned_config(1, 2048, 2048, 8192) == 1
    # interleaved hi/lo planes: 4 bytes per element of op(A) and op(B)^T
    assert native.mg_gemm_workspace_size(1, "N", "N", 8192, 8192, 8192) == 4 * 2 * 8192 * 8192
    assert native.mg_gemm_workspace_size(1, "N", "N", 256, 8192, 8192) > 0   # split-K partials only


def test_fp32_round_plan(rule):
    native = rule
    """Where the tile ladder's workgroups leave the last round on the compute
    units mostly empty, the FP32 rule re-plans tile and K ranges (3072^3:
    288 workgroups of 256 x 256 on 256 compute units before); shapes whose
    rounds come out whole keep the ladder's choice."""
    plan = lambda *s: (native.mg_tuned_config(0, *s), native.mg_split_count(0, *s))
    # the 256 x 256 tile runs as its two-staging-set form (17)
    assert plan(8192, 8192, 8192) == (17, 1)
    assert plan(4096, 4096, 4096) == (17, 1)
    assert plan(2048, 2048, 2048) == (18, 1)   # 128 x 128 unsplit, below
    assert plan(4096, 4096, 1024) == (17, 1)
    assert plan(256, 8192, 8192) == (17, 8)
    assert plan(8192, 8192, 256) == (20, 1)   # the 128 x 64 tile over eight waves
    # the 64 x 64 tile runs as its two-staging-set form (12), or with two K
    # groups (15) where its workgroups give each compute unit at most one
    assert plan(1024, 1024, 1024) == (15, 1)   # one workgroup per compute unit: two K groups
    assert plan(3072, 3072, 3072) == (12, 1)
    assert plan(6144, 6144, 6144) == (17, 4)
    assert plan(1536, 1536, 1536) == (12, 4)
    assert plan(1536, 1536, 4096) == (12, 4)
    # the workspace query follows the plan's K ranges
    assert native.mg_gemm_workspace_size(0, "N", "N", 1536, 1536, 4096) == 4 * 1536 * 1536 * 4
    # the 128 x 128 tile runs as eight waves with two staging sets (18)
    assert plan(1024, 4096, 1024) == (18, 1)
    assert plan(2048, 2048, 1024) == (18, 1)
    assert plan(3072, 4096, 4096) == (18, 1)
    # where the big tile would split K and unsplit 64 x 64 tiles give every
    # compute unit one or two workgroups, those run (two K groups, 15), up
    # to K = 4096; at K = 8192 the big tile's many short ranges stay
    assert plan(512, 2048, 2048) == (15, 1)
    assert plan(1024, 2048, 1024) == (15, 1)
    assert plan(2048, 1024, 2048) == (15, 1)
    assert plan(1024, 1024, 4096) == (15, 1)
    assert plan(512, 4096, 4096) == (15, 1)
    assert plan(1024, 2048, 8192) == (17, 8)
    assert plan(768, 1536, 8192) == (17, 13)
    # two K groups at two workgroups per compute unit only with K ranges of
    # 512 or more: shorter ones keep the one-group tile (12)
    # the same for the 128 x 128 tile (18) against split 256 x 256 tiles,
    # while K * tiles stays within 4096 per compute unit
    assert plan(4096, 1024, 2048) == (18, 1)
    assert plan(2048, 4096, 1024) == (18, 1)
    assert plan(2048, 2048, 4096) == (18, 1)
    assert plan(2048, 4096, 4096) == (17, 2)
    assert plan(2048, 2048, 8192) == (17, 4)
    # ... only where the smaller tiles' last round is at least 80 % full
    assert plan(3072, 1664, 3072) != (18, 1)   # 312 tiles of 128 x 128
    assert plan(896, 6144, 1536) != (18, 1)    # 336
    assert plan(1088, 1088, 2048) != (15, 1)   # 289 tiles of 64 x 64
    # tiles that keep 84 % of the compute units busy run whole up to K = 3072
    assert plan(7936, 2048, 1536) == (17, 1)   # 248 tiles of 256 x 256
    assert plan(2304, 6912, 768) == (17, 1)    # 243
    assert plan(768, 4992, 768) == (18, 1)     # 234 tiles of 128 x 128
    assert plan(3200, 4224, 8192) != (17, 1)   # longer K: no whole run
    # the round model decides wherever the last round is under 90 % full,
    # and weighs plans that keep 80 % of the compute units busy
    assert plan(3200, 4224, 8192) == (18, 4)   # 442 workgroups of 256 x 256: 86 %
    assert plan(3584, 3712, 3072) == (12, 1)   # 420: 82 %
    assert plan(7552, 1664, 8192) == (18, 1)   # 207 tiles of 128 x 128: 81 %
    assert plan(640, 3072, 8192) == (18, 2)   # 240 workgroups: 283.2 us against 292.4 for (15, 1)
    assert plan(640, 1536, 4096) == (15, 1)   # 240 tiles, 94 %: 84.5 us against 83.3 in two ranges
    assert plan(1536, 768, 128) == (12, 1)
    assert plan(512, 2560, 256) == (12, 1)
    assert plan(1024, 640, 512) == (12, 2)


def test_fp32_model_of_the_eight_wave_tile(rule):
    native = rule
    """Without the tuning table the rule plans 2048^3 as the committed
    table does: configuration 18, the 128 x 128 tile over eight waves,
    unsplit."""
    assert (native.mg_tuned_config(0, 2048, 2048, 2048), native.mg_split_count(0, 2048, 2048, 2048)) == (18, 1)
    native._load_default_tuning(native.lib())
    assert native.mg_tuned_config(0, 2048, 2048, 2048) == 18


def test_sixteen_bit_ladder_steps_down_from_split_k(rule):
    native = rule
    """Where 256 x 256 tiles would need a K split and unsplit 128 x 128 tiles
    fill the compute units, the 16-bit rule takes the 128 x 128 tile unsplit:
    on pre-packed planes as eight waves fed by direct copies (10).  bf16x3
    keeps the split for K ranges of 2048 or more; whole rounds of 256 x 256
    tiles stay; the 128 x 128 tile keeps its own split against 64 x 64 tiles;
    without pre-packed planes (M below 512) the in-kernel forms run."""
    for shape in ((2048, 2048, 1024), (1024, 4096, 1024), (2048, 2048, 2048), (4096, 2048, 2048),
                  (2560, 2560, 2560)):
        for path in (1, 2, 4):
            assert (native.mg_tuned_config(path, *shape), native.mg_split_count(path, *shape)) == (10, 1), \
                (path, shape)
    for path in (2, 4):
        assert native.mg_tuned_config(path, 2048, 2048, 8192) == 10
    assert native.mg_tuned_config(1, 2048, 2048, 8192) == 1 and native.mg_split_count(1, 2048, 2048, 8192) == 4
    for path in (1, 2, 4):
        assert native.mg_tuned_config(path, 3072, 3072, 3072) == (6 if path == 1 else 11)
    assert native.mg_tuned_config(1, 1024, 1024, 1024) == 2 and native.mg_split_count(1, 1024, 1024, 1024) == 4
    # 256 rows: no planes; 128 x 128 tiles (2 x 64 = 128) do not fill the
    # compute units, so the ladder's split stays
    assert native.mg_tuned_config(2, 256, 8192, 8192) == 1
    # K ranges of 512 or less: the step down already where 128 x 128 tiles
    # keep three quarters of the compute units busy (203-234 tiles)
    for path in (1, 2):
        for shape in ((3712, 896, 1024), (768, 4992, 768), (2048, 1664, 768)):
            assert (native.mg_tuned_config(path, *shape), native.mg_split_count(path, *shape)) == (10, 1), \
                (path, shape)
    # BF16 and FP16 also with ranges up to 1024 deep, bf16x3 not
    for path in (2, 4):
        assert (native.mg_tuned_config(path, 3584, 1152, 2048), native.mg_split_count(path, 3584, 1152, 2048)) == (10, 1)
        assert (native.mg_tuned_config(path, 2560, 1280, 3072), native.mg_split_count(path, 2560, 1280, 3072)) == (10, 1)
    assert native.mg_tuned_config(1, 2560, 1280, 3072) != 10
    # longer ranges keep the split there
    assert native.mg_split_count(2, 1792, 1920, 8192) == 4
    assert native.mg_tuned_config(2, 1792, 1920, 8192) == 11
    # unsplit 256 x 256 tiles spilling a second round under a quarter full
    # (270 and 312 tiles) step down too; 576 tiles (6144^2, a quarter) stay
    for path in (1, 2):
        for shape in ((4480, 3840, 256), (6144, 3328, 8192)):
            assert (native.mg_tuned_config(path, *shape), native.mg_split_count(path, *shape)) == (10, 1), \
                (path, shape)
    assert native.mg_tuned_config(2, 6144, 6144, 2048) == 11
    # bf16x3 steps down up to a third full (4096 x 5120: 320 tiles, 25 %;
    # 6144 x 3456: 336, 31 %); BF16 keeps the big tile there
    for shape in ((4096, 5120, 4096), (6144, 3456, 768)):
        assert native.mg_tuned_config(1, *shape) == 10, shape
    assert native.mg_tuned_config(2, 6144, 3456, 768) == 11


def test_sixteen_bit_short_k_ranges_take_64_tiles(rule):
    native = rule
    """BF16 and FP16: where the ladder's tile needs K ranges of 384 or less
    (K up to 2048, both sides at least 512) and 64 x 64 tiles alone give each
    compute unit one or two workgroups, those run unsplit (4); bf16x3 only
    up to K = 512; the narrow or long-K shapes keep the split."""
    for path in (2, 4):
        for shape in ((2176, 768, 512), (1280, 1280, 768), (2048, 1024, 1536)):
            assert (native.mg_tuned_config(path, *shape), native.mg_split_count(path, *shape)) == (4, 1), \
                (path, shape)
    assert (native.mg_tuned_config(1, 3328, 512, 512), native.mg_split_count(1, 3328, 512, 512)) == (4, 1)
    assert native.mg_tuned_config(1, 512, 2688, 768) != 4       # bf16x3 from K = 768
    assert native.mg_tuned_config(2, 256, 4480, 3072) != 4      # a side of 256
    assert native.mg_tuned_config(2, 512, 2176, 1536) != 4      # 512-deep ranges


def test_bf16x3_planes_bound(rule):
    native = rule
    """bf16x3 runs the 256 x 256 tile on pre-packed planes (6) once
    M N >= 1050 (M + N); below that its in-kernel form (1)."""
    assert native.mg_tuned_config(1, 5504, 1536, 4096) == 6     # 1201 (M + N)
    assert native.mg_tuned_config(1, 1536, 5760, 1024) == 6     # 1213
    assert native.mg_tuned_config(1, 2048, 2048, 8192) == 1     # 1024
    assert native.mg_tuned_config(1, 1024, 8192, 4096) == 1     # 910


def test_eight_bit_step_down_from_a_spilled_round(rule):
    native = rule
    """FP8 and INT8: 256 x 256 tiles that spill a second round under a
    quarter full (257-319 tiles) give way to the 128 x 128 direct tile;
    whole rounds and fuller second rounds keep the big tile."""
    for shape in ((4480, 3840, 256), (4352, 4096, 2048), (6144, 3328, 8192)):
        assert native.mg_tuned_config(3, *shape) == 10, shape
        assert native.mg_tuned_config(5, *shape) == 6, shape
    # FP8 up to a third full (330 tiles), INT8 a quarter
    assert native.mg_tuned_config(3, 3840, 5504, 1024) == 10
    assert native.mg_tuned_config(5, 3840, 5504, 1024) == 7
    for shape in ((4096, 4096, 4096), (6144, 6144, 2048)):
        assert native.mg_tuned_config(3, *shape) == 11, shape   # FP8: sixteen waves by rule
        assert native.mg_tuned_config(5, *shape) == 7, shape


def test_sixteen_bit_split_rule(rule):
    native = rule
    """16-bit paths split K into as many ranges as fit one round of
    workgroups (rounded down), unless unsplit 128 x 128 tiles fill the
    compute units (then those run, see the step-down test)."""
    for path in (1, 2, 4):
        assert native.mg_split_count(path, 3072, 3072, 3072) == 1     # 144 tiles of 256 x 256
        assert native.mg_split_count(path, 3072, 3072, 1024) == 1
        assert native.mg_split_count(path, 2560, 2560, 2560) == 1     # 400 tiles of 128 x 128
        assert native.mg_split_count(path, 1536, 1536, 4096) == 7     # 36 tiles: 252 workgroups
        assert native.mg_split_count(path, 2048, 2048, 2048) == 1     # 256 tiles of 128 x 128
        assert native.mg_split_count(path, 8192, 8192, 8192) == 1
    # 128 tiles of 256 x 256 in two ranges; BF16 and FP16 take 512 unsplit
    # 128 x 128 tiles instead, bf16x3 keeps 4096-deep ranges
    assert native.mg_split_count(1, 4096, 2048, 8192) == 2
    for path in (2, 4):
        assert native.mg_split_count(path, 4096, 2048, 8192) == 1


def test_fp8_big_tile_threshold(rule):
    native = rule
    """FP8 takes the 256 x 256 direct-copy tile, over sixteen waves, once
    its tiles keep more than half the compute units busy (FP8 never splits
    K); the tuned table keeps the eight-wave form where it measured that
    ahead (8192^3)."""
    assert native.mg_tuned_config(3, 3072, 3072, 3072) == 11    # 144 tiles
    # below that, 128 x 128 tiles over eight waves with direct copies
    assert native.mg_tuned_config(3, 2560, 2560, 2560) == 10    # 100 tiles
    assert native.mg_tuned_config(3, 8192, 8192, 8192) == 11
    native._load_default_tuning(native.lib())
    assert native.mg_tuned_config(3, 8192, 8192, 8192) == 7
    assert native.mg_tuned_config(5, 3072, 3072, 3072) == 7     # INT8, 144 tiles (sixteen waves)
    assert native.mg_tuned_config(5, 4096, 2048, 8192) == 6     # INT8, 128 tiles


def test_plan_without_workspace_is_chosen_for_an_unsplit_k_loop(rule):
    native = rule
    """mg_sgemm passes no workspace.  Its tile must be the best one for an
    unsplit K loop, not the split plan's tile run unsplit: at 6144^3 the split
    plan takes 256 x 256 tiles in four K ranges, while unsplit 128 x 128
    tiles fill the compute units' rounds better (the round plan's model puts
    256 x 256 unsplit at about 4.5 ms against 3.6 ms)."""
    n = 6144
    full = native.mg_gemm_workspace_size(0, "N", "N", n, n, n)
    assert full > 0
    assert native.mg_gemm_plan(0, n, n, n, full) == (0, 17, 4, 0)
    st, cfg, splits, packed = native.mg_gemm_plan(0, n, n, n, 0)
    assert (st, splits, packed) == (0, 1, 0)
    assert cfg == 18   # the 128 x 128 tile, run as eight waves with two staging sets
    # one byte short of the split's partials: planned as if no split existed
    assert native.mg_gemm_plan(0, n, n, n, full - 1) == (0, cfg, 1, 0)


SHAPES = [(1024, 1024, 1024), (2048, 2048, 2048), (1536, 1536, 1536), (3072, 3072, 3072), (8192, 8192, 256),
          (256, 8192, 8192), (16384, 1024, 4096), (64, 96, 2048), (512, 512, 8192), (8192, 8192, 8192)]


@pytest.mark.parametrize("path", [0, 1, 2, 4])
@pytest.mark.parametrize("M,N,K", SHAPES)
def test_plan_matches_queries_and_never_splits_without_room(native, path, M, N, K):
    full = native.mg_gemm_workspace_size(path, "N", "N", M, N, K)
    st, cfg, splits, packed = native.mg_gemm_plan(path, M, N, K, full)
    assert st == 0
    assert cfg == native.mg_tuned_config(path, M, N, K)
    assert splits == native.mg_split_count(path, M, N, K)
    st, cfg0, s0, p0 = native.mg_gemm_plan(path, M, N, K, 0)
    assert st == 0 and s0 == 1 and p0 == 0
    if splits == 1 and not packed:
        assert full == 0 and cfg0 == cfg


def test_plan_argument_errors(native):
    assert native.mg_gemm_plan(7, 8, 8, 8, 0)[0] == -101
    assert native.mg_gemm_plan(0, -1, 8, 8, 0)[0] == -2
    assert native.mg_gemm_plan(0, 8, -1, 8, 0)[0] == -3
    assert native.mg_gemm_plan(0, 8, 8, -1, 0)[0] == -4
    assert native.mg_gemm_plan(0, 2 ** 40, 8, 8, 0)[0] == -102
    # FP8 needs its packing workspace
    need = native.mg_gemm_workspace_size(3, "N", "N", 512, 512, 512)
    assert native.mg_gemm_plan(3, 512, 512, 512, need)[0] == 0
    assert native.mg_gemm_plan(3, 512, 512, 512, need - 1)[0] == -100


def test_exact_entries_precede_buckets_and_carry_splits(native, tmp_path):
    """An exact-shape line steers that shape only, ahead of the bucket line of
    its bucket; its K-range count becomes the plan's; a forced configuration
    still wins; without room for the partials a split entry is skipped."""
    p = tmp_path / "t.txt"
    # 1536^3 and 2048^3 share bucket 11
    p.write_text("0 11 11 11 3\n0 1536 1536 1536 0 x 3\n1 2048 2048 2048 2 x\n")
    assert native.mg_load_tuning(str(p)) == 0
    assert native.mg_tuned_config(0, 1536, 1536, 1536) == 0
    assert native.mg_tuned_config(0, 2048, 2048, 2048) == 3          # the bucket entry
    assert native.mg_split_count(0, 1536, 1536, 1536) == 3
    full = native.mg_gemm_workspace_size(0, "N", "N", 1536, 1536, 1536)
    assert native.mg_gemm_plan(0, 1536, 1536, 1536, full) == (0, 0, 3, 0)
    st, cfg, splits, _ = native.mg_gemm_plan(0, 1536, 1536, 1536, 0)
    assert st == 0 and splits == 1 and cfg == 3                       # falls back to the bucket entry
    # no split count given: the automatic split rule for that configuration
    assert native.mg_tuned_config(1, 2048, 2048, 2048) == 2
    assert native.mg_force_config(0, 5) == 0
    try:
        assert native.mg_tuned_config(0, 1536, 1536, 1536) == 5
    finally:
        native.mg_force_config(0, -1)
    # clearing the table drops exact entries too
    native.mg_load_tuning(None)
    assert native.mg_tuned_config(0, 1536, 1536, 1536) != 0 or native.mg_split_count(0, 1536, 1536, 1536) != 3


@pytest.mark.parametrize("text", ["0 0 8 8 3 x\n", "0 8 8 8 3 x 17\n", "0 8 8 8 3 x 0\n", "0 8 8 8 3 x z\n",
                                  "0 8 8 8 99 x 2\n", "0 3000000000 8 8 3 x 1\n", "9 8 8 8 3 x 1\n"])
def test_malformed_exact_entries_rejected(native, tmp_path, text):
    good = tmp_path / "good.txt"
    good.write_text("0 100 100 100 3 x 1\n")
    assert native.mg_load_tuning(str(good)) == 0
    bad = tmp_path / "bad.txt"
    bad.write_text(text)
    assert native.mg_load_tuning(str(bad)) == -103
    assert native.mg_tuned_config(0, 100, 100, 100) == 3


def test_committed_table_parses_and_its_exact_entries_are_admissible(native):
    """Every exact line of the committed table loads, names a configuration
    the blocking model admits for its shape, and a K-range count the library
    can cut K into."""
    from paper_2305_18236_amd import blocking
    path = os.path.join(os.path.dirname(autotune.__file__), "tuning_table.txt")
    assert native.mg_load_tuning(path) == 0
    for line in open(path):
        f = line.split()
        if line.startswith("#") or len(f) < 6 or f[5] != "x":
            continue
        pid, M, N, K, cfg = (int(v) for v in f[:5])
        splits = int(f[6]) if len(f) > 6 else -1
        cfgs = {c.id: c for c in blocking.library_configs(native, pid)}
        assert not blocking.feasible(cfgs[cfg]), line
        assert native.mg_tuned_config(pid, M, N, K) == cfg, line
        if splits > 1:
            assert blocking.effective_splits(K, splits) == splits, line


def test_committed_table_drives_the_tuned_shapes(native):
    """The committed exact entries are what single GEMMs of those shapes run,
    and for some of them that differs from the built-in rule (measured
    faster): e.g. BF16 at 1024^3 runs 64 x 64 tiles unsplit, where the rule
    would take 128 x 128 tiles in four K ranges."""
    path = os.path.join(os.path.dirname(autotune.__file__), "tuning_table.txt")
    entries = []
    for line in open(path):
        f = line.split()
        if not line.startswith("#") and len(f) >= 7 and f[5] == "x":
            entries.append(tuple(int(v) for v in f[:5]) + (int(f[6]),))
    assert len(entries) >= 90
    differ = 0
    for pid, M, N, K, cfg, splits in entries:
        full = native.mg_gemm_workspace_size(pid, "N", "N", M, N, K) if pid != 5 else 0
        if pid != 5:
            st, c, s, _ = native.mg_gemm_plan(pid, M, N, K, full)
            assert (st, c, s) == (0, cfg, splits), (pid, M, N, K)
    native.mg_load_tuning(None)
    for pid, M, N, K, cfg, splits in entries:
        if pid == 5:
            continue
        full = native.mg_gemm_workspace_size(pid, "N", "N", M, N, K)
        st, c, s, _ = native.mg_gemm_plan(pid, M, N, K, full)
        differ += (c, s) != (cfg, splits)
    assert differ >= 5
    assert (2, 1024, 1024, 1024, 4, 1) in entries
