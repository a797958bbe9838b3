// C-ABI host layer of mgemm: argument validation, BLAS quick returns,
// configuration choice (the blocking decision of Section 3.1) and launch on
// the caller's stream.  Every check here runs on the host before any device
// call, so invalid arguments never reach a kernel.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/mgemm.h"
#include "kernels.h"

namespace {

bool is_n(char t) { return t == 'N' || t == 'n'; }
bool is_t(char t) { return t == 'T' || t == 't' || t == 'C' || t == 'c'; }

// Configuration tables: the five mg_path values and MG_CONFIGS_I8.
constexpr int kPaths = 6;
std::atomic<int> g_forced[kPaths] = {{-1}, {-1}, {-1}, {-1}, {-1}, {-1}};
std::atomic<int> g_forced_splits[kPaths] = {{-1}, {-1}, {-1}, {-1}, {-1}, {-1}};
// Forced tile order: -1 automatic, else remap * 256 + group_m.
std::atomic<int> g_forced_order[kPaths] = {{-1}, {-1}, {-1}, {-1}, {-1}, {-1}};

// The raster of the single-GEMM kernels (tile_of): group_m tile rows per
// group, and whether each XCD gets a contiguous range of it.
struct TileOrder {
    int group_m, remap;
};

TileOrder tile_order(int path)
{
    const int f = g_forced_order[path].load();
    if (f >= 0) return {f & 255, f >> 8};
    return {4, 1};
}

bool valid_path(int path) { return path >= 0 && path < kPaths; }

// Paths of mg_gemm (FP32 operands).
bool float_path(int path) { return path >= 0 && path <= MG_PATH_FP16; }

// Paths the 16-bit matrix-core kernels run, and their TERMS kind.
bool is_16bit(int path) { return path == MG_PATH_BF16X3 || path == MG_PATH_BF16 || path == MG_PATH_FP16; }
int kind_of(int path) { return path == MG_PATH_BF16X3 ? 3 : path == MG_PATH_FP16 ? 16 : 1; }

// Whether configuration `cfg` of `path`'s table runs on that path.
bool config_valid(int path, int cfg);

// Paths the persistent batched kernel runs.
bool batched_path(int path) { return float_path(path) && path != MG_PATH_FP8_T128; }

int hip_status(hipError_t e) { return e == hipSuccess ? MG_OK : MG_ERR_HIP - int(e); }

// rows * ld must stay addressable; both are non-negative here.
bool fits(int64_t rows, int64_t ld) { return rows == 0 || ld <= INT64_MAX / 4 / rows; }

// BLAS-style validation of the mg_sgemm argument list (any element type).
int validate(char transA, char transB, int64_t M, int64_t N, int64_t K, const void* A,
             int64_t lda, const void* B, int64_t ldb, const void* C, int64_t ldc)
{
    if (!is_n(transA) && !is_t(transA)) return -1;
    if (!is_n(transB) && !is_t(transB)) return -2;
    if (M < 0) return -3;
    if (N < 0) return -4;
    if (K < 0) return -5;
    const bool ta = is_t(transA), tb = is_t(transB);
    const int64_t a_rows = ta ? K : M, a_cols = ta ? M : K;
    const int64_t b_rows = tb ? N : K, b_cols = tb ? K : N;
    if (A == nullptr && M > 0 && K > 0) return -7;
    if (lda < (a_cols > 1 ? a_cols : 1) || !fits(a_rows, lda)) return -8;
    if (B == nullptr && K > 0 && N > 0) return -9;
    if (ldb < (b_cols > 1 ? b_cols : 1) || !fits(b_rows, ldb)) return -10;
    if (C == nullptr && M > 0 && N > 0) return -12;
    if (ldc < (N > 1 ? N : 1) || !fits(M, ldc)) return -13;
    if (M > INT_MAX || N > INT_MAX || K > INT_MAX) return MG_ERR_TOO_LARGE;
    return MG_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// 16-byte panel loads with 32-bit in-panel offsets (see GemmArgs::vec_a).
bool fast_operand(const void* p, int64_t ld) { return aligned16(p) && ld % 4 == 0 && ld < (int64_t(1) << 22) - 64; }

// A dimension no compute entry point accepts (they return MG_ERR_TOO_LARGE);
// the query functions answer for it without forming products that overflow.
bool beyond_int(int64_t a, int64_t b, int64_t c) { return a > INT_MAX || b > INT_MAX || c > INT_MAX; }

int64_t tiles(int64_t M, int64_t N, int bm, int bn) { return ((M + bm - 1) / bm) * ((N + bn - 1) / bn); }
int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct ConfigTable {
    const mg::SgemmConfig* cfgs;
    int n;
};

ConfigTable table_of(int path)
{
    switch (path) {
    case MG_PATH_FP32: return {mg::kSgemmConfigs, mg::kNumSgemmConfigs};
    case MG_PATH_BF16X3:
    case MG_PATH_BF16:
    case MG_PATH_FP16: return {mg::kBf16Configs, mg::kNumBf16Configs};
    case MG_PATH_FP8_T128: return {mg::kFp8Configs, mg::kNumFp8Configs};
    case MG_CONFIGS_I8: return {mg::kI8Configs, mg::kNumI8Configs};
    default: return {nullptr, 0};
    }
}

// ---- Tuning table: (mode, path, bucket(M), bucket(N), bucket(K)) ->
// configuration id, written by the autotuner.  mode 0 ('s') is read by single
// GEMMs, mode 1 ('b') by the batched kernel (which falls back to mode 0).
// bucket(x) = round(log2 x), clamped to [0, kBuckets).  -1: not tuned.
constexpr int kBuckets = 21;
int8_t g_table[2][kPaths][kBuckets][kBuckets][kBuckets];
std::once_flag g_table_init;
std::mutex g_table_mutex;

void table_clear()
{
    std::memset(g_table, -1, sizeof(g_table));
}

bool config_valid(int path, int cfg)
{
    return cfg >= 0 && cfg < table_of(path).n;
}

int bucket(int64_t x)
{
    if (x <= 1) return 0;
    int b = 63 - __builtin_clzll(uint64_t(x));   // 2^b <= x < 2^(b+1), b >= 1
    // round to the nearer power of two: x >= 1.5 * 2^b, written without
    // forming 2x (which overflows for x near INT64_MAX)
    if (x - (int64_t(1) << b) >= (int64_t(1) << (b - 1))) ++b;
    return b < kBuckets ? b : kBuckets - 1;
}

int table_lookup(int path, int64_t M, int64_t N, int64_t K, int mode = 0)
{
    std::call_once(g_table_init, table_clear);
    return g_table[mode][path][bucket(M)][bucket(N)][bucket(K)];
}

// Exact-shape entries ('x' lines of the table): the configuration and the
// number of K ranges the autotuner measured best for one (path, M, N, K).
// They take precedence over the log2 buckets, which cannot tell apart shapes
// such as 1536^3 and 2048^3 whose best plans differ.  Replaced as a whole by
// mg_load_tuning; read without locking (load the table before launching
// GEMMs from other threads).
struct ExactEntry {
    int path;
    int64_t M, N, K;
    int cfg;
    int splits;   // K ranges (1: no split); -1: the automatic rule's
};
std::vector<ExactEntry> g_exact;

const ExactEntry* exact_lookup(int path, int64_t M, int64_t N, int64_t K)
{
    for (const ExactEntry& e : g_exact)
        if (e.path == path && e.M == M && e.N == N && e.K == K) return &e;
    return nullptr;
}

int device_cus();

// ---- Split-K: when a GEMM has fewer output tiles than the GPU has compute
// units, the K loop is cut into ranges that separate workgroups multiply; the
// partial products go to the workspace and a reduction kernel sums them in a
// fixed order and applies alpha and beta.
constexpr int64_t kSplitGrain = 128;   // K range granularity (multiple of every BK)
constexpr int64_t kMinRange = 256;     // shortest K range the rule cuts
constexpr int kMaxSplits = 16;

// Split factor the automatic rule gives `t` output tiles: enough K ranges for
// one workgroup per compute unit, each at least kMinRange deep.
// The 16-bit paths' split rule: as many K ranges as fit one round of
// workgroups (rounded down, where the FP32 rule rounds up).  Their GEMMs run
// two to eight times faster than FP32, so a second, nearly empty round of
// split workgroups costs more than the idle compute units of an unsplit
// one: 144 tiles (3072^3) run unsplit, 128 tiles (4096 x 2048 x 8192) in two
// ranges.  Measured (us, rounded up -> down): BF16 3072^3 131.1 -> 101.8,
// 3072 x 3072 x 1024 75.6 -> 47.8; bf16x3 3072^3 249.3 -> 208.8, 1536 x
// 1536 x 4096 125.6 -> 86.2.
int splits_16bit(int64_t t, int64_t K, int64_t cus)
{
    if (t <= 0 || t >= cus) return 1;
    const int64_t s = std::min<int64_t>({cus / t, K / kMinRange, kMaxSplits});
    return s < 2 ? 1 : int(s);
}

// The ladder's fill test: enough K ranges for one workgroup per compute
// unit, rounded up.
int fill_splits(int64_t t, int64_t K)
{
    const int64_t cus = device_cus();
    if (t <= 0 || t >= cus) return 1;
    const int64_t s = std::min<int64_t>({(cus + t - 1) / t, K / kMinRange, kMaxSplits});
    return s < 2 ? 1 : int(s);
}

int auto_splits(int64_t t, int64_t K)
{
    const int64_t cus = device_cus();
    if (t <= 0 || t >= cus) return 1;   // no tiles (M or N is 0): nothing to split
    // Tiles that already keep 84 % of the compute units busy run whole up to
    // K = 3072: two K ranges would leave as many idle in each of two rounds
    // and add the reduction (us, two ranges -> one: 7936 x 2048 x 1536 on 248
    // tiles of 256 x 256 436.2 -> 392.3, 2816 x 5120 x 1536 on 220 431.7 ->
    // 392.4, 2688 x 5888 x 2048 559.6 -> 515.6, 2944 x 4608 x 3072 795.2 ->
    // 758.5; 768 x 4992 x 768 on 234 tiles of 128 x 128 71.8 -> 58.2).  With
    // longer K the reduction weighs less and the split stays (3200 x 4224 x
    // 8192: 2134.1 against 2209.0 whole).
    if (K <= 3072 && t * 100 >= 84 * cus) return 1;
    const int64_t s = std::min<int64_t>({(cus + t - 1) / t, K / kMinRange, kMaxSplits});
    return s < 2 ? 1 : int(s);
}

// Automatic configuration.  Measured on MI355X (FP32 and bf16x3 sweeps over
// 1024^3 .. 8192^3 and skinny shapes): the 256 x 256 tile is the most
// efficient whenever the tiles, times the split factor, give every compute
// unit a workgroup; otherwise the next smaller tile with its split.  For FP32
// with very short K (<= 256) the 128 x 64 tile is chosen instead: several
// per compute unit, so one workgroup's C0 reads and stores overlap another's
// matrix work (8192 x 8192 x 256, beta 0.5: 359 us against 373 us with
// 256 x 256 tiles and 398 us with 64 x 64).  The 16-bit paths keep the
// ladder there (bf16x3 at the same shape: 222 us with 256 x 256 tiles, 303 us
// with 64 x 64).
bool uses_planes(int path, int cfg, int64_t M, int64_t N, int64_t K);

// The tile ladder (see choose_config): the largest tile whose tiles, times
// the automatic split, give every compute unit a workgroup.
int ladder_choice(int path, int64_t M, int64_t N, int64_t K, int64_t cus, bool split_ok)
{
    // tile ids by decreasing size: 256 x 256, 128 x 128, 64 x 64
    static const int kFp32Ladder[3] = {5, 0, 3};
    static const int kBf16Ladder[3] = {1, 2, 4};
    const int* ladder = path == MG_PATH_FP32 ? kFp32Ladder : kBf16Ladder;
    const ConfigTable t = table_of(path);
    if (path == MG_PATH_FP32 && K <= 256 && tiles(M, N, 128, 64) >= cus) return 4;
    for (int i = 0; i < 3; ++i) {
        const mg::SgemmConfig& c = t.cfgs[ladder[i]];
        const int64_t n = tiles(M, N, c.bm, c.bn);
        if (path != MG_PATH_FP32) {
            // 16-bit paths: this tile if its workgroups keep half the
            // compute units busy (see splits_16bit).  On pre-packed planes:
            // the same 256 x 256 tiles with
            // panels copied straight into LDS (6), bit-identical to (1) and
            // faster (8192^3 end to end: BF16 1078-1080 against 975-997
            // TFLOP/s, FP16 1023-1030 against 941-948, bf16x3 430-433 against
            // 354-360).  Without the planes' workspace configuration 6 runs as
            // configuration 1.  bf16x3's pack reads and writes 4 bytes per
            // element of both operands, which the faster GEMM repays only when
            // each operand is re-read often enough: op(A) by the N / 256 column
            // tiles, op(B) by the M / 256 row tiles, so 1/M + 1/N must be small.
            // Measured end to end (NN, TFLOP/s): wins at 3072^3 198 -> 242,
            // 4096 x 2048 x 8192 283 -> 347, 2048 x 8192 x 2048 342 -> 390,
            // 4096^3 360 -> 409; losses at 2048^3 235 -> 224, 2048 x 2048 x 8192
            // 327 -> 312, 1024 x 8192 x 4096 327 -> 305; ties at 16384 x 1024 x
            // 4096 and 8192 x 1024 x 8192.  1/M + 1/N <= 0.0008 separated them
            // then.  With the faster direct-copy kernels the bound moved:
            // M N >= 1050 (M + N) for bf16x3 (22 random shapes between the
            // two bounds, us, in-kernel split -> planes: 5504 x 1536 x 4096
            // 345.6 -> 253.9, 1536 x 5760 x 1024 102.4 -> 78.7, 2688 x 2176 x
            // 8192 396.6 -> 319.3; 4-36 % faster, 19 % in geometric mean).
            // At 900 (M + N) the earlier losses return (2048 x 2048 x 8192:
            // 212.8 against 202.5, 1024 x 8192 x 4096: 219.9 against 206.9).
            const int s16 = split_ok ? splits_16bit(n, K, cus) : 1;
            if (n * s16 * 2 < cus) continue;
            // BF16 and FP16: a tile that needs a K split into ranges of 384
            // or less (K up to 2048, M and N at least 512) gives way to the
            // 64 x 64 tile if that one alone gives each compute unit one or
            // two workgroups.  On 16 random shapes of that kind it was 9-52 %
            // faster (us, plan -> 4 unsplit: 2176 x 768 x 512 25.2 -> 16.1,
            // 2048 x 1024 x 1536 in six ranges 1.35x, 1280 x 1280 x 768
            // 1.25x).  Outside it the step lost: a side of 256 or 384 (the
            // 256 x 256 in-kernel tile split 7-12 ways ran 2-3x faster),
            // longer ranges (up to 9 % slower at 512 deep).  bf16x3's three
            // products per step keep the larger tiles ahead from K = 768
            // (512 x 2688 x 768: 24.7 us split against 31.0); up to K = 512
            // it steps down too (8 random shapes: 12 % faster in geometric
            // mean, 3328 x 512 x 512 25.2 -> 21.2).
            const int64_t n64 = tiles(M, N, 64, 64);
            if (i < 2 && s16 > 1 && n64 >= cus && n64 <= 2 * cus && std::min(M, N) >= 512 &&
                ((path == MG_PATH_BF16 || path == MG_PATH_FP16) ? K <= 2048 && K / s16 <= 384 : K <= 512))
                return ladder[2];
            // The 256 x 256 tile, when it needs a K split, gives way to the
            // 128 x 128 tile if that one fills the GPU unsplit: on pre-packed
            // planes as eight waves fed by direct copies (10), else in its
            // in-kernel form.  Measured (NN, beta 0.5, us, 256 x 256 split
            // -> 10 unsplit): BF16 4096 x 2048 x 2048 74.9 -> 55.6, 2560^3
            // 72.3 -> 56.6, 2048 x 2048 x 8192 119.9 -> 111.5; bf16x3 2048^3
            // 73.8 -> 67.3, 2048 x 2048 x 1024 51.4 -> 40.7, 4096 x 2048 x
            // 2048 122.8 -> 109.4, 2560^3 120.3 -> 115.3.  bf16x3 keeps the
            // split for K ranges of 2048 and more (2048 x 2048 x 8192: 213.4
            // against 237.5).  The 128 x 128 tile itself keeps its split
            // against the 64 x 64 one (bf16x3 1024^3: 25.0 us in four K
            // ranges, 32.0 us unsplit on 64 x 64 tiles).
            // Where the split's K ranges are 512 deep or less (BF16 and
            // FP16: 1024; 24 random shapes between the two bounds ran 1-31 %
            // faster, 13 % in geometric mean) it does so
            // once the 128 x 128 tiles keep three quarters of the compute
            // units busy (us, plan -> 10 unsplit: BF16 3712 x 896 x 1024 on
            // 203 tiles 40.8 -> 27.8, 768 x 4992 x 768 on 234 37.9 -> 25.0;
            // bf16x3 50.3 -> 41.1 and 48.0 -> 35.9; on 26 random shapes the
            // step gained 22-52 % with 256-deep ranges and lost up to 11 %
            // with ranges of 1536 and more).  And unsplit
            // 256 x 256 tiles that spill a second round under a quarter full
            // give way too (BF16 4480 x 3840 x 256, 270 tiles: 44.8 -> 38.0,
            // 6144 x 3328 x 8192, 312 tiles: 448.3 -> 413.6; bf16x3 67.3 ->
            // 50.9 and 1086.7 -> 956.5; 54 random shapes of both paths: 12 %
            // faster in geometric mean, none slower by over 3 %).  bf16x3
            // steps down up to a third full (26 random shapes with 320-341
            // tiles: 12 % faster in geometric mean, 2560 x 8192 x 512 101.8
            // -> 81.2, 4096 x 5120 x 4096 548.5 -> 462.8; none slower by over
            // 2 %).
            const int64_t n128 = tiles(M, N, t.cfgs[ladder[1]].bm, t.cfgs[ladder[1]].bn);
            if (i == 0 && s16 > 1 && (path != MG_PATH_BF16X3 || K / s16 < 2048) &&
                (n128 >= cus || (n128 * 4 >= cus * 3 && K / s16 <= (path == MG_PATH_BF16X3 ? 512 : 1024))))
                return uses_planes(path, 10, M, N, K) ? 10 : ladder[1];
            if (i == 0 && s16 == 1 && n > cus && n < 2 * cus && (n - cus) * (path == MG_PATH_BF16X3 ? 3 : 4) < cus)
                return uses_planes(path, 10, M, N, K) ? 10 : ladder[1];
            // BF16 and FP16 run that tile over sixteen 64 x 64 waves (11,
            // four per SIMD, bit-identical to 6): end to end, us, 6 -> 11:
            // BF16 8192^3 1030.1 -> 1008.0, 6144^3 540.1 -> 519.4, 4096^3
            // 142.3 -> 141.0; FP16 8192^3 1066.6 -> 1037.5.  bf16x3 keeps
            // eight (8192^3 2454 against 2482 with sixteen).
            if (ladder[i] == 1 && uses_planes(path, 6, M, N, K) &&
                (path != MG_PATH_BF16X3 || M * N >= 1050 * (M + N)))
                return path == MG_PATH_BF16X3 ? 6 : 11;
            return ladder[i];
        }
        const int s = split_ok ? fill_splits(n, K) : 1;
        if (n * s < cus) continue;
        // FP32: when this tile needs K ranges as short as kMinRange to fill
        // the GPU and the next smaller tile fills it unsplit, the smaller one
        // wins (1024^3, beta 0.5: 64 x 64 unsplit 31.6 us, 128 x 128 in four
        // 256-deep ranges plus the reduction 37.6 us).  bf16x3 keeps the split
        // there (25.0 us against 32.0 us).
        if (s > 1 && K / s <= kMinRange && i + 1 < 3) {
            const mg::SgemmConfig& d = t.cfgs[ladder[i + 1]];
            if (tiles(M, N, d.bm, d.bn) >= cus) return ladder[i + 1];
        }
        return ladder[i];
    }
    return ladder[2];
}

// ---- FP32 rounds of workgroups.  The ladder ignores how the workgroups
// fall into rounds over the compute units: 3072^3 in 256 x 256 tiles and two
// K ranges is 288 workgroups on 256 compute units, a second round nearly
// empty (784 us, against 510 us for 64 x 64 tiles unsplit).  Where the
// ladder's choice leaves its last round less than 80 % full, the plan below
// compares the 256 x 256, 128 x 128 and 64 x 64 tiles with 1-8 K ranges by
// a time model fitted to MI355X measurements (per compute unit: 0.55,
// 0.509, 0.483 TFLOP/s and 32, 9.5, 2 us of fixed cost per round of 1, 2, 5
// resident workgroups, half that for split workgroups, which do not read C;
// the reduction streams the partials and C at 5 TB/s, plus 5 us), and takes
// the best if it is 5 % faster.
// Shapes whose rounds come out whole (every power-of-two shape from 2048^3
// up) keep the ladder's choice.
struct Fp32Plan {
    int cfg;
    int splits;   // requested K ranges; -1: the automatic split
};

int64_t effective_splits(int64_t K, int64_t s)
{
    if (s < 2 || K < 2 * kSplitGrain) return 1;
    const int64_t chunk = round_up((K + s - 1) / s, kSplitGrain);
    return (K + chunk - 1) / chunk;
}

double fp32_model_us(int cfg, int64_t M, int64_t N, int64_t K, int64_t s, int64_t cus)
{
    const int bm = cfg == 5 ? 256 : cfg == 0 ? 128 : 64;
    const int64_t occ = cfg == 5 ? 1 : cfg == 0 ? 2 : 5;
    // the 128 x 128 figures are configuration 18's (it runs wherever the
    // plan picks that tile): 2048 x 2048 x 1024 75.3 us, 2048^3 141.3 us,
    // 1024 x 2048 x 1024 in two K ranges 47.9 us; the model gives 75.4,
    // 141.4 and 47.8
    const double rate = cfg == 5 ? 0.55 : cfg == 0 ? 0.509 : 0.483;   // TFLOP/s per compute unit
    const double fixed = cfg == 5 ? 32.0 : cfg == 0 ? 9.5 : 2.0;      // us per round
    const int64_t per_cu = (tiles(M, N, bm, bm) * s + cus - 1) / cus;
    const double wg_us = 2.0 * bm * bm * double((K + s - 1) / s) / (rate * 1e6);
    // a split's workgroups store partial products without reading C (half
    // the fixed cost); the reduction then streams s partials and C at 5 TB/s
    double t = double(per_cu) * wg_us + (s > 1 ? 0.5 : 1.0) * fixed * double((per_cu + occ - 1) / occ);
    if (s > 1) t += 4.0 * double(s + 1) * double(M) * double(N) / 5e6 + 5.0;
    return t;
}

Fp32Plan fp32_plan(int64_t M, int64_t N, int64_t K, int pick, bool split_ok)
{
    const Fp32Plan keep{pick, -1};
    if ((pick != 5 && pick != 0) || M <= 0 || N <= 0 || K <= 0 || beyond_int(M, N, K)) return keep;
    const int64_t cus = device_cus();
    const int bm = pick == 5 ? 256 : 128;
    const int64_t s0 = split_ok ? effective_splits(K, auto_splits(tiles(M, N, bm, bm), K)) : 1;
    const int64_t n = tiles(M, N, bm, bm) * s0;
    const int64_t rounds = (n + cus - 1) / cus;
    // Where the big tile would split K and the 64 x 64 tiles unsplit already
    // give every compute unit one or two workgroups, those win up to K = 4096
    // (two workgroups per unit with two K groups each, configuration 15; us,
    // NN, plan -> 64 x 64 unsplit): 1024 x 2048 x 1024 in two ranges of 128 x
    // 128 tiles 47.2 -> 43.6, 2048 x 1024 x 2048 in eight ranges of 256 x 256
    // 93.5 -> 79.0, 512 x 4096 x 2048 93.9 -> 78.6, 1024 x 1024 x 4096 in
    // sixteen 93.2 -> 85.0, 512 x 2048 x 2048 in four of 128 x 128 46.6 ->
    // 45.6; TT alike.  At K = 8192 the many short ranges of the big tile stay
    // faster (1024 x 2048 x 8192: 277.7 against 294.9).
    // (Both only where the smaller tiles' last round is at least 80 % full:
    // 3072 x 1664 x 3072, 312 tiles of 128 x 128, ran 407 us unsplit against
    // 322 us in two K ranges.)
    auto full = [&](int64_t t) { return t * 10 >= ((t + cus - 1) / cus) * cus * 8; };
    const int64_t t64 = tiles(M, N, 64, 64);
    if (s0 > 1 && K <= 4096 && t64 >= cus && t64 <= 2 * cus && full(t64)) return Fp32Plan{3, 1};
    // Likewise the 128 x 128 tile unsplit (as eight waves, configuration 18)
    // against the 256 x 256 tile's K ranges, while each compute unit's share
    // K * tiles / cus stays within 4096 x one tile (us, NN, 17 split ->
    // 18 unsplit): 4096 x 1024 x 2048 in four ranges 155.8 -> 140.0, 2048 x
    // 4096 x 1024 in two 160.7 -> 145.9, 2048 x 2048 x 4096 in four 278.5 ->
    // 272.2, 2048 x 4096 x 2048 in two 282.9 -> 277.8; beyond it the split
    // wins (2048 x 4096 x 4096: 527.1 against 541.1; 2048 x 2048 x 8192:
    // 523.9 against 534.5).
    const int64_t t128 = tiles(M, N, 128, 128);
    if (pick == 5 && s0 > 1 && t128 >= cus && t128 <= 2 * cus && full(t128) && K * t128 <= 4096 * cus)
        return Fp32Plan{0, 1};
    // The model decides unless the last round is at least 90 % full, and
    // weighs every plan that keeps at least 80 % of the compute units busy.
    // Against the earlier bounds (80 % full; every unit busy), measured on
    // 47 random shapes whose plan changed (NN, us): 5.7 % faster in
    // geometric mean, none slower by over 3 %; e.g. 2816 x 4736 x 1024
    // 316.9 -> 255.1, 7552 x 1664 x 8192 2119.7 -> 1599.2 (128 x 128 tiles
    // unsplit on 81 % of the units), 3200 x 4224 x 8192 2118.9 -> 1795.7.
    if (n * 10 >= rounds * cus * 9) return keep;   // last round at least 90 % full
    Fp32Plan best = keep;
    double best_t = 0.95 * fp32_model_us(pick, M, N, K, s0, cus);
    static const int kCfgs[3] = {5, 0, 3};
    static const int kSplits[6] = {1, 2, 3, 4, 6, 8};
    for (int c : kCfgs) {
        const int tb = c == 5 ? 256 : c == 0 ? 128 : 64;
        for (int req : kSplits) {
            if (req > 1 && !split_ok) break;
            const int64_t se = effective_splits(K, req);
            if (req > 1 && (se < 2 || K / se < kMinRange)) continue;
            if (tiles(M, N, tb, tb) * se * 10 < cus * 8) continue;   // 80 % of the units busy
            const double t = fp32_model_us(c, M, N, K, se, cus);
            if (t < best_t) {
                best = Fp32Plan{c, req};
                best_t = t;
            }
        }
    }
    return best;
}

// The 64 x 64 FP32 tile with two register staging sets (12) replaces the
// one-set form (3) wherever the rule picks that tile: measured (NN, beta
// 0.5, % of the FP32 peak) 1024^3 46.2 -> 50.9, 1536^3 in four K ranges
// 55.7 -> 56.4, 3072^3 71.2 -> 74.3.  When its workgroups (tiles times K
// ranges) give each compute unit at most one, the form with two K groups of
// waves (15) takes it instead, two waves per SIMD where the others have
// one: 1024^3 50.9 -> 54.3.  So it does at two workgroups per compute unit
// when each K range is at least 512 long (us, 12 -> 15: 1024 x 2048 x 1024
// 44.3 -> 43.6, 2048 x 1024 x 2048 82.0 -> 79.0, 640 x 3072 x 8192 307.9 ->
// 292.5, 640 x 1536 x 4096 in two ranges 84.9 -> 81.8; at 512 they tie);
// shorter ranges leave each K group too few panels (1536 x 768 x 128 9.9 ->
// 10.5, 512 x 2560 x 256 15.0 -> 15.3).  At 3072^3, several workgroups per
// compute unit, the two tie.
// Likewise the 256 x 256 tile runs as its two-staging-set form (17):
// measured against configuration 5 (% of the FP32 peak, same box, three
// shuffled rounds): 8192^3 85.8 -> 88.2, 4096^3 84.5 -> 86.5,
// 16384 x 1024 x 4096 84.2 -> 86.4, 6144^3 in four K ranges 79.8 -> 81.9.
// And the 128 x 128 tile runs as eight 64 x 32 waves with two staging sets
// (18), faster than the four-wave configuration 0 at every shape measured
// with the same K ranges (NN, beta 0.5, us): 1024 x 4096 x 1024 94.7 ->
// 75.4, 512 x 2048 x 2048 in four ranges 53.9 -> 46.3, 3072 x 4096 x 4096
// 869 -> 821, 1792 x 1536 x 4096 in three ranges 211.5 -> 203.6.
// The 128 x 64 tile of short K loops runs over eight 32 x 32 waves with two
// staging sets (20), in every layout faster than configuration 4 (% of the
// FP32 peak, NN / NT / TN / TT): 8192 x 8192 x 256 62.1 / 62.4 / 61.3 / 61.4
// -> 64.3 / 64.4 / 63.0 / 63.4, 8192 x 8192 x 512 69.1 / 69.1 / 69.1 / 68.7
// -> 72.3 / 72.7 / 71.0 / 72.1, 4096 x 4096 x 256 59.5 / 59.1 / 59.6 /
// 59.4 -> 62.5 / 62.8 / 61.6 / 62.1.
int fp32_small_tile(int cfg, int64_t M, int64_t N, int64_t K, int splits, bool split_ok)
{
    if (cfg == 5) return 17;
    if (cfg == 0) return 18;
    if (cfg == 4) return 20;
    if (cfg != 3) return cfg;
    const int64_t cus = device_cus();
    const int64_t t = tiles(M, N, 64, 64);
    const int64_t s = splits > 0 ? effective_splits(K, splits) : (split_ok ? effective_splits(K, auto_splits(t, K)) : 1);
    return t * s <= cus || (t * s <= 2 * cus && (K + s - 1) / s >= 512) ? 15 : 12;
}

int choose_config(int path, int64_t M, int64_t N, int64_t K, bool split_ok)
{
    const int64_t cus = device_cus();
    if (path == MG_PATH_FP8_T128) {
        // 256 x 256: panels copied straight into LDS (7): 2359-2418 TFLOP/s
        // at 8192^3 against 2200-2378 for the interleaved pack (5) and 1970
        // for the plain loop (4); 128 x 128: the interleaved pack (6) beats
        // the direct copy (8), 1904-1954 vs 1764-1839.  The big tile wins as
        // soon as its tiles keep more than half the compute units busy
        // (3072^3, 144 tiles: 45.7 us against 48.8 us; 2560^3, 100 tiles:
        // 128 x 128 is best, 28.5 us).  The 128 x 128 tile runs as eight
        // 64 x 32 waves fed by direct copies (10), bit-identical to 8 and
        // faster than the interleaved pack (GEMM only, us, 6 -> 10: 2048^3
        // 17.7 -> 14.8, 2560^3 27.1 -> 25.0, 4096 x 2048 x 2048 24.6 -> 22.3,
        // 1536^3 14.1 -> 11.4).
        // 256 x 256 tiles that spill a second round under a quarter full
        // give way to the 128 x 128 tile (us, 7 -> 10: 4480 x 3840 x 256 on
        // 270 tiles 46.5 -> 36.4, 4352 x 4096 x 2048 on 272 94.4 -> 77.3,
        // 4608 x 4096 x 4096 on 288 148.5 -> 126.2, 6144 x 3328 x 8192 on
        // 312 292.0 -> 274.3).
        // The 256 x 256 tile runs over sixteen 64 x 64 waves (11): on 22
        // shapes off the tuned table with 100-1024 tiles it was ahead of the
        // eight-wave form in 21, by up to 6.8 %, and 0.7 % behind in one
        // (GEMM only, us, 7 -> 11: 8192 x 8192 x 2048 252.5 -> 236.3, 6144
        // x 7168 x 2048 168.5 -> 163.0, 7168 x 7168 x 4096 331.2 -> 320.0,
        // 2816 x 3584 x 2048 51.7 -> 49.2).  The tuned table keeps 7 where
        // it measured that ahead (4096^3, 8192^3).
        // Up to a third full, as bf16x3: 12 random shapes with 320-341
        // tiles all ran faster on the 128 x 128 tile (0-15 %, 6 % in
        // geometric mean; INT8 lost up to 10 % there and keeps a quarter).
        const int64_t n256 = tiles(M, N, 256, 256);
        if (n256 > cus && n256 < 2 * cus && (n256 - cus) * 3 < cus) return 10;
        if (n256 * 2 > cus) return 11;
        if (tiles(M, N, 128, 128) >= 128) return 10;
        return 3;
    }
    if (path == MG_CONFIGS_I8) {
        // 256 x 256: panels copied straight into LDS (5): 2255 TOP/s at
        // 8192^3 against 2128-2190 for the interleaved pack (3) and 1870 for
        // the plain loop (0); 128 x 128: the interleaved pack (4).  As for
        // FP8, the big tile from more than half the compute units' worth of
        // tiles on (3072^3, 144 tiles: 47.5 us against 54.1 us; 4096 x 2048 x
        // 8192, 128 tiles: 81.2 us for 128 x 128 against 100.6 us).  The
        // 128 x 128 tile runs as eight 64 x 32 waves fed by direct copies
        // (6): GEMM only, us, 4 -> 6: 2048^3 16.9 -> 14.6, 2560^3 27.3 ->
        // 22.9, 4096 x 2048 x 2048 25.5 -> 22.4
        // The 256 x 256 tile runs over sixteen 64 x 64 waves (7): GEMM only,
        // us, 5 -> 7: 8192^3 479.6 -> 473.0, 6144^3 245.9 -> 236.2, 4096^3
        // 66.6 -> 65.8.
        // The same step down as FP8 (us, 7 -> 6: 4480 x 3840 x 256 34.0 ->
        // 25.3, 4352 x 4096 x 2048 77.2 -> 69.7, 4608 x 4096 x 4096 122.6 ->
        // 109.4, 6144 x 3328 x 8192 222.2 -> 205.9).
        const int64_t n256 = tiles(M, N, 256, 256);
        if (n256 > cus && n256 < 2 * cus && (n256 - cus) * 4 < cus) return 6;
        if (n256 * 2 > cus) return 7;
        if (tiles(M, N, 128, 128) >= 128) return 6;
        return 2;
    }
    // Tiny FP32 products: no packing (the Tiling strategy) is fastest, as the
    // paper finds for small matrices (measured: 0.84x the packed time at 16^3,
    // 0.95x at 32^3, even at 64^3, packing ahead from 128^3 on).
    if (path == MG_PATH_FP32 && std::max({M, N, K}) <= 32) return 8;
    const int pick = ladder_choice(path, M, N, K, cus, split_ok);
    // BF16 and FP16 (one product per step) run the 128 x 128 tile as eight
    // 32 x 64 waves (9): two waves per SIMD where configuration 2 has one,
    // 4-10 % faster at every shape measured (us, configuration 2 -> 9, the
    // same K ranges: 1024^3 26.3 -> 22.6, 2048^3 43.0 -> 39.9, 2048 x 2048 x
    // 1024 30.1 -> 26.9, 2048 x 2048 x 8192 125.9 -> 113.1).  bf16x3's three
    // products per step keep four waves busy (2048^3 in two K ranges: 70.1
    // us against 77.2-78.4 with eight).
    if (pick == 2 && (path == MG_PATH_BF16 || path == MG_PATH_FP16)) return 9;
    if (path != MG_PATH_FP32) return pick;
    const Fp32Plan fp = fp32_plan(M, N, K, pick, split_ok);
    return fp32_small_tile(fp.cfg, M, N, K, fp.splits, split_ok);
}

int pick_config(int path, int64_t M, int64_t N, int64_t K, bool split_ok = true);

// ---- FP8 packed layout: q is Rp x Kp bytes, scales (Rp/128) x (Kp/128) bytes.
// The GEMM kernels address a 256-row panel of q with 32-bit byte offsets, so
// K is limited to 2^23 (256 rows x 2^23 bytes = 2^31).
constexpr int64_t kMaxFp8K = int64_t(1) << 23;
int64_t fp8_rows(int64_t R) { return round_up(R > 0 ? R : 1, 256); }
int64_t fp8_kp(int64_t K) { return round_up(K > 0 ? K : 1, 128); }
size_t fp8_q_bytes(int64_t R, int64_t K) { return size_t(fp8_rows(R)) * size_t(fp8_kp(K)); }
size_t fp8_s_bytes(int64_t R, int64_t K) { return size_t(fp8_rows(R) / 128) * size_t(fp8_kp(K) / 128); }
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Fp8Workspace {
    size_t qa, qb, sa, sb, total;
};

Fp8Workspace fp8_workspace(int64_t M, int64_t N, int64_t K)
{
    Fp8Workspace w{};
    w.qa = 0;
    w.qb = w.qa + align256(fp8_q_bytes(M, K));
    w.sa = w.qb + align256(fp8_q_bytes(N, K));
    w.sb = w.sa + align256(fp8_s_bytes(M, K));
    w.total = w.sb + align256(fp8_s_bytes(N, K));
    return w;
}

// ---- BF16 paths, pre-packed form: hi (and lo) planes of op(A) and op(B)^T,
// rows padded to 256, K padded to 128, bf16.  Used where converting each
// operand once beats converting it in every workgroup that reads it, as
// measured at 8192^3 on MI355X: plain BF16 (687 vs 482 TFLOP/s: the packed
// operands also halve the GEMM's global traffic) for min(M, N) >= 512.  On
// bf16x3 the packed operands are as large as the FP32 ones and the in-kernel
// conversion hides behind the matrix core (about 370 vs 347 TFLOP/s), so
// bf16x3 converts in the kernel.
// The packed-operand kernels address a 256-row panel with 32-bit byte
// offsets (row * row stride), so the pre-packed planes are used only while
// 256 rows of up to 4 bytes per k (bf16x3's interleaved terms) stay within
// 2^31 bytes; longer K converts in the kernel, whose loads fall back to
// 64-bit addressing.
constexpr int64_t kMaxPrepackK = int64_t(1) << 21;

bool bf16_prepack_pays(int path, int64_t M, int64_t N, int64_t K)
{
    return (path == MG_PATH_BF16 || path == MG_PATH_FP16) && M >= 512 && N >= 512 && K >= 32 && K <= kMaxPrepackK;
}

// Whether configuration `cfg` of a 16-bit path multiplies pre-packed planes.
// bf16x3 packs only for its direct forms (6, 7, 10), into interleaved planes: with
// the in-kernel conversion its packed operands would be as large as the
// FP32 ones for no gain (about 347 against 370 TFLOP/s at 8192^3).
bool uses_planes(int path, int cfg, int64_t M, int64_t N, int64_t K)
{
    if (path == MG_PATH_BF16X3)
        return (cfg == 6 || cfg == 7 || cfg == 10 || cfg == 11) && M >= 512 && N >= 512 && K >= 32 &&
               K <= kMaxPrepackK;
    return bf16_prepack_pays(path, M, N, K);
}

struct Bf16Workspace {
    int64_t Mp, Np, Kp;
    size_t a_hi, a_lo, b_hi, b_lo, total;
};

Bf16Workspace bf16_workspace(int path, int64_t M, int64_t N, int64_t K)
{
    Bf16Workspace w{};
    const int nl = path == MG_PATH_BF16X3 ? 2 : 1;
    w.Mp = round_up(M, 256);
    w.Np = round_up(N, 256);
    w.Kp = round_up(K, 128);
    const size_t pa = align256(size_t(w.Mp) * size_t(w.Kp) * 2), pb = align256(size_t(w.Np) * size_t(w.Kp) * 2);
    w.a_hi = 0;
    w.a_lo = pa;                       // used only when nl == 2
    w.b_hi = size_t(nl) * pa;
    w.b_lo = w.b_hi + pb;
    w.total = size_t(nl) * (pa + pb);
    return w;
}

struct SplitPlan {
    int splits;          // 1: no split
    int64_t chunk, ldp, stride;
    size_t bytes;
};

SplitPlan split_plan(int path, int cfg, int64_t M, int64_t N, int64_t K, bool split_ok = true)
{
    SplitPlan p{1, 0, 0, 0, 0};
    if (!split_ok || path == MG_PATH_FP8_T128 || path == MG_CONFIGS_I8 || M <= 0 || N <= 0 || K < 2 * kSplitGrain)
        return p;
    const mg::SgemmConfig& c = table_of(path).cfgs[cfg];
    int s = g_forced_splits[path].load();
    if (s < 0) {
        // the K ranges tuned with this configuration for this exact shape
        const ExactEntry* e = exact_lookup(path, M, N, K);
        if (e != nullptr && e->cfg == cfg && e->splits > 0) s = e->splits;
    }
    if (s < 0 && path == MG_PATH_FP32) {
        // the K ranges the round plan chose with this configuration
        const Fp32Plan fp = fp32_plan(M, N, K, ladder_choice(path, M, N, K, device_cus(), true), true);
        if (fp.cfg == cfg || (fp.cfg == 3 && (cfg == 12 || cfg == 15)) || (fp.cfg == 5 && cfg == 17) ||
            (fp.cfg == 0 && cfg == 18) || (fp.cfg == 4 && cfg == 20))
            s = fp.splits;
    }
    if (s < 0) s = path == MG_PATH_FP32 ? auto_splits(tiles(M, N, c.bm, c.bn), K)
                                        : splits_16bit(tiles(M, N, c.bm, c.bn), K, device_cus());
    if (s < 2) return p;
    p.chunk = round_up((K + s - 1) / s, kSplitGrain);
    p.splits = int((K + p.chunk - 1) / p.chunk);
    if (p.splits < 2) return SplitPlan{1, 0, 0, 0, 0};
    p.ldp = round_up(N, 4);
    p.stride = M * p.ldp;
    p.bytes = align256(size_t(p.splits) * size_t(p.stride) * sizeof(float));
    return p;
}

// ---- INT8 packed layout: Rp x Kp int8 rows (Rp = roundup(R, 256), Kp =
// roundup(K, 128)); the longest K whose sums stay inside int32.
constexpr int64_t kMaxI8K = 131071;

struct I8Workspace {
    size_t qa, qb, total;
};

I8Workspace i8_workspace(int64_t M, int64_t N, int64_t K)
{
    I8Workspace w{};
    w.qa = 0;
    w.qb = align256(fp8_q_bytes(M, K));
    w.total = w.qb + align256(fp8_q_bytes(N, K));
    return w;
}

int run_i8_pack(bool trans, int64_t R, int64_t K, const int8_t* X, int64_t ldx, int8_t* q, hipStream_t stream)
{
    const bool vec = aligned16(X) && ldx % 16 == 0;
    return hip_status(mg::launch_i8_pack(trans, X, ldx, R, K, vec, q, fp8_kp(K), fp8_rows(R), fp8_kp(K), stream));
}

int run_i8_packed(int64_t M, int64_t N, int64_t K, int32_t alpha, const int8_t* qA, const int8_t* qB, int32_t beta,
                  int32_t* C, int64_t ldc, hipStream_t stream)
{
    const int cfg = pick_config(MG_CONFIGS_I8, M, N, K);
    mg::I8Args g{};
    g.qA = qA; g.qB = qB; g.C = C;
    g.M = M; g.N = N; g.Kp = fp8_kp(K);
    g.ldq = g.Kp; g.ldc = ldc;
    g.alpha = alpha; g.beta = beta;
    const TileOrder o = tile_order(MG_CONFIGS_I8);
    g.group_m = o.group_m;
    g.remap = o.remap;
    return hip_status(mg::launch_gemm_i8(cfg, g, stream));
}

int run_fp8_packed(int64_t M, int64_t N, int64_t K, float alpha, const uint8_t* qA, const uint8_t* sA,
                   const uint8_t* qB, const uint8_t* sB, float beta, float* C, int64_t ldc,
                   hipStream_t stream)
{
    const int cfg = pick_config(MG_PATH_FP8_T128, M, N, K);
    mg::Fp8Args g{};
    g.qA = qA; g.qB = qB; g.sA = sA; g.sB = sB; g.C = C;
    g.M = M; g.N = N; g.Kp = fp8_kp(K);
    g.ldq = g.Kp; g.lds = g.Kp / 128; g.ldc = ldc;
    g.alpha = alpha; g.beta = beta;
    const TileOrder o = tile_order(MG_PATH_FP8_T128);
    g.group_m = o.group_m;
    g.remap = o.remap;
    return hip_status(mg::launch_gemm_fp8(cfg, g, stream));
}

int run_fp8_pack(bool trans, int64_t R, int64_t K, const float* X, int64_t ldx, uint8_t* q,
                 uint8_t* sc, hipStream_t stream)
{
    const int64_t Rp = fp8_rows(R), Kp = fp8_kp(K);
    const bool vec = aligned16(X) && ldx % 4 == 0;
    return hip_status(mg::launch_fp8_pack(trans, X, ldx, R, K, vec, q, Kp, sc, Kp / 128, Rp, Kp, stream));
}

// forced > tuned for this exact shape > tuned for its bucket > default
// rule.  split_ok: whether a K split may be planned (false when the caller's
// workspace cannot hold the partial products); an exact entry tuned with a
// split does not apply then, since its tile was chosen for split K loops.
int pick_config(int path, int64_t M, int64_t N, int64_t K, bool split_ok)
{
    int cfg = g_forced[path].load();
    if (cfg >= 0) return cfg;
    std::call_once(g_table_init, table_clear);
    const ExactEntry* e = exact_lookup(path, M, N, K);
    if (e != nullptr && (split_ok || e->splits <= 1)) return e->cfg;
    cfg = table_lookup(path, M, N, K);
    if (config_valid(path, cfg)) return cfg;
    return choose_config(path, M, N, K, split_ok);
}

// What mg_gemm runs on a non-FP8 path for a workspace of `avail` usable
// bytes: the best plan when the workspace holds everything it needs (the
// pre-packed 16-bit planes and the split-K partials); otherwise the plan
// made as if no split were possible (a configuration chosen for an unsplit
// K loop), with the planes when they still fit.
struct GemmPlan {
    int cfg;
    SplitPlan split;
    size_t planes;   // bytes of pre-packed planes at the start of the workspace (0: none)
};

GemmPlan plan_gemm(int path, int64_t M, int64_t N, int64_t K, size_t avail)
{
    auto planes_of = [&](int cfg) -> size_t {
        return is_16bit(path) && uses_planes(path, cfg, M, N, K) ? align256(bf16_workspace(path, M, N, K).total) : 0;
    };
    GemmPlan p{pick_config(path, M, N, K, true), {}, 0};
    p.split = split_plan(path, p.cfg, M, N, K, true);
    const size_t planes = planes_of(p.cfg);
    if (avail >= planes + p.split.bytes) {
        p.planes = planes;
        return p;
    }
    p.cfg = pick_config(path, M, N, K, false);
    p.split = split_plan(path, p.cfg, M, N, K, false);
    const size_t planes_b = planes_of(p.cfg);
    p.planes = avail >= planes_b ? planes_b : 0;
    return p;
}

// split_ws: workspace for the partial products of a split-K plan (nullptr:
// no split).  bf16_planes: workspace for pre-packed BF16 operands.
int run_gemm(int path, bool ta, bool tb, int64_t M, int64_t N, int64_t K, float alpha,
             const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
             int64_t ldc, hipStream_t stream, int cfg, const SplitPlan& plan, void* split_ws,
             void* bf16_planes)
{
    const ConfigTable t = table_of(path);
    const mg::SgemmConfig& c = t.cfgs[cfg];
    if (tiles(M, N, c.bm, c.bn) > INT_MAX) return MG_ERR_TOO_LARGE;
    mg::GemmArgs g{};
    g.A = A; g.B = B; g.C = C;
    g.M = M; g.N = N; g.K = K;
    g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.alpha = alpha; g.beta = beta;
    const TileOrder o = tile_order(path);
    g.group_m = o.group_m;
    g.remap = o.remap;
    g.vec_a = fast_operand(A, lda);
    g.vec_b = fast_operand(B, ldb);
    g.vec_c = aligned16(C) && ldc % 4 == 0;
    const bool split = split_ws != nullptr && plan.splits > 1;
    if (split) {
        g.part = static_cast<float*>(split_ws);
        g.k_chunk = plan.chunk;
        g.ldp = plan.ldp;
        g.part_stride = plan.stride;
    }
    auto finish = [&](hipError_t e) {
        if (e != hipSuccess || !split) return hip_status(e);
        return hip_status(mg::launch_splitk_reduce(g, plan.splits, C, ldc, stream));
    };
    switch (path) {
    case MG_PATH_FP32: return finish(mg::launch_sgemm(cfg, ta, tb, g, stream));
    case MG_PATH_BF16X3:
    case MG_PATH_BF16:
    case MG_PATH_FP16: {
        const int terms = kind_of(path);
        if (bf16_planes == nullptr) return finish(mg::launch_gemm_bf16(terms, cfg, ta, tb, g, stream));
        // pack each operand once, then multiply the packed planes
        const Bf16Workspace w = bf16_workspace(path, M, N, K);
        uint8_t* base = static_cast<uint8_t*>(bf16_planes);
        uint16_t* ahi = reinterpret_cast<uint16_t*>(base + w.a_hi);
        uint16_t* alo = reinterpret_cast<uint16_t*>(base + w.a_lo);
        uint16_t* bhi = reinterpret_cast<uint16_t*>(base + w.b_hi);
        uint16_t* blo = reinterpret_cast<uint16_t*>(base + w.b_lo);
        if (terms == 3) {
            // interleaved planes (configuration 6): A at a_hi, B at b_hi,
            // 2 Kp elements per row, both terms in one plane
            hipError_t e = mg::launch_bf16_pack_interleaved(ta, A, lda, M, K, fast_operand(A, lda), ahi, 2 * w.Kp,
                                                            w.Mp, w.Kp, stream);
            if (e != hipSuccess) return hip_status(e);
            e = mg::launch_bf16_pack_interleaved(!tb, B, ldb, N, K, fast_operand(B, ldb), bhi, 2 * w.Kp, w.Np, w.Kp,
                                                 stream);
            if (e != hipSuccess) return hip_status(e);
            g.A = reinterpret_cast<const float*>(ahi);
            g.B = reinterpret_cast<const float*>(bhi);
            g.lda = g.ldb = 2 * w.Kp;
            return finish(mg::launch_gemm_bf16(terms, cfg, false, true, g, stream, true));
        }
        hipError_t e = mg::launch_bf16_pack(ta, terms, A, lda, M, K, fast_operand(A, lda), ahi, alo, w.Kp,
                                            w.Mp, w.Kp, stream);
        if (e != hipSuccess) return hip_status(e);
        // op(B)^T is N x K: stored as is when transB is 'T', transposed when 'N'
        e = mg::launch_bf16_pack(!tb, terms, B, ldb, N, K, fast_operand(B, ldb), bhi, blo, w.Kp, w.Np, w.Kp,
                                 stream);
        if (e != hipSuccess) return hip_status(e);
        g.A = reinterpret_cast<const float*>(ahi);
        g.B = reinterpret_cast<const float*>(bhi);
        g.lda = g.ldb = w.Kp;
        g.plane_a = int64_t(w.a_lo - w.a_hi) / 2;
        g.plane_b = int64_t(w.b_lo - w.b_hi) / 2;
        return finish(mg::launch_gemm_bf16(terms, cfg, false, true, g, stream, true));
    }
    default: return MG_ERR_UNSUPPORTED;
    }
}

// ---- Batched: the tile variant of one problem (index into the batched set).
const int* batched_cfgs(int path)
{
    return path == MG_PATH_FP32 ? mg::kSgemmBatchedCfg : mg::kBf16BatchedCfg;
}

int batched_count(int path)
{
    return path == MG_PATH_FP32 ? mg::kSgemmBatchedVariants : mg::kBf16BatchedVariants;
}

int choose_batched_variant(int path, int64_t M, int64_t N, int64_t K)
{
    const int* cfgs = batched_cfgs(path);
    const int nv = batched_count(path);
    int tuned = g_forced[path].load();
    if (tuned < 0) tuned = table_lookup(path, M, N, K, 1);
    if (tuned < 0) tuned = table_lookup(path, M, N, K, 0);
    for (int v = 0; v < nv; ++v)
        if (cfgs[v] == tuned) return v;
    if (M >= 128 && N >= 128) return nv - 1;   // 128 x 128
    if (M >= 128 && nv == 3) return 1;         // 128 x 64
    return 0;                                  // 64 x 64
}

// Compute units of the current device, queried once per device.  Threads
// that race on the first query each store the same value into an atomic
// slot, so concurrent callers never read a torn or half-written entry.
int device_cus()
{
    static std::atomic<int> cus[64];   // zero-initialised (static storage)
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cus[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
            n = 256;
        cus[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

// Batched workspace: a 256-byte header holding the work-list counter, then
// the problem descriptors.  Both travel in one host-to-device copy, which also
// resets the counter to 0 for every launch.
constexpr size_t kBatchedHeader = 256;

size_t batched_workspace(int64_t count)
{
    return count > 0 ? kBatchedHeader + size_t(count) * sizeof(mg::BatchProblem) : 0;
}

// ---- SYR2K: square tile configuration and split of each tile's K loop.
// The triangle of T x T tiles has T(T+1)/2 tiles; when that count is not a
// whole number of rounds over the compute units, the last round runs mostly
// idle.  Cutting every tile's K loop (both products, 2*ceil(K/BK) panels)
// into S ranges turns the tiles into S times as many shorter work items; S is
// chosen to minimise  rounds(S) / S  +  S * r,  the makespan in whole-tile
// units plus the reduction, which moves 8 bytes per triangle entry and split
// (r = that traffic's time over one tile's matrix-core time, taken as
// 0.18 * tiles / K from the measured FP32 rates: 0.53 TFLOP/s per CU, ~6 TB/s).
struct Syr2kPlan {
    int cfg, splits;
    int64_t chunk, ldp, stride;
    size_t bytes;
};

Syr2kPlan syr2k_plan(int64_t N, int64_t K)
{
    Syr2kPlan p{-1, 1, 0, 0, 0, 0};
    const int64_t cus = device_cus();
    auto tri = [&](int64_t b) { const int64_t t = (N + b - 1) / b; return t * (t + 1) / 2; };
    int cfg = g_forced[MG_PATH_FP32].load();
    if (cfg >= 0 && !mg::syr2k_config_supported(cfg)) return p;
    // 256 x 256 tiles once their triangle fills four rounds of the compute
    // units; below that the eight-wave 128 x 128 tile, whose finer triangle
    // splits into more even rounds; 64 x 64 only for triangles under half a
    // round of 128 x 128 tiles.
    if (cfg < 0) cfg = tri(256) >= 4 * cus ? 5 : 2 * tri(128) >= cus ? 18 : 3;
    p.cfg = cfg;
    const int bt = table_of(MG_PATH_FP32).cfgs[cfg].bm;
    const int bk = mg::syr2k_panel_depth(cfg);
    const int64_t tiles_n = tri(bt);
    const int64_t panels = 2 * ((K + bk - 1) / bk);
    int s = g_forced_splits[MG_PATH_FP32].load();
    if (s < 0) {
        const double r = 0.18 * double(tiles_n) / double(K);
        double best = 1e30;
        s = 1;
        for (int c = 1; c <= kMaxSplits && 2 * K / c >= kMinRange; ++c) {
            const double rounds = double((tiles_n * c + cus - 1) / cus);
            const double cost = rounds / c + c * r;
            if (cost < best - 1e-9) {
                best = cost;
                s = c;
            }
        }
    }
    if (s > 1) {
        p.chunk = (panels + s - 1) / s;
        p.splits = int((panels + p.chunk - 1) / p.chunk);
    }
    if (p.splits > 1) {
        p.ldp = round_up(N, 4);
        p.stride = N * p.ldp;
        p.bytes = align256(size_t(p.splits) * size_t(p.stride) * sizeof(float));
    } else {
        p.chunk = 0;
    }
    return p;
}

// ---- Allocation-free GEMM (mg_gemm_noalloc): a fixed scratch buffer in
// device memory stands in for the caller's workspace.  The array is a
// file-scope device variable, so each GPU the library runs on holds its own
// copy for the life of the process.  Host code never uses the array's name
// as an address (on the host it is only a stand-in for the symbol): the
// device address comes from hipGetSymbolAddress, taken once per device with
// that device current, and only that pointer is passed to kernels.
constexpr size_t kScratchBytes = MG_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::atomic<void*> g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mutex;

// Device address of the current device's scratch, or nullptr with *err set.
void* scratch_ptr(hipError_t* err)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *err = e != hipSuccess ? e : hipErrorInvalidDevice;
        return nullptr;
    }
    void* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (p != nullptr) return p;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
    if (p == nullptr) {
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        g_scratch_ptr[dev].store(p, std::memory_order_release);
    }
    return p;
}

}  // namespace

extern "C" {

int mg_gemm(int path, char transA, char transB, int64_t M, int64_t N, int64_t K, float alpha,
            const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
            int64_t ldc, void* workspace, size_t workspace_bytes, void* stream)
{
    int st = validate(transA, transB, M, N, K, A, lda, B, ldb, C, ldc);
    if (st != MG_OK) return st;
    if (!float_path(path)) return MG_ERR_UNSUPPORTED;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (path == MG_PATH_FP8_T128) {
        if (K > kMaxFp8K) return MG_ERR_TOO_LARGE;
        const size_t need = fp8_workspace(M, N, K).total;
        if (M > 0 && N > 0 && K > 0 && alpha != 0.f &&
            (workspace == nullptr || workspace_bytes < need ||
             (reinterpret_cast<uintptr_t>(workspace) & 255) != 0))
            return MG_ERR_WORKSPACE;
    }
    if (M == 0 || N == 0) return MG_OK;
    if (K == 0 || alpha == 0.f) {
        if (beta == 1.f) return MG_OK;
        return hip_status(mg::launch_scale_c(C, M, N, ldc, beta, s));
    }
    if (path == MG_PATH_FP8_T128) {
        const Fp8Workspace w = fp8_workspace(M, N, K);
        uint8_t* base = static_cast<uint8_t*>(workspace);
        st = run_fp8_pack(is_t(transA), M, K, A, lda, base + w.qa, base + w.sa, s);
        if (st != MG_OK) return st;
        // op(B)^T is N x K: stored as is when transB is 'T', transposed when 'N'.
        st = run_fp8_pack(!is_t(transB), N, K, B, ldb, base + w.qb, base + w.sb, s);
        if (st != MG_OK) return st;
        return run_fp8_packed(M, N, K, alpha, base + w.qa, base + w.sa, base + w.qb, base + w.sb,
                              beta, C, ldc, s);
    }
    // Optional workspace uses: pre-packed 16-bit planes at its start, then
    // the split-K partials (plan_gemm).
    uint8_t* ws = static_cast<uint8_t*>(workspace);
    const size_t avail = (ws != nullptr && (reinterpret_cast<uintptr_t>(ws) & 255) == 0) ? workspace_bytes : 0;
    const GemmPlan gp = plan_gemm(path, M, N, K, avail);
    void* planes = gp.planes ? ws : nullptr;
    void* split_ws = gp.split.splits > 1 ? ws + gp.planes : nullptr;
    return run_gemm(path, is_t(transA), is_t(transB), M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s, gp.cfg,
                    gp.split, split_ws, planes);
}

int mg_gemm_noalloc(int path, char transA, char transB, int64_t M, int64_t N, int64_t K, float alpha,
                    const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
                    int64_t ldc, void* stream)
{
    const int st = validate(transA, transB, M, N, K, A, lda, B, ldb, C, ldc);
    if (st != MG_OK) return st;
    if (!float_path(path)) return MG_ERR_UNSUPPORTED;
    if (path == MG_PATH_FP8_T128) {
        if (K > kMaxFp8K) return MG_ERR_TOO_LARGE;
        // the packed FP8 operands are required, and must fit the scratch
        if (M > 0 && N > 0 && K > 0 && alpha != 0.f && fp8_workspace(M, N, K).total > kScratchBytes)
            return MG_ERR_SCRATCH;
    }
    if (M == 0 || N == 0) return MG_OK;
    hipError_t e = hipSuccess;
    void* ws = scratch_ptr(&e);
    if (ws == nullptr) return hip_status(e);
    // the plan mg_gemm makes for a workspace of kScratchBytes (plan_gemm)
    return mg_gemm(path, transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, kScratchBytes, stream);
}

int mg_sgemm(char transA, char transB, int64_t M, int64_t N, int64_t K, float alpha,
             const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
             int64_t ldc, void* stream)
{
    return mg_gemm(MG_PATH_FP32, transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                   nullptr, 0, stream);
}

size_t mg_gemm_workspace_size(int path, char transA, char transB, int64_t M, int64_t N, int64_t K)
{
    (void)transA; (void)transB;
    if (M <= 0 || N <= 0 || K <= 0 || !float_path(path) || beyond_int(M, N, K)) return 0;
    if (path == MG_PATH_FP8_T128) return K > kMaxFp8K ? 0 : fp8_workspace(M, N, K).total;
    const GemmPlan gp = plan_gemm(path, M, N, K, SIZE_MAX);
    return gp.planes + gp.split.bytes;
}

int mg_gemm_plan(int path, int64_t M, int64_t N, int64_t K, size_t workspace_bytes, int* out3)
{
    if (!float_path(path)) return MG_ERR_UNSUPPORTED;
    if (M < 0) return -2;
    if (N < 0) return -3;
    if (K < 0) return -4;
    if (out3 == nullptr) return -6;
    if (beyond_int(M, N, K)) return MG_ERR_TOO_LARGE;
    if (path == MG_PATH_FP8_T128) {
        if (K > kMaxFp8K) return MG_ERR_TOO_LARGE;
        out3[0] = pick_config(path, M, N, K);
        out3[1] = 1;
        out3[2] = 1;
        return (M > 0 && N > 0 && K > 0 && workspace_bytes < fp8_workspace(M, N, K).total) ? MG_ERR_WORKSPACE
                                                                                           : MG_OK;
    }
    const GemmPlan gp = plan_gemm(path, M, N, K, workspace_bytes);
    out3[0] = gp.cfg;
    out3[1] = gp.split.splits > 1 ? gp.split.splits : 1;
    out3[2] = gp.planes ? 1 : 0;
    return MG_OK;
}

int mg_fp8_packed_size(int64_t R, int64_t K, size_t* q_bytes, size_t* scale_bytes)
{
    if (R < 0) return -1;
    if (K < 0) return -2;
    if (beyond_int(R, K, 0)) return MG_ERR_TOO_LARGE;
    if (q_bytes) *q_bytes = fp8_q_bytes(R, K);
    if (scale_bytes) *scale_bytes = fp8_s_bytes(R, K);
    return MG_OK;
}

int mg_fp8_pack(char trans, int64_t R, int64_t K, const float* X, int64_t ldx, uint8_t* q,
                uint8_t* scales, void* stream)
{
    if (!is_n(trans) && !is_t(trans)) return -1;
    if (R < 0) return -2;
    if (K < 0) return -3;
    if (X == nullptr && R > 0 && K > 0) return -4;
    const int64_t cols = is_t(trans) ? R : K, rows = is_t(trans) ? K : R;
    if (ldx < (cols > 1 ? cols : 1) || !fits(rows, ldx)) return -5;
    if (q == nullptr) return -6;
    if (scales == nullptr) return -7;
    if (R > INT_MAX || K > INT_MAX) return MG_ERR_TOO_LARGE;
    return run_fp8_pack(is_t(trans), R, K, X, ldx, q, scales, reinterpret_cast<hipStream_t>(stream));
}

int mg_gemm_fp8_packed(int64_t M, int64_t N, int64_t K, float alpha, const uint8_t* qA,
                       const uint8_t* sA, const uint8_t* qB, const uint8_t* sB, float beta, float* C,
                       int64_t ldc, void* stream)
{
    if (M < 0) return -1;
    if (N < 0) return -2;
    if (K < 0) return -3;
    if (qA == nullptr || sA == nullptr) return -5;
    if (qB == nullptr || sB == nullptr) return -7;
    if (C == nullptr && M > 0 && N > 0) return -10;
    if (ldc < (N > 1 ? N : 1) || !fits(M, ldc)) return -11;
    if (M > INT_MAX || N > INT_MAX || K > kMaxFp8K) return MG_ERR_TOO_LARGE;
    if ((reinterpret_cast<uintptr_t>(qA) & 15) || (reinterpret_cast<uintptr_t>(qB) & 15)) return -5;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (M == 0 || N == 0) return MG_OK;
    if (K == 0 || alpha == 0.f) {
        if (beta == 1.f) return MG_OK;
        return hip_status(mg::launch_scale_c(C, M, N, ldc, beta, s));
    }
    return run_fp8_packed(M, N, K, alpha, qA, sA, qB, sB, beta, C, ldc, s);
}

int mg_syr2k(int path, char uplo, char trans, int64_t N, int64_t K, float alpha, const float* A, int64_t lda,
             const float* B, int64_t ldb, float beta, float* C, int64_t ldc, void* workspace,
             size_t workspace_bytes, void* stream)
{
    const bool lower = uplo == 'L' || uplo == 'l';
    if (!lower && uplo != 'U' && uplo != 'u') return -1;
    if (!is_n(trans) && !is_t(trans)) return -2;
    if (N < 0) return -3;
    if (K < 0) return -4;
    const bool tr = is_t(trans);
    const int64_t rows = tr ? K : N, cols = tr ? N : K;   // stored shape of A and B
    if (A == nullptr && N > 0 && K > 0) return -6;
    if (lda < (cols > 1 ? cols : 1) || !fits(rows, lda)) return -7;
    if (B == nullptr && N > 0 && K > 0) return -8;
    if (ldb < (cols > 1 ? cols : 1) || !fits(rows, ldb)) return -9;
    if (C == nullptr && N > 0) return -11;
    if (ldc < (N > 1 ? N : 1) || !fits(N, ldc)) return -12;
    if (path != MG_PATH_FP32) return MG_ERR_UNSUPPORTED;
    if (N > INT_MAX || K > INT_MAX) return MG_ERR_TOO_LARGE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (N == 0) return MG_OK;
    if (K == 0 || alpha == 0.f) {
        if (beta == 1.f) return MG_OK;
        return hip_status(mg::launch_scale_tri(C, N, ldc, beta, lower, s));
    }
    const Syr2kPlan plan = syr2k_plan(N, K);
    if (plan.cfg < 0) return MG_ERR_UNSUPPORTED;
    const int64_t t = (N + 63) / 64;
    if (t * (t + 1) / 2 > INT_MAX) return MG_ERR_TOO_LARGE;
    mg::GemmArgs g{};
    g.A = A; g.B = B; g.C = C;
    g.M = N; g.N = N; g.K = K;
    g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.alpha = alpha; g.beta = beta;
    g.vec_a = fast_operand(A, lda);
    g.vec_b = fast_operand(B, ldb);
    g.vec_c = aligned16(C) && ldc % 4 == 0;
    const bool split = plan.splits > 1 && workspace != nullptr && workspace_bytes >= plan.bytes &&
                       (reinterpret_cast<uintptr_t>(workspace) & 255) == 0;
    if (!split) return hip_status(mg::launch_syr2k(plan.cfg, lower, tr, 1, g, s));
    g.part = static_cast<float*>(workspace);
    g.k_chunk = plan.chunk;
    g.ldp = plan.ldp;
    g.part_stride = plan.stride;
    hipError_t e = mg::launch_syr2k(plan.cfg, lower, tr, plan.splits, g, s);
    if (e != hipSuccess) return hip_status(e);
    return hip_status(mg::launch_syr2k_reduce(g, plan.splits, lower, s));
}

size_t mg_syr2k_workspace_size(int path, int64_t N, int64_t K)
{
    if (path != MG_PATH_FP32 || N <= 0 || K <= 0 || beyond_int(N, K, 0)) return 0;
    return syr2k_plan(N, K).bytes;
}

int mg_syr2k_plan(int path, int64_t N, int64_t K, int* out2)
{
    if (path != MG_PATH_FP32) return MG_ERR_UNSUPPORTED;
    if (N < 0) return -3;
    if (K < 0) return -4;
    if (out2 == nullptr) return -5;
    if (N > INT_MAX || K > INT_MAX) return MG_ERR_TOO_LARGE;
    if (N == 0 || K == 0) {   // no tile kernel runs
        out2[0] = -1;
        out2[1] = 0;
        return MG_OK;
    }
    const Syr2kPlan plan = syr2k_plan(N, K);
    if (plan.cfg < 0) return MG_ERR_UNSUPPORTED;
    out2[0] = plan.cfg;
    out2[1] = plan.splits;
    return MG_OK;
}

size_t mg_gemm_i8_workspace_size(int64_t M, int64_t N, int64_t K)
{
    if (M <= 0 || N <= 0 || K <= 0 || beyond_int(M, N, K)) return 0;
    return i8_workspace(M, N, K).total;
}

int mg_gemm_i8(char transA, char transB, int64_t M, int64_t N, int64_t K, int32_t alpha, const int8_t* A,
               int64_t lda, const int8_t* B, int64_t ldb, int32_t beta, int32_t* C, int64_t ldc,
               void* workspace, size_t workspace_bytes, void* stream)
{
    int st = validate(transA, transB, M, N, K, A, lda, B, ldb, C, ldc);
    if (st != MG_OK) return st;
    if (K > kMaxI8K) return MG_ERR_TOO_LARGE;
    const bool product = M > 0 && N > 0 && K > 0 && alpha != 0;
    if (product && (workspace == nullptr || workspace_bytes < i8_workspace(M, N, K).total ||
                    (reinterpret_cast<uintptr_t>(workspace) & 255) != 0))
        return MG_ERR_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (M == 0 || N == 0) return MG_OK;
    if (!product) {
        if (beta == 1) return MG_OK;
        return hip_status(mg::launch_scale_c_i32(C, M, N, ldc, beta, s));
    }
    const I8Workspace w = i8_workspace(M, N, K);
    int8_t* base = static_cast<int8_t*>(workspace);
    st = run_i8_pack(is_t(transA), M, K, A, lda, base + w.qa, s);
    if (st != MG_OK) return st;
    // op(B)^T is N x K: stored as is when transB is 'T', transposed when 'N'.
    st = run_i8_pack(!is_t(transB), N, K, B, ldb, base + w.qb, s);
    if (st != MG_OK) return st;
    return run_i8_packed(M, N, K, alpha, base + w.qa, base + w.qb, beta, C, ldc, s);
}

int mg_i8_packed_size(int64_t R, int64_t K, size_t* bytes)
{
    if (R < 0) return -1;
    if (K < 0) return -2;
    if (beyond_int(R, K, 0)) return MG_ERR_TOO_LARGE;
    if (bytes) *bytes = fp8_q_bytes(R, K);
    return MG_OK;
}

int mg_i8_pack(char trans, int64_t R, int64_t K, const int8_t* X, int64_t ldx, int8_t* q, void* stream)
{
    if (!is_n(trans) && !is_t(trans)) return -1;
    if (R < 0) return -2;
    if (K < 0) return -3;
    if (X == nullptr && R > 0 && K > 0) return -4;
    const int64_t cols = is_t(trans) ? R : K, rows = is_t(trans) ? K : R;
    if (ldx < (cols > 1 ? cols : 1) || !fits(rows, ldx)) return -5;
    if (q == nullptr || (reinterpret_cast<uintptr_t>(q) & 15) != 0) return -6;
    if (R > INT_MAX || K > kMaxI8K) return MG_ERR_TOO_LARGE;
    return run_i8_pack(is_t(trans), R, K, X, ldx, q, reinterpret_cast<hipStream_t>(stream));
}

int mg_gemm_i8_packed(int64_t M, int64_t N, int64_t K, int32_t alpha, const int8_t* qA, const int8_t* qB,
                      int32_t beta, int32_t* C, int64_t ldc, void* stream)
{
    if (M < 0) return -1;
    if (N < 0) return -2;
    if (K < 0) return -3;
    if (qA == nullptr || (reinterpret_cast<uintptr_t>(qA) & 15) != 0) return -5;
    if (qB == nullptr || (reinterpret_cast<uintptr_t>(qB) & 15) != 0) return -6;
    if (C == nullptr && M > 0 && N > 0) return -8;
    if (ldc < (N > 1 ? N : 1) || !fits(M, ldc)) return -9;
    if (M > INT_MAX || N > INT_MAX || K > kMaxI8K) return MG_ERR_TOO_LARGE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (M == 0 || N == 0) return MG_OK;
    if (K == 0 || alpha == 0) {
        if (beta == 1) return MG_OK;
        return hip_status(mg::launch_scale_c_i32(C, M, N, ldc, beta, s));
    }
    return run_i8_packed(M, N, K, alpha, qA, qB, beta, C, ldc, s);
}

int mg_num_configs(int path)
{
    return table_of(path).n;
}

int mg_config_info(int path, int index, int* out6)
{
    if (out6 == nullptr) return MG_ERR_UNSUPPORTED;
    const ConfigTable t = table_of(path);
    if (index >= 0 && index < t.n) {
        const mg::SgemmConfig& c = t.cfgs[index];
        out6[0] = c.id; out6[1] = c.bm; out6[2] = c.bn; out6[3] = c.bk; out6[4] = c.wm; out6[5] = c.wn;
        return MG_OK;
    }
    return MG_ERR_UNSUPPORTED;
}

int mg_config_packs(int path, int index)
{
    const ConfigTable t = table_of(path);
    if (index < 0 || index >= t.n) return MG_ERR_UNSUPPORTED;
    return t.cfgs[index].direct ? 0 : 1;
}

int mg_config_uses_mfma(int path, int index)
{
    const ConfigTable t = table_of(path);
    if (index < 0 || index >= t.n) return MG_ERR_UNSUPPORTED;
    return t.cfgs[index].valu ? 0 : 1;
}

int mg_force_config(int path, int config_id)
{
    if (!valid_path(path)) return MG_ERR_UNSUPPORTED;
    if (config_id != -1 && !config_valid(path, config_id)) return MG_ERR_UNSUPPORTED;
    g_forced[path].store(config_id);
    return MG_OK;
}

int mg_force_splits(int path, int splits)
{
    if (!valid_path(path)) return MG_ERR_UNSUPPORTED;
    if (splits < -1 || splits == 0 || splits > kMaxSplits) return MG_ERR_UNSUPPORTED;
    g_forced_splits[path].store(splits);
    return MG_OK;
}

int mg_force_tile_order(int path, int remap, int group_m)
{
    if (!valid_path(path)) return MG_ERR_UNSUPPORTED;
    if (remap == -1) {
        g_forced_order[path].store(-1);
        return MG_OK;
    }
    if ((remap != 0 && remap != 1) || group_m < 1 || group_m > 64) return MG_ERR_UNSUPPORTED;
    g_forced_order[path].store(remap * 256 + group_m);
    return MG_OK;
}

int mg_split_count(int path, int64_t M, int64_t N, int64_t K)
{
    if (table_of(path).n == 0 || M <= 0 || N <= 0 || K <= 0 || beyond_int(M, N, K)) return 1;
    return split_plan(path, pick_config(path, M, N, K), M, N, K).splits;
}

int mg_bf16_split(const float* x, int64_t n, uint16_t* hi, uint16_t* lo, void* stream)
{
    if (n < 0) return -2;
    if (n == 0) return MG_OK;
    if (x == nullptr) return -1;
    if (hi == nullptr) return -3;
    return hip_status(mg::launch_bf16_split(x, n, hi, lo, reinterpret_cast<hipStream_t>(stream)));
}

int mg_load_tuning(const char* path)
{
    std::call_once(g_table_init, table_clear);
    std::lock_guard<std::mutex> lock(g_table_mutex);
    if (path == nullptr) {
        table_clear();
        g_exact.clear();
        return MG_OK;
    }
    FILE* f = std::fopen(path, "r");
    if (!f) return MG_ERR_BAD_TABLE;
    static int8_t fresh[2][kPaths][kBuckets][kBuckets][kBuckets];
    std::memset(fresh, -1, sizeof(fresh));
    std::vector<ExactEntry> exact;
    char line[256];
    int bad = 0;
    while (std::fgets(line, sizeof(line), f)) {
        const char* q = line;
        while (*q == ' ' || *q == '\t') ++q;
        if (*q == '#' || *q == '\n' || *q == '\r' || *q == 0) continue;
        long long p, a, b, c, cfg, splits = -1;
        char mode[8] = "s";
        int used = 0;
        const int got = std::sscanf(q, "%lld %lld %lld %lld %lld %7s %n", &p, &a, &b, &c, &cfg, mode, &used);
        if (got < 5 || p < 0 || p >= kPaths || cfg < 0 || cfg > 127 || !config_valid(int(p), int(cfg)) ||
            mode[1] != 0) {
            bad = 1;
            break;
        }
        if (mode[0] == 'x') {
            // exact shape: M N K (1 .. INT_MAX) and an optional K-range count
            if (got == 6 && q[used] != 0 && q[used] != '\n' && q[used] != '\r' && q[used] != '#') {
                char* end = nullptr;
                splits = std::strtoll(q + used, &end, 10);
                if (end == q + used) {
                    bad = 1;
                    break;
                }
            }
            if (a < 1 || b < 1 || c < 1 || a > INT_MAX || b > INT_MAX || c > INT_MAX ||
                !(splits == -1 || (splits >= 1 && splits <= kMaxSplits))) {
                bad = 1;
                break;
            }
            exact.push_back(ExactEntry{int(p), a, b, c, int(cfg), int(splits)});
            continue;
        }
        if (!(mode[0] == 's' || mode[0] == 'b') || a < 0 || a >= kBuckets || b < 0 || b >= kBuckets || c < 0 ||
            c >= kBuckets) {
            bad = 1;
            break;
        }
        fresh[mode[0] == 'b' ? 1 : 0][p][a][b][c] = int8_t(cfg);
    }
    std::fclose(f);
    if (bad) return MG_ERR_BAD_TABLE;
    std::memcpy(g_table, fresh, sizeof(g_table));
    g_exact.swap(exact);
    return MG_OK;
}

int mg_tuned_config(int path, int64_t M, int64_t N, int64_t K)
{
    if (!valid_path(path) || M < 0 || N < 0 || K < 0) return MG_ERR_UNSUPPORTED;
    if (beyond_int(M, N, K)) return MG_ERR_TOO_LARGE;
    return pick_config(path, M, N, K);
}

int mg_batched_config(int path, int64_t M, int64_t N, int64_t K)
{
    if (!batched_path(path) || M < 0 || N < 0 || K < 0) return MG_ERR_UNSUPPORTED;
    if (beyond_int(M, N, K)) return MG_ERR_TOO_LARGE;
    return batched_cfgs(path)[choose_batched_variant(path, M, N, K)];
}

size_t mg_gemm_batched_workspace_size(int path, int64_t count)
{
    if (!batched_path(path) || count < 0 || count > INT_MAX) return 0;
    return batched_workspace(count);
}

}  // extern "C"

namespace {

// stamps: nullptr, or room for 2 * grid words (checked by the caller).
int run_batched(int path, int64_t count, const mg_problem* problems, void* workspace, size_t workspace_bytes,
                void* stream, int64_t* bad_problem, unsigned long long* stamps, int* grid_out)
{
    if (grid_out) *grid_out = 0;
    if (!batched_path(path)) return MG_ERR_UNSUPPORTED;
    if (count < 0) return -2;
    if (count > INT_MAX) return MG_ERR_TOO_LARGE;
    if (count > 0 && problems == nullptr) return -3;
    // validate every problem before touching the device
    for (int64_t i = 0; i < count; ++i) {
        const mg_problem& q = problems[i];
        const int st = validate(q.transA, q.transB, q.M, q.N, q.K, q.A, q.lda, q.B, q.ldb, q.C, q.ldc);
        if (st != MG_OK) {
            if (bad_problem) *bad_problem = i;
            return st;
        }
    }
    if (count == 0) return MG_OK;
    if (workspace == nullptr || workspace_bytes < batched_workspace(count) ||
        (reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
        return MG_ERR_WORKSPACE;

    const ConfigTable t = table_of(path);
    const int* cfgs = batched_cfgs(path);
    std::vector<mg::BatchProblem> host;
    host.reserve(size_t(count));
    for (int64_t i = 0; i < count; ++i) {
        const mg_problem& q = problems[i];
        if (q.M == 0 || q.N == 0) continue;
        mg::BatchProblem b{};
        b.variant = choose_batched_variant(path, q.M, q.N, q.K);
        const mg::SgemmConfig& c = t.cfgs[cfgs[b.variant]];
        b.ta = is_t(q.transA);
        b.tb = is_t(q.transB);
        b.g.A = q.A; b.g.B = q.B; b.g.C = q.C;
        b.g.M = q.M; b.g.N = q.N;
        b.g.K = (q.alpha == 0.f) ? 0 : q.K;   // alpha == 0: A and B are not read
        b.g.lda = q.lda; b.g.ldb = q.ldb; b.g.ldc = q.ldc;
        b.g.alpha = q.alpha; b.g.beta = q.beta;
        b.g.tiles_m = int((q.M + c.bm - 1) / c.bm);
        b.g.tiles_n = int((q.N + c.bn - 1) / c.bn);
        b.g.group_m = 1;
        b.g.vec_a = fast_operand(q.A, q.lda);
        b.g.vec_b = fast_operand(q.B, q.ldb);
        b.g.vec_c = aligned16(q.C) && q.ldc % 4 == 0;
        host.push_back(b);
    }
    if (host.empty()) return MG_OK;
    // longest tiles first
    std::stable_sort(host.begin(), host.end(), [&](const mg::BatchProblem& x, const mg::BatchProblem& y) {
        const mg::SgemmConfig& cx = t.cfgs[cfgs[x.variant]];
        const mg::SgemmConfig& cy = t.cfgs[cfgs[y.variant]];
        return int64_t(cx.bm) * cx.bn * (x.g.K + 1) > int64_t(cy.bm) * cy.bn * (y.g.K + 1);
    });
    int64_t total = 0;
    for (auto& b : host) {
        b.tile_begin = total;
        total += int64_t(b.g.tiles_m) * b.g.tiles_n;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::vector<uint8_t> upload(kBatchedHeader + host.size() * sizeof(mg::BatchProblem), 0);
    std::memcpy(upload.data() + kBatchedHeader, host.data(), host.size() * sizeof(mg::BatchProblem));
    hipError_t e = hipMemcpyAsync(workspace, upload.data(), upload.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_status(e);
    const int64_t slots = int64_t(device_cus()) * mg::batched_blocks_per_cu(path);
    const int grid = int(std::min<int64_t>(total, slots));
    uint8_t* base = static_cast<uint8_t*>(workspace);
    if (grid_out) *grid_out = grid;
    return hip_status(mg::launch_gemm_batched(path, reinterpret_cast<const mg::BatchProblem*>(base + kBatchedHeader),
                                              int(host.size()), total, grid,
                                              reinterpret_cast<unsigned long long*>(base), stamps, s));
}

}  // namespace

extern "C" {

int mg_gemm_batched(int path, int64_t count, const mg_problem* problems, void* workspace,
                    size_t workspace_bytes, void* stream, int64_t* bad_problem)
{
    return run_batched(path, count, problems, workspace, workspace_bytes, stream, bad_problem, nullptr, nullptr);
}

int mg_batched_slots(int path)
{
    if (!batched_path(path)) return 0;
    return int(std::min<int64_t>(int64_t(device_cus()) * mg::batched_blocks_per_cu(path), INT_MAX / 2));
}

int mg_gemm_batched_timed(int path, int64_t count, const mg_problem* problems, void* workspace,
                          size_t workspace_bytes, void* stream, int64_t* bad_problem,
                          unsigned long long* stamps, int64_t stamps_len, int* grid)
{
    if (grid) *grid = 0;
    if (!batched_path(path)) return MG_ERR_UNSUPPORTED;
    if (stamps == nullptr || stamps_len < 2 * int64_t(mg_batched_slots(path))) return -8;
    return run_batched(path, count, problems, workspace, workspace_bytes, stream, bad_problem, stamps, grid);
}

int64_t mg_wall_clock_hz(void)
{
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return -1;
    return int64_t(khz) * 1000;
}

int mg_shader_clock_mhz(void* stream, int64_t microseconds, double* mhz)
{
    if (microseconds < 1 || microseconds > 1000000) return -2;
    if (mhz == nullptr) return -3;
    const int64_t hz = mg_wall_clock_hz();
    if (hz <= 0) return MG_ERR_HIP - int(hipErrorNoDevice);
    const int64_t ticks = std::max<int64_t>(1, hz * microseconds / 1000000);
    return hip_status(mg::measure_sclk(reinterpret_cast<hipStream_t>(stream), ticks, double(hz), mhz));
}

const char* mg_status_string(int status)
{
    switch (status) {
    case MG_OK: return "success";
    case -1: return "invalid argument 1 (transA)";
    case -2: return "invalid argument 2 (transB)";
    case -3: return "invalid argument 3 (M < 0)";
    case -4: return "invalid argument 4 (N < 0)";
    case -5: return "invalid argument 5 (K < 0)";
    case -7: return "invalid argument 7 (A is NULL)";
    case -8: return "invalid argument 8 (lda too small or too large)";
    case -9: return "invalid argument 9 (B is NULL)";
    case -10: return "invalid argument 10 (ldb too small or too large)";
    case -12: return "invalid argument 12 (C is NULL)";
    case -13: return "invalid argument 13 (ldc too small or too large)";
    case MG_ERR_WORKSPACE: return "workspace missing or too small";
    case MG_ERR_UNSUPPORTED: return "unsupported path or configuration";
    case MG_ERR_TOO_LARGE: return "dimension too large for the kernels";
    case MG_ERR_BAD_TABLE: return "tuning table unreadable or malformed";
    case MG_ERR_SCRATCH: return "problem needs more than the allocation-free entry point's scratch memory";
    default: break;
    }
    if (status <= MG_ERR_HIP) return hipGetErrorString(hipError_t(MG_ERR_HIP - status));
    return "unknown status";
}

}  // extern "C"
