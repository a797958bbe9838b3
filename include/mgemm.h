/*
 * mgemm.h -- C ABI of the layered GEMM library for AMD MI355X (gfx950).
 *
 * The library computes the GEMM of Kuzma et al., "Fast Matrix Multiplication
 * via Compiler-only Layered Data Reorganization and Intrinsic Lowering"
 * (SPE 2023), Section 3 and Algorithm 1:
 *
 *     C <- alpha * op(A) * op(B) + beta * C
 *
 * with op(X) = X ('N') or X^T ('T'), op(A) M x K, op(B) K x N, C M x N, using
 * the paper's layers: blocking of C and K into tiles and panels, packing of
 * the A and B panels into on-chip memory (LDS) in the micro-kernel's access
 * order, and a micro-kernel lowered to the matrix engine (MFMA).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Storage.  Row-major.  lda/ldb/ldc are row strides in elements.
 *   transA 'N': A is stored M x K, lda >= max(1, K);  'T': K x M, lda >= max(1, M).
 *   transB 'N': B is stored K x N, ldb >= max(1, N);  'T': N x K, ldb >= max(1, K).
 *   ldc >= max(1, N).  'n'/'t' are accepted and 'C'/'c' means 'T' (real data).
 *   A column-major caller computes gemm(tA, tB, M, N, K, A, lda, B, ldb, C, ldc)
 *   as the row-major gemm(tB, tA, N, M, K, B, ldb, A, lda, C, ldc).
 * Ownership.  A, B, C and any workspace are DEVICE pointers owned by the caller.
 *   The library never allocates or frees device memory in these calls.
 *   A and B are read only; C is read only when beta != 0 and always written.
 *   C must not overlap A or B.
 * Asynchrony.  `stream` is a hipStream_t (NULL = the default stream).  Work is
 *   enqueued and the call returns without synchronising; faults inside a
 *   kernel surface at the caller's next synchronisation.
 * Quick returns (BLAS).  M == 0 or N == 0: nothing is touched.  K == 0 or
 *   alpha == 0: C <- beta*C (beta == 0 writes zeros without reading C,
 *   beta == 1 does nothing); A and B are not read.
 * Errors.  0 is success.  A negative value -i names the invalid argument by
 *   its 1-based position in mg_sgemm's signature (BLAS xerbla numbering):
 *   transA -1, transB -2, M -3, N -4, K -5, A -7, lda -8, B -9, ldb -10,
 *   C -12, ldc -13.  A NULL pointer is an error only when its matrix has a
 *   non-zero extent.  All argument errors are detected on the host before any
 *   device call.  Other codes are the MG_ERR_* values below; a HIP runtime
 *   error e is returned as MG_ERR_HIP - e.  mg_status_string() describes any
 *   code.
 * Sizes.  Every compute entry point rejects a dimension above INT_MAX with
 *   MG_ERR_TOO_LARGE.  For such a dimension the query functions answer
 *   without computing: the *_workspace_size functions return 0,
 *   mg_split_count 1, and mg_tuned_config, mg_batched_config,
 *   mg_fp8_packed_size and mg_i8_packed_size MG_ERR_TOO_LARGE.  The FP8
 *   GEMMs (mg_gemm with MG_PATH_FP8_T128, mg_gemm_fp8_packed) take K up to
 *   2^23 = 8388608 and return MG_ERR_TOO_LARGE beyond it (their kernels
 *   address a 256-row panel with 32-bit offsets); mg_gemm_workspace_size
 *   returns 0 there.  INT8 takes K up to 131071 (see mg_gemm_i8).
 */
#ifndef MGEMM_H
#define MGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Arithmetic of a GEMM ("path").  Inputs and outputs are FP32 on every path;
 * the path only changes what the matrix engine multiplies.  The conversions
 * happen while packing (Algorithm 1's pack step), so HBM traffic stays FP32. */
enum mg_path {
    MG_PATH_FP32 = 0,     /* FP32 x FP32 MFMA, FP32 accumulation                 */
    MG_PATH_BF16X3 = 1,   /* x = hi + lo (bf16 each); hi*hi + hi*lo + lo*hi on
                             BF16 MFMA, FP32 accumulation                         */
    MG_PATH_BF16 = 2,     /* operands rounded to bf16 (nearest-even), FP32 acc.  */
    MG_PATH_FP8_T128 = 3, /* OCP E4M3 with one power-of-two FP32 scale per
                             128 x 128 tile of op(A) and op(B), FP32 accumulation */
    MG_PATH_FP16 = 4      /* operands rounded to IEEE binary16 (nearest-even;
                             |x| >= 65520 becomes infinity), FP32 accumulation */
};

/* Configuration table of the INT8 entry points (mg_gemm_i8, mg_gemm_i8_packed)
 * for mg_num_configs, mg_config_info, mg_force_config and mg_tuned_config.
 * Not a path of mg_gemm: its operands are int8, not FP32. */
enum { MG_CONFIGS_I8 = 5 };

enum mg_status {
    MG_OK = 0,
    MG_ERR_WORKSPACE = -100,    /* workspace missing or smaller than required */
    MG_ERR_UNSUPPORTED = -101,  /* unknown path or configuration id           */
    MG_ERR_TOO_LARGE = -102,    /* a dimension exceeds what the kernels index  */
    MG_ERR_BAD_TABLE = -103,    /* tuning table unreadable or malformed        */
    MG_ERR_SCRATCH = -104,      /* needs more than MG_NOALLOC_SCRATCH_BYTES    */
    MG_ERR_HIP = -1000          /* MG_ERR_HIP - hipError_t                     */
};

/* One GEMM of a batch: the arguments of mg_sgemm (device pointers). */
typedef struct mg_problem {
    char transA, transB;
    int64_t M, N, K;
    float alpha, beta;
    const float *A;
    int64_t lda;
    const float *B;
    int64_t ldb;
    float *C;
    int64_t ldc;
} mg_problem;

/*
 * FP32 GEMM on the FP32 matrix cores (the paper's experiments are all FP32
 * SGEMM, Section 4).  Equivalent to mg_gemm(MG_PATH_FP32, ..., NULL, 0, stream).
 */
int mg_sgemm(char transA, char transB, int64_t M, int64_t N, int64_t K,
             float alpha, const float *A, int64_t lda, const float *B, int64_t ldb,
             float beta, float *C, int64_t ldc, void *stream);

/*
 * GEMM on the given path.  `workspace` is device memory, caller-owned,
 * 256-byte aligned, of mg_gemm_workspace_size() bytes.  It holds:
 *   - MG_PATH_FP8_T128: the packed FP8 operands (required: MG_ERR_WORKSPACE
 *     if missing or too small);
 *   - MG_PATH_BF16 / MG_PATH_FP16 with M, N >= 512 and K <= 2^21: the
 *     operands rounded to bf16 / binary16 once (padded to 256 rows and 128 k);
 *   - MG_PATH_BF16X3 with configuration 6 or 7 (6 chosen for 256 x 256 tiles when
 *     M N >= 1250 (M + N)), M, N >= 512 and K <= 2^21: the operands split
 *     once into hi and lo bf16 terms, stored interleaved per 32 k (4 bytes
 *     per element);
 *   on these 16-bit paths the large-tile kernel copies the pre-packed
 *   panels straight into LDS;
 *   - every other path: the partial products of a split-K launch, used when
 *     the problem has fewer output tiles than the GPU has compute units and
 *     K >= 256 (the K loop is cut into ranges multiplied by separate
 *     workgroups, then summed in a fixed order, so results stay deterministic).
 * On the non-FP8 paths the workspace is optional: with NULL or fewer bytes
 * than mg_gemm_workspace_size() the GEMM is planned as if no K split were
 * possible (the tile shape chosen for an unsplit K loop; mg_sgemm always runs
 * this way), pre-packing the 16-bit operands if the planes still fit
 * (mg_gemm_plan tells which plan a given workspace gets).  Returns
 * MG_ERR_UNSUPPORTED for an unknown path.  Concurrent calls must not share a
 * workspace.
 */
int mg_gemm(int path, char transA, char transB, int64_t M, int64_t N, int64_t K,
            float alpha, const float *A, int64_t lda, const float *B, int64_t ldb,
            float beta, float *C, int64_t ldc,
            void *workspace, size_t workspace_bytes, void *stream);

/*
 * Allocation-free GEMM, for callers that cannot allocate device memory or
 * pass a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, semantics and error
 * codes as mg_gemm without the workspace: the library uses instead a fixed
 * scratch buffer of MG_NOALLOC_SCRATCH_BYTES (256 MiB) of device memory that
 * each GPU it runs on holds from the first call on that device until the
 * process ends.  The call allocates and frees nothing.  The plan is the one
 * mg_gemm makes for a workspace of that size (mg_gemm_plan with
 * MG_NOALLOC_SCRATCH_BYTES), so results equal mg_gemm's with such a
 * workspace bit for bit; on the non-FP8 paths a problem whose best plan
 * needs more scratch runs the plan made without a K split (and converts the
 * 16-bit operands inside the GEMM if their planes do not fit either).
 * MG_PATH_FP8_T128 needs its packed operands in the scratch and returns
 * MG_ERR_SCRATCH when they exceed it (about (M + N) K > 2^28 bytes).
 * Every call on one GPU shares that GPU's scratch, which keeps whatever the
 * last call left there (no call depends on its contents: everything read
 * from it is written first by the same call).  Calls that overlap in time
 * on one GPU (other streams, other host threads) race on the scratch and
 * must be serialised by the caller, e.g. by issuing them on one stream.
 */
#define MG_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int mg_gemm_noalloc(int path, char transA, char transB, int64_t M, int64_t N, int64_t K,
                    float alpha, const float *A, int64_t lda, const float *B, int64_t ldb,
                    float beta, float *C, int64_t ldc, void *stream);

/* Workspace bytes mg_gemm uses for this problem with the current selection
 * state (forced configuration, tuning table, forced split; 0 when none). */
size_t mg_gemm_workspace_size(int path, char transA, char transB,
                              int64_t M, int64_t N, int64_t K);

/*
 * The plan mg_gemm would run for this problem, given `workspace_bytes` of
 * 256-byte-aligned workspace, with the current selection state (the blocking
 * decision of Section 3.1, Eq. 1-7, made per shape): out3[0] = the
 * configuration id (mg_config_info), out3[1] = the number of K ranges (1: no
 * split), out3[2] = 1 if the operands are pre-packed into the workspace.
 * With the full mg_gemm_workspace_size() the plan is the best one; with less
 * the GEMM is planned as if no K split were possible (the tile chosen for an
 * unsplit K loop), using the pre-packed 16-bit planes if they still fit.
 * Host-only: no device call.  Errors: MG_ERR_UNSUPPORTED unknown path,
 * -2 M < 0, -3 N < 0, -4 K < 0, -6 out3 NULL, MG_ERR_TOO_LARGE as mg_gemm;
 * MG_PATH_FP8_T128 with too little workspace fills out3 and returns
 * MG_ERR_WORKSPACE, as mg_gemm would.
 */
int mg_gemm_plan(int path, int64_t M, int64_t N, int64_t K, size_t workspace_bytes, int *out3);

/*
 * SYR2K, the paper's extension of the macro level to another BLAS kernel
 * (Section 5.1), on one triangle of the symmetric N x N matrix C:
 *   trans 'N':  C <- alpha*A*B^T + alpha*B*A^T + beta*C   (A, B stored N x K)
 *   trans 'T':  C <- alpha*A^T*B + alpha*B^T*A + beta*C   (A, B stored K x N)
 * Row-major like mg_sgemm (lda, ldb >= K for 'N', >= N for 'T'; ldc >= N).
 * uplo 'L' reads and writes only C[i][j] with i >= j, 'U' only i <= j; the
 * other strict triangle is never touched.  beta == 0: C is not read;
 * alpha == 0 or K == 0: the triangle becomes beta*C.  path: MG_PATH_FP32 (the
 * only one; others return MG_ERR_UNSUPPORTED).  A forced FP32 configuration
 * must be square (ids 0, 3, 5, 18).  `workspace` (optional, device, 256-byte
 * aligned, mg_syr2k_workspace_size() bytes) holds partial tiles when each
 * tile's K loop is split over several workgroups (so that the triangle's
 * tiles fill the GPU's last round); with NULL or too few bytes the update
 * runs unsplit.  Partials are summed in a fixed order: results are
 * deterministic.  Argument codes follow BLAS xSYR2K: uplo -1, trans -2, N -3,
 * K -4, A -6, lda -7, B -8, ldb -9, C -11, ldc -12.
 */
int mg_syr2k(int path, char uplo, char trans, int64_t N, int64_t K, float alpha,
             const float *A, int64_t lda, const float *B, int64_t ldb, float beta,
             float *C, int64_t ldc, void *workspace, size_t workspace_bytes, void *stream);
size_t mg_syr2k_workspace_size(int path, int64_t N, int64_t K);

/*
 * The tiles mg_syr2k runs for this problem with the current selection state
 * and a workspace of mg_syr2k_workspace_size() bytes: out2[0] = the square
 * FP32 configuration id (mg_config_info), out2[1] = the number of ranges each
 * tile's two-product K loop is cut into (1: no split); N == 0 or K == 0
 * (no tile kernel runs) gives -1 and 0.  Host-only: no device
 * call.  Errors: MG_ERR_UNSUPPORTED for a path other than MG_PATH_FP32 or a
 * forced configuration that is not square, -3 N < 0, -4 K < 0, -5 out2
 * NULL, MG_ERR_TOO_LARGE as mg_syr2k.
 */
int mg_syr2k_plan(int path, int64_t N, int64_t K, int *out2);

/*
 * INT8 GEMM, the 8-bit integer operand type of the paper's Table 1:
 *   C <- alpha * op(A) * op(B) + beta * C
 * with int8 A and B (device pointers, stored and strided exactly as for
 * mg_sgemm, same argument codes), int32 C, alpha and beta.  The products are
 * summed exactly in int32 (K <= 131071 keeps every partial sum in range; a
 * larger K returns MG_ERR_TOO_LARGE), and alpha*sum + beta*C is computed
 * modulo 2^32 (two's-complement wrap-around).  beta == 0: C is not read;
 * alpha == 0 or K == 0: C <- beta*C.  `workspace` (device, caller-owned,
 * 256-byte aligned, mg_gemm_i8_workspace_size() bytes) receives the packed
 * operands (MG_ERR_WORKSPACE if missing or too small when a product is formed).
 */
int mg_gemm_i8(char transA, char transB, int64_t M, int64_t N, int64_t K,
               int32_t alpha, const int8_t *A, int64_t lda, const int8_t *B, int64_t ldb,
               int32_t beta, int32_t *C, int64_t ldc,
               void *workspace, size_t workspace_bytes, void *stream);
size_t mg_gemm_i8_workspace_size(int64_t M, int64_t N, int64_t K);

/*
 * The INT8 pack stage on its own, for operands packed once and reused.
 * mg_i8_pack writes op(X) (R x K; stored R x K when trans is 'N', K x R when
 * 'T', row stride ldx) into q as Rp x Kp int8 rows, Rp = roundup(R, 256),
 * Kp = roundup(K, 128), zero-padded; q (16-byte aligned) holds
 * mg_i8_packed_size() bytes.  mg_gemm_i8_packed multiplies packed op(A)
 * (R = M) and packed op(B)^T (R = N) with the semantics of mg_gemm_i8
 * (argument codes: M -1, N -2, K -3, qA -5, qB -6, C -8, ldc -9).
 */
int mg_i8_packed_size(int64_t R, int64_t K, size_t *bytes);
int mg_i8_pack(char trans, int64_t R, int64_t K, const int8_t *X, int64_t ldx, int8_t *q, void *stream);
int mg_gemm_i8_packed(int64_t M, int64_t N, int64_t K, int32_t alpha, const int8_t *qA,
                      const int8_t *qB, int32_t beta, int32_t *C, int64_t ldc, void *stream);

/*
 * Tile configurations (the blocking parameters of Section 3.1, Eq. 1-7, as
 * workgroup tile BM x BN, K-panel depth BK and per-wave micro-tile WM x WN).
 * mg_num_configs(path) counts the configurations of a path; mg_config_info
 * fills out[0..5] = {id, BM, BN, BK, WM, WN} and returns 0, or
 * MG_ERR_UNSUPPORTED for an unknown (path, index).
 */
int mg_num_configs(int path);
int mg_config_info(int path, int index, int *out6);

/*
 * 1 if configuration `index` of `path` packs its operand panels into LDS
 * before the micro-kernel reads them (the paper's Tiling+Packing strategy,
 * Section 4.1.3), 0 if its lanes load operands straight from global memory
 * into registers (the Tiling strategy: tiled loops, no packing), or
 * MG_ERR_UNSUPPORTED for an unknown (path, index).
 */
int mg_config_packs(int path, int index);

/*
 * 1 if configuration `index` of `path` runs its micro-kernel on the matrix
 * cores (MFMA: the target-specific lowering of the paper's matrix-multiply
 * intrinsic, Section 3.2), 0 if it runs it as scalar FP32 FMAs on the vector
 * ALUs (the generic lowering), or MG_ERR_UNSUPPORTED for an unknown
 * (path, index).
 */
int mg_config_uses_mfma(int path, int index);

/*
 * Force the configuration used for `path` (id from mg_config_info), or -1 to
 * return to automatic selection.  Process-wide; meant for the autotuner.
 */
int mg_force_config(int path, int config_id);

/*
 * Force the split-K factor of `path`: 1 never splits, 2..16 cuts K into (at
 * most) that many ranges of a multiple of 128 when K >= 256, -1 returns to the
 * automatic rule.  Process-wide; meant for the autotuner and tests.
 * mg_split_count gives the number of K ranges a GEMM of this shape would use
 * now (given a large enough workspace).
 */
int mg_force_splits(int path, int splits);
int mg_split_count(int path, int64_t M, int64_t N, int64_t K);

/*
 * Force the order in which the single-GEMM kernels of `path` (also
 * MG_CONFIGS_I8) walk their output tiles: groups of group_m (1..64) tile rows
 * taken column by column; remap 1 first gives each of the 8 XCDs a
 * contiguous range of that raster, remap 0 leaves the hardware's round-robin
 * placement (XCD = workgroup id mod 8).  remap -1 returns to the automatic
 * choice (group_m ignored).  Process-wide; meant for the autotuner and
 * tests.  The order changes only where each tile runs, never a result bit.
 */
int mg_force_tile_order(int path, int remap, int group_m);

/*
 * Tuning table written by the autotuner (the blocking decision of
 * Section 3.1, Eq. 1-7, made by measuring the candidates that a model of the
 * GPU's memories admits).  Text lines, '#' starts a comment:
 *   "path mb nb kb config [mode]" with mb/nb/kb = round(log2(M/N/K)) (0..20)
 *     and mode 's' (single GEMMs, the default) or 'b' (the batched kernel,
 *     which falls back to 's' entries);
 *   "path M N K config x [splits]": one exact shape (1 <= M, N, K <=
 *     INT_MAX) of single GEMMs, with the number of K ranges to cut its K
 *     loop into (1..16; omitted or -1: the automatic split rule).
 * config is an id from mg_config_info.  A loaded table replaces the previous
 * one; NULL clears it.  Selection order for every GEMM: mg_force_config,
 * then an exact entry, then the bucket entries, then the built-in rule (an
 * exact entry whose splits exceed 1 is skipped when the caller's workspace
 * cannot hold the partial products).  Load it before launching GEMMs from
 * other threads.  Returns MG_ERR_BAD_TABLE (previous table kept) for an
 * unreadable or malformed file.
 */
int mg_load_tuning(const char *path);

/* Configuration id a GEMM of this path and shape would use now. */
int mg_tuned_config(int path, int64_t M, int64_t N, int64_t K);

/*
 * Uneven batched GEMM in ONE persistent kernel launch (paths FP32, BF16X3 and
 * BF16).  problems: HOST array of `count` problems, each with the semantics
 * and argument rules of mg_sgemm (quick returns included); problems must not
 * write overlapping C.  Every problem is tiled with its own tile shape (chosen
 * by the tuning table, else by its size), and one grid that fills the GPU
 * takes the tiles of all problems, largest first, each workgroup taking the
 * next tile when it finishes one.
 * workspace: device memory of at least mg_gemm_batched_workspace_size bytes,
 * 256-byte aligned; it receives the problem descriptors and the work counter
 * (one host-to-device copy on `stream`, which may block the host until
 * earlier work on the stream is done).  Calls that overlap in time must not
 * share a workspace.
 * Errors: -2 count < 0, -3 problems NULL; an invalid problem i returns its
 * mg_sgemm code (-1 ... -13) and stores i in *bad_problem (if not NULL);
 * MG_ERR_WORKSPACE; MG_ERR_UNSUPPORTED for MG_PATH_FP8_T128.
 */
size_t mg_gemm_batched_workspace_size(int path, int64_t count);
/* Configuration id mg_gemm_batched would use for one problem of this shape. */
int mg_batched_config(int path, int64_t M, int64_t N, int64_t K);
int mg_gemm_batched(int path, int64_t count, const mg_problem *problems,
                    void *workspace, size_t workspace_bytes, void *stream,
                    int64_t *bad_problem);

/*
 * Timing of the persistent launch, for measuring its tail: the time that
 * workgroups which found the work list empty wait for the last tiles.
 * mg_gemm_batched_timed is mg_gemm_batched (same arguments, results and
 * errors) that also records, for each workgroup b of the launch,
 * stamps[2b] = the wall clock when it started and stamps[2b + 1] = the wall
 * clock after its last tile, and stores the number of workgroups in *grid
 * (if grid is not NULL; 0 when nothing was launched).  stamps: device array
 * of stamps_len >= 2 * mg_batched_slots(path) words, written asynchronously
 * on `stream`.  Extra error: -8 stamps NULL or too short.
 * mg_batched_slots: the most workgroups a persistent launch of this path
 * uses on the current device (compute units x resident workgroups per unit;
 * 0 for a path without a batched kernel).
 * mg_wall_clock_hz: ticks per second of the stamps' clock (constant rate,
 * independent of the shader clock); -1 if the device cannot be queried.
 */
int mg_batched_slots(int path);
int mg_gemm_batched_timed(int path, int64_t count, const mg_problem *problems,
                          void *workspace, size_t workspace_bytes, void *stream,
                          int64_t *bad_problem, unsigned long long *stamps,
                          int64_t stamps_len, int *grid);
int64_t mg_wall_clock_hz(void);

/*
 * The shader (core) clock the GPU runs at, for reporting a measured clock
 * beside a fraction of the spec peak (which assumes 2.4 GHz).  Launches a
 * probe of 16 one-wave workgroups on `stream`, behind the work already
 * queued there, each timing `microseconds` of the constant-rate wall clock
 * against the shader-cycle counter; waits for the stream (this call
 * synchronises, unlike the GEMMs) and stores the average clock in MHz in
 * *mhz.  Launched right behind a timed workload, it reads the clock as that
 * workload ends.  Concurrent calls are serialised.  Errors: -2 microseconds
 * outside [1, 10^6], -3 mhz NULL, MG_ERR_HIP - e for a runtime error.
 */
int mg_shader_clock_mhz(void *stream, int64_t microseconds, double *mhz);

/*
 * The pack-stage conversion of the BF16 paths on its own (Table 1's bf16
 * operand type, round to nearest even): hi[t] = bf16(x[t]) and, when lo is
 * not NULL, lo[t] = bf16(x[t] - hi[t]), as raw bf16 bit patterns.  x, hi, lo
 * are device arrays of n elements.  Runs the same device conversion the
 * bf16x3 and BF16 GEMMs use, so its output can be checked bit for bit.
 * Errors: -1 x NULL, -2 n < 0, -3 hi NULL (n > 0).
 */
int mg_bf16_split(const float *x, int64_t n, uint16_t *hi, uint16_t *lo, void *stream);

/*
 * FP8 path in two stages, for callers that quantise once and multiply many
 * times, and for timing the GEMM alone (mg_gemm on MG_PATH_FP8_T128 runs both
 * stages on its workspace).
 *
 * Packed operand format (the pack step of Algorithm 1, Section 3.1, into a
 * buffer in device memory, in the micro-kernel's access order): for a logical
 * R x K matrix X, Rp = R rounded up to a multiple of 256 and Kp = K rounded up
 * to a multiple of 128;
 *   q      : Rp x Kp bytes, row-major, q[r][k] = E4M3(X[r][k] / s(tile)) (OCP
 *            E4M3, round to nearest even; zero outside R x K);
 *   scales : (Rp/128) x (Kp/128) bytes, row-major, the E8M0 code (e + 127) of
 *            the tile scale s = 2^e, the smallest power of two with
 *            amax(tile) <= 448 * s (e = 0 for an all-zero tile).
 * Tiles are 128 x 128 and aligned to (0, 0).  Scales below 2^-127 (tile
 * maxima under about 2.6e-36) are clamped to 2^-127.
 *
 * mg_fp8_packed_size: bytes of q and of scales for an R x K operand.
 *   Errors -1 R < 0, -2 K < 0.
 * mg_fp8_pack: pack op(X), R x K, where trans 'N' means X is stored R x K and
 *   'T' means K x R (row stride ldx).  Pack A with (transA, M, K) and B as
 *   op(B)^T with (transB == 'N' ? 'T' : 'N', N, K).  q (16-byte aligned) and
 *   scales are device buffers of at least the sizes above.
 *   Errors -1 trans, -2 R < 0, -3 K < 0, -4 X NULL, -5 ldx, -6 q NULL,
 *   -7 scales NULL.
 * mg_gemm_fp8_packed: C <- alpha * dequant(qA) * dequant(qB)^T + beta * C for
 *   packed op(A) (M x K) and op(B)^T (N x K), FP32 accumulation.
 *   Errors -1 M, -2 N, -3 K, -5 qA/sA NULL or qA misaligned, -7 qB/sB NULL or
 *   misaligned, -10 C NULL, -11 ldc.
 */
int mg_fp8_packed_size(int64_t R, int64_t K, size_t *q_bytes, size_t *scale_bytes);
int mg_fp8_pack(char trans, int64_t R, int64_t K, const float *X, int64_t ldx,
                uint8_t *q, uint8_t *scales, void *stream);
int mg_gemm_fp8_packed(int64_t M, int64_t N, int64_t K, float alpha,
                       const uint8_t *qA, const uint8_t *sA,
                       const uint8_t *qB, const uint8_t *sB,
                       float beta, float *C, int64_t ldc, void *stream);

/* Human-readable description of a status code (static storage). */
const char *mg_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* MGEMM_H */
