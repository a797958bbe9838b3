/* Memory- and UB-checked run of the oracle's C code (built with
 * AddressSanitizer and UndefinedBehaviorSanitizer on the CPU).  Every buffer
 * is allocated with exactly the extent the call may touch, so a read or
 * write one element past it is reported; C0 is NULL whenever beta == 0, so
 * reading it would fault.  Exit status 0 when every call returned 0. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_gemm(char transA, char transB, int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                int64_t lda, const double *B, int64_t ldb, double beta, const double *C0, int64_t ldc0,
                double *C, double *D, int64_t ldc, int nthreads);
int oracle_gemm_entries(char transA, char transB, int64_t K, double alpha, const double *A, int64_t lda,
                        const double *B, int64_t ldb, double beta, const double *C0, int64_t ldc0,
                        int64_t count, const int64_t *I, const int64_t *J, double *C, double *D, int nthreads);
double oracle_round_to_bits(double x, int bits, int emin);
void oracle_bf16_split(int64_t n, const double *x, double *hi, double *lo);
void oracle_fp16_round(int64_t n, const double *x, double *out);
double oracle_e4m3_value(double x);
unsigned char oracle_e4m3_encode(double v);   /* exactly representable E4M3 values and NaN only */
double oracle_e4m3_decode(unsigned char b);
double oracle_tile_scale(double amax);
void oracle_fp8_quantize(int64_t rows, int64_t cols, const double *X, int64_t ldx, int64_t tile, uint8_t *q,
                         float *scales);
int oracle_gemm_i8(char transA, char transB, int64_t M, int64_t N, int64_t K, int32_t alpha, const int8_t *A,
                   int64_t lda, const int8_t *B, int64_t ldb, int32_t beta, const int32_t *C0, int64_t ldc0,
                   int32_t *C, int64_t ldc, int threads);
int oracle_syr2k(char uplo, char trans, int64_t N, int64_t K, double alpha, const double *A, int64_t lda,
                 const double *B, int64_t ldb, double beta, double *C, int64_t ldc, double *D, int threads);

static int failures = 0;
#define CHECK(cond) do { if (!(cond)) { fprintf(stderr, "failed: %s (line %d)\n", #cond, __LINE__); ++failures; } } while (0)

/* stored extent of an operand: rows x ld with the last row only `cols` long */
static int64_t extent(int64_t rows, int64_t cols, int64_t ld) { return rows == 0 ? 0 : (rows - 1) * ld + cols; }

static double *doubles(int64_t n, unsigned seed)
{
    double *p = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i) p[i] = (double)((int)((seed * 2654435761u + (unsigned)i * 40503u) % 17u) - 8);
    return p;
}

int main(void)
{
    const char tr[2] = {'N', 'T'};
    for (int64_t M = 0; M <= 5; ++M)
        for (int64_t N = 0; N <= 5; N += 1)
            for (int64_t K = 0; K <= 6; K += 3)
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int pad = 0; pad <= 2; pad += 2) {
                            const int64_t ar = a ? K : M, ac = a ? M : K, br = b ? N : K, bc = b ? K : N;
                            const int64_t lda = (ac > 1 ? ac : 1) + pad, ldb = (bc > 1 ? bc : 1) + pad;
                            double *A = doubles(extent(ar, ac, lda), 1), *B = doubles(extent(br, bc, ldb), 2);
                            double *C0 = doubles(extent(M, N, N + pad), 3);
                            double *C = malloc((size_t)(M * N > 0 ? M * N : 1) * sizeof(double));
                            double *D = malloc((size_t)(M * N > 0 ? M * N : 1) * sizeof(double));
                            CHECK(oracle_gemm(tr[a], tr[b], M, N, K, 1.5, A, lda, B, ldb, 0.0, NULL, 1, C, D, N, 2) == 0);
                            CHECK(oracle_gemm(tr[a], tr[b], M, N, K, -2.0, A, lda, B, ldb, 0.5, C0, N + pad, C, NULL, N, 1) == 0);
                            if (M > 0 && N > 0) {
                                int64_t I[2] = {0, M - 1}, J[2] = {N - 1, 0};
                                double c[2], d[2];
                                CHECK(oracle_gemm_entries(tr[a], tr[b], K, -2.0, A, lda, B, ldb, 0.5, C0, N + pad, 2, I, J, c, d, 2) == 0);
                                CHECK(c[0] == C[N - 1] && c[1] == C[(M - 1) * N]);
                            }
                            free(A); free(B); free(C0); free(C); free(D);
                        }
    /* INT8 with wrap-around alpha/beta */
    for (int64_t M = 1; M <= 4; ++M)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                const int64_t N = 3, K = 5;
                const int64_t lda = a ? M : K, ldb = b ? K : N;
                int8_t *A = malloc((size_t)extent(a ? K : M, lda, lda)), *B = malloc((size_t)extent(b ? N : K, ldb, ldb));
                for (int64_t i = 0; i < extent(a ? K : M, lda, lda); ++i) A[i] = (int8_t)(i * 37 - 128);
                for (int64_t i = 0; i < extent(b ? N : K, ldb, ldb); ++i) B[i] = (int8_t)(i * 53 + 7);
                int32_t *C0 = malloc((size_t)(M * N) * sizeof(int32_t)), *C = malloc((size_t)(M * N) * sizeof(int32_t));
                for (int64_t i = 0; i < M * N; ++i) C0[i] = (int32_t)(i * 1000003);
                CHECK(oracle_gemm_i8(tr[a], tr[b], M, N, K, 2147483647, A, lda, B, ldb, -2147483647 - 1, C0, N, C, N, 2) == 0);
                CHECK(oracle_gemm_i8(tr[a], tr[b], M, N, K, 3, A, lda, B, ldb, 0, NULL, 1, C, N, 1) == 0);
                free(A); free(B); free(C0); free(C);
            }
    /* SYR2K on both triangles and both transposes */
    for (int u = 0; u < 2; ++u)
        for (int t = 0; t < 2; ++t) {
            const int64_t N = 5, K = 4, ld = t ? N : K;
            double *A = doubles(extent(t ? K : N, ld, ld), 4), *B = doubles(extent(t ? K : N, ld, ld), 5);
            double *C = doubles(N * N, 6), *D = malloc((size_t)(N * N) * sizeof(double));
            CHECK(oracle_syr2k(u ? 'U' : 'L', tr[t], N, K, 1.5, A, ld, B, ld, 0.5, C, N, D, 2) == 0);
            free(A); free(B); free(C); free(D);
        }
    /* conversions on special values, ragged FP8 tiles */
    const double special[] = {0.0, -0.0, 1.0, -1.5, 65504.0, 65520.0, 1e-8, -1e-45, 448.0, 464.0, 1e30,
                              INFINITY, -INFINITY, NAN, 3.0e38, 1.1754943508222875e-38};
    const int ns = (int)(sizeof(special) / sizeof(special[0]));
    double hi[16], lo[16], h16[16];
    oracle_bf16_split(ns, special, hi, lo);
    oracle_fp16_round(ns, special, h16);
    for (int i = 0; i < ns; ++i) {
        (void)oracle_round_to_bits(special[i], 8, -126);
        const double v = oracle_e4m3_value(special[i]);   /* round (saturating), then encode */
        CHECK(isnan(v) || oracle_e4m3_decode(oracle_e4m3_encode(v)) == v);
        if (isfinite(special[i])) (void)oracle_tile_scale(fabs(special[i]));
    }
    for (int b = 0; b < 256; ++b) (void)oracle_e4m3_decode((unsigned char)b);
    {
        const int64_t rows = 130, cols = 257, ldx = 260, tile = 128;
        double *X = doubles(extent(rows, cols, ldx), 7);
        uint8_t *q = malloc((size_t)(rows * cols));
        float *sc = malloc((size_t)(((rows + tile - 1) / tile) * ((cols + tile - 1) / tile)) * sizeof(float));
        oracle_fp8_quantize(rows, cols, X, ldx, tile, q, sc);
        free(X); free(q); free(sc);
    }
    if (failures) fprintf(stderr, "%d failures\n", failures);
    return failures ? 1 : 0;
}
