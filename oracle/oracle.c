/*
 * oracle.c -- plain, slow, FP64 reference for the layered GEMM library.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file; only the tests, the package smoke check and the benchmark's
 * CPU-baseline leg do. It shares no code, header, table or constant with the
 * GPU library.
 *
 * What it computes (Kuzma et al., "Fast Matrix Multiplication via
 * Compiler-only Layered Data Reorganization and Intrinsic Lowering", SPE 2023):
 *
 *   gemm     The GEMM definition the paper implements (Section 3, Algorithm 1
 *            and the prose after it: C is scaled by beta once and the product
 *            of A and B, scaled by alpha, is added; lda/ldb/ldc are the row
 *            strides of the stored matrices).  Written as the textbook
 *            triple loop: every C[i][j] is one dot product over k in
 *            ascending order, in FP64.  FP32 inputs widen exactly to FP64 and
 *            every FP32 x FP32 product is exact in FP64.
 *            Readings where the paper is silent (BLAS conventions):
 *              - beta == 0: C0 is not read (NaN in C0 does not propagate);
 *              - alpha == 0 or K == 0: the product is not formed, C = beta*C0.
 *            Alongside C it returns the error denominator
 *              D[i][j] = |alpha| * sum_k |opA[i][k]|*|opB[k][j]| + |beta|*|C0[i][j]|.
 *
 *   round_to_bits
 *            Round to nearest, ties to even, to a binary format with a given
 *            number of significant bits and minimum normal exponent.  Used
 *            for bfloat16 (8 bits, emin -126) and OCP FP8 E4M3 (4 bits,
 *            emin -6).  The paper's Table 1 lists 16-bit and 8-bit operand
 *            types for the matrix engine; the rounding rule itself is the
 *            IEEE default (round to nearest even), which the paper does not
 *            restate.
 *
 *   bf16 split  x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (the
 *            split-operand precision scheme; x - hi is exact in FP64).
 *
 *   fp8 tile quantisation
 *            Per 128x128 tile: s = the smallest power of two with
 *            amax <= 448*s (s = 1 for an all-zero tile), q = E4M3(x/s)
 *            saturated to +-448.
 *
 *   fp16 round
 *            IEEE binary16 round-to-nearest-even (11 significant bits, min
 *            normal 2^-14, subnormals below); a result above the largest
 *            finite value 65504 becomes infinity.  Table 1's 16-bit floating
 *            operand type beside bfloat16.
 *
 *   int8 gemm
 *            Table 1's 8-bit integer operands: C = alpha*op(A)*op(B) + beta*C0
 *            with int8 A and B and int32 C, alpha and beta.  The products are
 *            summed exactly (int64), and alpha*sum + beta*C0 is reduced
 *            modulo 2^32 into the int32 range (two's-complement wrap-around),
 *            the reading taken for integer overflow, which the paper does not
 *            discuss.  Same BLAS quick returns as gemm.
 *
 *   syr2k    The paper's worked extension of the macro level to another BLAS
 *            kernel (Section 5.1): one triangle of
 *              C = alpha*A*B^T + alpha*B*A^T + beta*C   (trans 'N', A, B N x K)
 *              C = alpha*A^T*B + alpha*B^T*A + beta*C   (trans 'T', A, B K x N)
 *            C symmetric, only the lower (uplo 'L': i >= j) or upper ('U':
 *            i <= j) triangle read and written, BLAS conventions otherwise.
 *            Written as the two dot products of the definition per entry.
 *
 * Build: gcc -O2 -fopenmp -fno-fast-math -ffp-contract=off -shared -fPIC.
 * With contraction off, every multiply and add is a separately rounded IEEE
 * FP64 operation, so results do not depend on the compiler or thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <omp.h>

/* ---------------------------------------------------------------- GEMM -- */

/* op(A)[i][k]: 'N' means A is stored M x K (row stride lda), 'T' means K x M. */
static double op_a(const double *A, int64_t lda, int ta, int64_t i, int64_t k)
{
    return ta ? A[k * lda + i] : A[i * lda + k];
}

/* op(B)[k][j]: 'N' means B is stored K x N (row stride ldb), 'T' means N x K. */
static double op_b(const double *B, int64_t ldb, int tb, int64_t k, int64_t j)
{
    return tb ? B[j * ldb + k] : B[k * ldb + j];
}

static int is_trans(char t) { return t == 'T' || t == 't' || t == 'C' || t == 'c'; }

/* One output entry: the dot product over k in ascending order, then alpha and beta. */
static void gemm_entry(int ta, int tb, int64_t K, double alpha,
                       const double *A, int64_t lda, const double *B, int64_t ldb,
                       double beta, const double *C0, int64_t ldc0,
                       int64_t i, int64_t j, double *c_out, double *d_out)
{
    double sum = 0.0, asum = 0.0;
    if (alpha != 0.0) {
        for (int64_t k = 0; k < K; ++k) {
            double a = op_a(A, lda, ta, i, k);
            double b = op_b(B, ldb, tb, k, j);
            sum += a * b;
            asum += fabs(a) * fabs(b);
        }
    }
    double c = alpha * sum;
    double d = fabs(alpha) * asum;
    if (beta != 0.0) {
        double c0 = C0[i * ldc0 + j];
        c += beta * c0;
        d += fabs(beta) * fabs(c0);
    }
    *c_out = c;
    *d_out = d;
}

/*
 * Full GEMM.  C and D are M x N with row stride ldc.  D may be NULL.
 * Returns 0, or -1 for an invalid transpose character.
 */
int oracle_gemm(char transA, char transB, int64_t M, int64_t N, int64_t K,
                double alpha, const double *A, int64_t lda,
                const double *B, int64_t ldb,
                double beta, const double *C0, int64_t ldc0,
                double *C, double *D, int64_t ldc, int nthreads)
{
    if (!(transA == 'N' || transA == 'n' || is_trans(transA))) return -1;
    if (!(transB == 'N' || transB == 'n' || is_trans(transB))) return -1;
    int ta = is_trans(transA), tb = is_trans(transB);
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            double c, d;
            gemm_entry(ta, tb, K, alpha, A, lda, B, ldb, beta, C0, ldc0, i, j, &c, &d);
            C[i * ldc + j] = c;
            if (D) D[i * ldc + j] = d;
        }
    }
    return 0;
}

/* The same definition at a list of (I[s], J[s]) positions only. */
int oracle_gemm_entries(char transA, char transB, int64_t K,
                        double alpha, const double *A, int64_t lda,
                        const double *B, int64_t ldb,
                        double beta, const double *C0, int64_t ldc0,
                        int64_t count, const int64_t *I, const int64_t *J,
                        double *C, double *D, int nthreads)
{
    if (!(transA == 'N' || transA == 'n' || is_trans(transA))) return -1;
    if (!(transB == 'N' || transB == 'n' || is_trans(transB))) return -1;
    int ta = is_trans(transA), tb = is_trans(transB);
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 16)
    for (int64_t s = 0; s < count; ++s) {
        double c, d;
        gemm_entry(ta, tb, K, alpha, A, lda, B, ldb, beta, C0, ldc0, I[s], J[s], &c, &d);
        C[s] = c;
        if (D) D[s] = d;
    }
    return 0;
}

/* ------------------------------------------------------------ rounding -- */

/*
 * Nearest value with `bits` significant bits (implicit bit included) whose
 * exponent is at least `emin` (below that the quantum is fixed, giving
 * subnormals), ties to even.  x / quantum is exact (power-of-two scaling),
 * and nearbyint() in the default rounding mode rounds half to even.
 * Overflow is left to the caller.
 */
double oracle_round_to_bits(double x, int bits, int emin)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);               /* |x| = f * 2^e, f in [0.5, 1): leading bit 2^(e-1) */
    int lead = e - 1;
    if (lead < emin) lead = emin;
    double quantum = ldexp(1.0, lead - (bits - 1));
    return nearbyint(x / quantum) * quantum;
}

/* bfloat16 round-to-nearest-even of a value held in a double; overflow -> inf. */
static double to_bf16(double x)
{
    double r = oracle_round_to_bits(x, 8, -126);
    if (isfinite(r) && fabs(r) >= ldexp(1.0, 128)) r = copysign(INFINITY, r);
    return r;
}

/* Split x into hi = bf16(x) and lo = bf16(x - hi). */
void oracle_bf16_split(int64_t n, const double *x, double *hi, double *lo)
{
    for (int64_t t = 0; t < n; ++t) {
        double h = to_bf16(x[t]);
        hi[t] = h;
        lo[t] = isfinite(h) ? to_bf16(x[t] - h) : 0.0;
    }
}

/* bfloat16 rounding of each element. */
void oracle_bf16_round(int64_t n, const double *x, double *out)
{
    for (int64_t t = 0; t < n; ++t) out[t] = to_bf16(x[t]);
}

/* binary16 round-to-nearest-even of a value held in a double; overflow -> inf. */
static double to_fp16(double x)
{
    double r = oracle_round_to_bits(x, 11, -14);
    if (isfinite(r) && fabs(r) > 65504.0) r = copysign(INFINITY, r);
    return r;
}

/* binary16 rounding of each element. */
void oracle_fp16_round(int64_t n, const double *x, double *out)
{
    for (int64_t t = 0; t < n; ++t) out[t] = to_fp16(x[t]);
}

/* ------------------------------------------------------------- FP8 E4M3 -- */

/* OCP E4M3 ("fn"): 1 sign, 4 exponent (bias 7), 3 mantissa bits, max 448,
 * min normal 2^-6, no infinities, NaN = S.1111.111. */
#define E4M3_MAX 448.0

/* Round to E4M3 with saturation to +-448; returns the value. */
double oracle_e4m3_value(double x)
{
    if (isnan(x)) return x;
    double r = oracle_round_to_bits(x, 4, -6);
    if (r > E4M3_MAX) r = E4M3_MAX;
    if (r < -E4M3_MAX) r = -E4M3_MAX;
    return r;
}

/* Encode an exactly representable E4M3 value (or NaN) as its byte. */
uint8_t oracle_e4m3_encode(double v)
{
    if (isnan(v)) return 0x7F;
    uint8_t sign = signbit(v) ? 0x80 : 0x00;
    double a = fabs(v);
    if (a == 0.0) return sign;
    int e;
    frexp(a, &e);
    int lead = e - 1;                       /* a in [2^lead, 2^(lead+1)) */
    if (lead < -6) {                        /* subnormal: a = m * 2^-9 */
        int m = (int)(a / ldexp(1.0, -9));
        return (uint8_t)(sign | m);
    }
    int m = (int)(a / ldexp(1.0, lead - 3)) - 8;   /* 3 mantissa bits */
    return (uint8_t)(sign | ((lead + 7) << 3) | m);
}

/* Decode an E4M3 byte to its value. */
double oracle_e4m3_decode(uint8_t b)
{
    int sign = b >> 7, ex = (b >> 3) & 0xF, m = b & 7;
    double v;
    if (ex == 0xF && m == 7) return NAN;
    if (ex == 0) v = m * ldexp(1.0, -9);
    else v = (8 + m) * ldexp(1.0, ex - 7 - 3);
    return sign ? -v : v;
}

/* The smallest power of two s with amax <= 448 * s; 1 for amax == 0. */
double oracle_tile_scale(double amax)
{
    if (amax == 0.0 || !isfinite(amax)) return 1.0;
    int e;
    frexp(amax, &e);
    double s = ldexp(1.0, e - 11);          /* 448*s < amax here */
    while (!(amax <= E4M3_MAX * s)) s *= 2.0;
    return s;
}

/*
 * Quantise a logical rows x cols matrix X (row stride ldx) in tiles of
 * tile x tile.  q receives rows x cols E4M3 bytes (row stride cols);
 * scales receives ceil(rows/tile) x ceil(cols/tile) floats (row-major).
 * Partial tiles at the edges use their own amax.
 */
void oracle_fp8_quantize(int64_t rows, int64_t cols, const double *X, int64_t ldx,
                         int64_t tile, uint8_t *q, float *scales)
{
    int64_t tr = (rows + tile - 1) / tile, tc = (cols + tile - 1) / tile;
    for (int64_t bi = 0; bi < tr; ++bi) {
        for (int64_t bj = 0; bj < tc; ++bj) {
            int64_t i1 = (bi + 1) * tile < rows ? (bi + 1) * tile : rows;
            int64_t j1 = (bj + 1) * tile < cols ? (bj + 1) * tile : cols;
            double amax = 0.0;
            for (int64_t i = bi * tile; i < i1; ++i)
                for (int64_t j = bj * tile; j < j1; ++j)
                    if (fabs(X[i * ldx + j]) > amax) amax = fabs(X[i * ldx + j]);
            double s = oracle_tile_scale(amax);
            scales[bi * tc + bj] = (float)s;
            for (int64_t i = bi * tile; i < i1; ++i)
                for (int64_t j = bj * tile; j < j1; ++j)
                    q[i * cols + j] = oracle_e4m3_encode(oracle_e4m3_value(X[i * ldx + j] / s));
        }
    }
}

/* --------------------------------------------------------------- INT8 -- */

/* Reduce an int64 modulo 2^32 into [-2^31, 2^31) (two's complement). */
static int32_t wrap32(int64_t v)
{
    return (int32_t)(uint32_t)(uint64_t)v;
}

/*
 * C[i][j] = wrap32(alpha * sum_k opA[i][k]*opB[k][j] + beta * C0[i][j]) for
 * int8 A, B (stored as for gemm) and int32 C0 / C (row stride ldc).  The sum
 * is exact in int64 for K < 2^49.  beta == 0: C0 not read; alpha == 0 or
 * K == 0: C = wrap32(beta * C0).
 */
int oracle_gemm_i8(char transA, char transB, int64_t M, int64_t N, int64_t K, int32_t alpha,
                   const int8_t *A, int64_t lda, const int8_t *B, int64_t ldb, int32_t beta,
                   const int32_t *C0, int64_t ldc0, int32_t *C, int64_t ldc, int threads)
{
    int ta = is_trans(transA), tb = is_trans(transB);
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            int64_t acc = 0;
            if (alpha != 0)
                for (int64_t k = 0; k < K; ++k) {
                    int64_t a = ta ? A[k * lda + i] : A[i * lda + k];
                    int64_t b = tb ? B[j * ldb + k] : B[k * ldb + j];
                    acc += a * b;
                }
            int64_t v = (int64_t)alpha * acc;
            if (beta != 0) v += (int64_t)beta * C0[i * ldc0 + j];
            C[i * ldc + j] = wrap32(v);
        }
    }
    return 0;
}

/* -------------------------------------------------------------- SYR2K -- */

/*
 * One triangle of C = alpha*(X*Y^T + Y*X^T) + beta*C in place (C row-major,
 * N x N, row stride ldc), with X = A, Y = B as N x K matrices when trans is
 * 'N' (element (i, k) at A[i*lda + k]) or as the transposes of the stored
 * K x N matrices when trans is 'T' (element (i, k) at A[k*lda + i]).
 * D (row stride N) receives the error denominator
 *   |alpha| * sum_k (|x_ik||y_jk| + |y_ik||x_jk|) + |beta||c_ij|
 * on the triangle.  Entries outside the triangle are not touched.
 */
int oracle_syr2k(char uplo, char trans, int64_t N, int64_t K, double alpha, const double *A,
                 int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                 double *D, int threads)
{
    int lower = (uplo == 'L' || uplo == 'l');
    int tr = is_trans(trans);
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < N; ++i) {
        int64_t j0 = lower ? 0 : i, j1 = lower ? i + 1 : N;
        for (int64_t j = j0; j < j1; ++j) {
            double s1 = 0.0, s2 = 0.0, d = 0.0;
            if (alpha != 0.0) {
                for (int64_t k = 0; k < K; ++k) {
                    double xi = tr ? A[k * lda + i] : A[i * lda + k];
                    double yj = tr ? B[k * ldb + j] : B[j * ldb + k];
                    s1 += xi * yj;
                    d += fabs(xi) * fabs(yj);
                }
                for (int64_t k = 0; k < K; ++k) {
                    double yi = tr ? B[k * ldb + i] : B[i * ldb + k];
                    double xj = tr ? A[k * lda + j] : A[j * lda + k];
                    s2 += yi * xj;
                    d += fabs(yi) * fabs(xj);
                }
            }
            double c = C[i * ldc + j];
            double r = alpha * (s1 + s2);
            double db = fabs(alpha) * d;
            if (beta != 0.0) {
                r += beta * c;
                db += fabs(beta) * fabs(c);
            }
            C[i * ldc + j] = (alpha == 0.0 || K == 0) ? (beta != 0.0 ? beta * c : 0.0) : r;
            if (D) D[i * N + j] = db;
        }
    }
    return 0;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
