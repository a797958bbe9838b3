// Memory- and UB-checked run of the library's host code (the C ABI's
// argument validation, tuning-table parser, configuration rules, workspace
// and split planning) with AddressSanitizer and UndefinedBehaviorSanitizer.
// Only calls that return before any device work are made, so it runs on a
// machine without a GPU.  Exit status 0 when every result is the documented
// one.
#include <climits>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/mgemm.h"

static int failures = 0;
#define CHECK(cond) do { if (!(cond)) { std::fprintf(stderr, "failed: %s (line %d)\n", #cond, __LINE__); ++failures; } } while (0)

static const float* FA = reinterpret_cast<const float*>(0x1000);   // never dereferenced
static float* FC = reinterpret_cast<float*>(0x2000);

static std::string write_table(const char* name, const char* text)
{
    std::string path = std::string("/tmp/mgemm_asan_") + name;
    FILE* f = std::fopen(path.c_str(), "w");
    std::fputs(text, f);
    std::fclose(f);
    return path;
}

int main()
{
    // --- mg_sgemm / mg_gemm argument validation (first invalid argument wins)
    CHECK(mg_sgemm('X', 'N', 4, 5, 6, 1.f, FA, 6, FA, 5, 0.f, FC, 5, nullptr) == -1);
    CHECK(mg_sgemm('N', 'Q', 4, 5, 6, 1.f, FA, 6, FA, 5, 0.f, FC, 5, nullptr) == -2);
    CHECK(mg_sgemm('N', 'N', -1, 5, 6, 1.f, FA, 6, FA, 5, 0.f, FC, 5, nullptr) == -3);
    CHECK(mg_sgemm('N', 'N', 4, -1, 6, 1.f, FA, 6, FA, 5, 0.f, FC, 5, nullptr) == -4);
    CHECK(mg_sgemm('N', 'N', 4, 5, -1, 1.f, FA, 6, FA, 5, 0.f, FC, 5, nullptr) == -5);
    CHECK(mg_sgemm('N', 'N', 4, 5, 6, 1.f, nullptr, 6, FA, 5, 0.f, FC, 5, nullptr) == -7);
    CHECK(mg_sgemm('T', 'N', 4, 5, 6, 1.f, FA, 3, FA, 5, 0.f, FC, 5, nullptr) == -8);
    CHECK(mg_sgemm('N', 'N', 4, 5, 6, 1.f, FA, INT64_MAX, FA, 5, 0.f, FC, 5, nullptr) == -8);
    CHECK(mg_sgemm('N', 'N', 4, 5, 6, 1.f, FA, 6, nullptr, 5, 0.f, FC, 5, nullptr) == -9);
    CHECK(mg_sgemm('N', 't', 4, 5, 6, 1.f, FA, 6, FA, 5, 0.f, FC, 5, nullptr) == -10);
    CHECK(mg_sgemm('N', 'N', 4, 5, 6, 1.f, FA, 6, FA, 5, 0.f, nullptr, 5, nullptr) == -12);
    CHECK(mg_sgemm('N', 'N', 4, 5, 6, 1.f, FA, 6, FA, 5, 0.f, FC, 4, nullptr) == -13);
    CHECK(mg_sgemm('N', 'N', 0, 5, 6, 1.f, nullptr, 6, FA, 5, 0.f, nullptr, 5, nullptr) == MG_OK);
    CHECK(mg_sgemm('N', 'N', INT64_MAX, 5, 6, 1.f, FA, 6, FA, 5, 0.f, FC, 5, nullptr) != MG_OK);
    CHECK(mg_gemm(99, 'N', 'N', 4, 5, 6, 1.f, FA, 6, FA, 5, 0.f, FC, 5, nullptr, 0, nullptr) == MG_ERR_UNSUPPORTED);
    CHECK(mg_gemm(MG_PATH_FP8_T128, 'N', 'N', 4, 5, 6, 1.f, FA, 6, FA, 5, 0.f, FC, 5, nullptr, 0, nullptr) ==
          MG_ERR_WORKSPACE);
    for (int path = 0; path < 5; ++path)
        CHECK(mg_gemm(path, 'N', 'N', 4, 0, 6, 1.f, FA, 6, FA, 1, 0.f, FC, 1, nullptr, 0, nullptr) == MG_OK);

    // --- INT8 and SYR2K validation
    const int8_t* IA = reinterpret_cast<const int8_t*>(0x1000);
    int32_t* IC = reinterpret_cast<int32_t*>(0x2000);
    CHECK(mg_gemm_i8('N', 'N', 4, 5, 131072, 1, IA, 131072, IA, 5, 0, IC, 5, nullptr, 0, nullptr) == MG_ERR_TOO_LARGE);
    CHECK(mg_gemm_i8('N', 'N', 4, 5, 6, 1, IA, 6, IA, 5, 0, IC, 5, nullptr, 0, nullptr) == MG_ERR_WORKSPACE);
    CHECK(mg_gemm_i8('Z', 'N', 4, 5, 6, 1, IA, 6, IA, 5, 0, IC, 5, nullptr, 0, nullptr) == -1);
    CHECK(mg_syr2k(0, 'X', 'N', 4, 4, 1.f, FA, 4, FA, 4, 0.f, FC, 4, nullptr, 0, nullptr) < 0);
    CHECK(mg_syr2k(0, 'L', 'X', 4, 4, 1.f, FA, 4, FA, 4, 0.f, FC, 4, nullptr, 0, nullptr) < 0);
    CHECK(mg_syr2k(2, 'L', 'N', 4, 4, 1.f, FA, 4, FA, 4, 0.f, FC, 4, nullptr, 0, nullptr) == MG_ERR_UNSUPPORTED);
    CHECK(mg_syr2k(0, 'L', 'N', 0, 4, 1.f, FA, 4, FA, 4, 0.f, FC, 1, nullptr, 0, nullptr) == MG_OK);

    // --- batched validation
    mg_problem p[3] = {};
    for (auto& q : p) {
        q.transA = 'N'; q.transB = 'N'; q.M = 4; q.N = 5; q.K = 6; q.alpha = 1.f; q.beta = 0.f;
        q.A = FA; q.lda = 6; q.B = FA; q.ldb = 5; q.C = FC; q.ldc = 5;
    }
    p[2].ldb = 2;
    int64_t bad = -1;
    CHECK(mg_gemm_batched(0, 3, p, nullptr, 0, nullptr, &bad) == -10 && bad == 2);
    p[2].ldb = 5;
    CHECK(mg_gemm_batched(0, 3, p, nullptr, 0, nullptr, &bad) == MG_ERR_WORKSPACE);
    CHECK(mg_gemm_batched(0, 0, nullptr, nullptr, 0, nullptr, nullptr) == MG_OK);
    CHECK(mg_gemm_batched(0, -1, p, nullptr, 0, nullptr, nullptr) == -2);
    CHECK(mg_gemm_batched(3, 3, p, nullptr, 0, nullptr, nullptr) == MG_ERR_UNSUPPORTED);
    CHECK(mg_gemm_batched_timed(0, 3, p, nullptr, 0, nullptr, nullptr, nullptr, 0, nullptr) == -8);
    CHECK(mg_gemm_batched_workspace_size(0, 1000) >= 1000 * 64);

    // --- tuning tables
    CHECK(mg_load_tuning("/nonexistent/table.txt") == MG_ERR_BAD_TABLE);
    CHECK(mg_load_tuning(write_table("bad1", "0 5 5 5\n").c_str()) == MG_ERR_BAD_TABLE);
    CHECK(mg_load_tuning(write_table("bad2", "0 99 5 5 1\n").c_str()) == MG_ERR_BAD_TABLE);
    CHECK(mg_load_tuning(write_table("bad3", "0 5 5 5 999\n").c_str()) == MG_ERR_BAD_TABLE);
    CHECK(mg_load_tuning(write_table("bad4", "7 5 5 5 1 s\n").c_str()) == MG_ERR_BAD_TABLE);
    CHECK(mg_load_tuning(write_table("bad5", "0 5 5 5 1 q\n").c_str()) == MG_ERR_BAD_TABLE);
    CHECK(mg_load_tuning(write_table("bad9", "0 0 5 5 1 x\n").c_str()) == MG_ERR_BAD_TABLE);
    CHECK(mg_load_tuning(write_table("bad10", "0 5 5 5 1 x 17\n").c_str()) == MG_ERR_BAD_TABLE);
    CHECK(mg_load_tuning(write_table("bad11", "0 9999999999 5 5 1 x 2\n").c_str()) == MG_ERR_BAD_TABLE);
    CHECK(mg_load_tuning(write_table("bad12", "0 5 5 5 1 x y\n").c_str()) == MG_ERR_BAD_TABLE);
    CHECK(mg_load_tuning(write_table("exact", "0 1536 1536 1536 0 x 3\n0 11 11 11 3\n").c_str()) == MG_OK);
    CHECK(mg_tuned_config(0, 1536, 1536, 1536) == 0);
    CHECK(mg_tuned_config(0, 2048, 2048, 2048) == 3);
    CHECK(mg_split_count(0, 1536, 1536, 1536) == 3);
    CHECK(mg_load_tuning(write_table("bad6", "0 -1 5 5 1\n").c_str()) == MG_ERR_BAD_TABLE);
    std::string longline(100000, '7');
    CHECK(mg_load_tuning(write_table("bad8", (longline + "\n").c_str()) .c_str()) == MG_ERR_BAD_TABLE);
    CHECK(mg_load_tuning(write_table("good", "# comment\n\n0 13 13 13 2\n0 13 13 13 3 b\n1 10 10 10 4 s\n").c_str()) == MG_OK);
    CHECK(mg_tuned_config(0, 8192, 8192, 8192) == 2);
    CHECK(mg_batched_config(0, 8192, 8192, 8192) >= 0);
    CHECK(mg_load_tuning(nullptr) == MG_OK);

    // --- rules and plans over ordinary and extreme shapes
    const int64_t dims[] = {0, 1, 7, 64, 255, 256, 1000, 4096, 8192, 65536, INT_MAX, int64_t(INT_MAX) + 1, INT64_MAX};
    for (int path = 0; path < 6; ++path)
        for (int64_t M : dims)
            for (int64_t N : dims)
                for (int64_t K : dims) {
                    (void)mg_tuned_config(path, M, N, K);
                    (void)mg_split_count(path, M, N, K);
                    (void)mg_batched_config(path, M, N, K);
                    (void)mg_gemm_workspace_size(path, 'N', 'T', M, N, K);
                    (void)mg_syr2k_workspace_size(path, M, K);
                    (void)mg_gemm_i8_workspace_size(M, N, K);
                }
    size_t q = 0, s = 0;
    for (int64_t R : dims)
        for (int64_t K : dims) {
            (void)mg_fp8_packed_size(R, K, &q, &s);
            (void)mg_i8_packed_size(R, K, &q);
        }
    CHECK(mg_fp8_packed_size(-1, 5, &q, &s) != MG_OK);

    // --- registry, forcing, strings
    int info[6];
    for (int path = -1; path < 8; ++path) {
        const int n = mg_num_configs(path);
        for (int i = -1; i <= n; ++i) {
            const int st = mg_config_info(path, i, info);
            CHECK((st == MG_OK) == (path >= 0 && i >= 0 && i < n));
            (void)mg_config_packs(path, i);
            (void)mg_config_uses_mfma(path, i);
        }
        (void)mg_force_config(path, 1000);
        (void)mg_force_splits(path, 1000);
    }
    for (int path = 0; path < 6; ++path) {
        mg_force_config(path, -1);
        mg_force_splits(path, -1);
    }
    const int codes[] = {0, -1, -13, -14, -100, -101, -102, -103, -1000, -1001, -1999, INT_MIN, INT_MAX};
    for (int c : codes) CHECK(mg_status_string(c) != nullptr);
    CHECK(mg_bf16_split(nullptr, 5, nullptr, nullptr, nullptr) == -1);
    CHECK(mg_bf16_split(FA, -1, nullptr, nullptr, nullptr) == -2);

    if (failures) std::fprintf(stderr, "%d failures\n", failures);
    return failures ? 1 : 0;
}
