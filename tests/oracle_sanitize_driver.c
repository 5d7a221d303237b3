/* Drives every entry point of the CPU oracle (oracle/csk_oracle.c) on small
 * seeded inputs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py): any
 * out-of-bounds access, leak or undefined operation aborts the run.  The
 * results themselves are checked by the other oracle tests. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

uint64_t orc_splitmix64_mix(uint64_t z);
void orc_splitmix64_stream(uint64_t seed, int64_t count, uint64_t* out);
void orc_hash(uint64_t seed, int64_t m, int64_t d, uint32_t* bucket, int8_t* sign);
void orc_bucket_sort(const uint32_t* bucket, int64_t m, int64_t d, uint32_t* perm, uint32_t* ptr);
void orc_sketch_dense_f64(const double* A, int64_t m, int64_t n, int64_t lda, const double* B, int64_t nrhs,
                          int64_t ldb, int64_t d, uint64_t seed, double* At, int64_t ldat, double* Bt, int64_t ldbt);
void orc_sketch_dense_f32(const float* A, int64_t m, int64_t n, int64_t lda, const double* B, int64_t nrhs,
                          int64_t ldb, int64_t d, uint64_t seed, double* At, int64_t ldat, double* Bt, int64_t ldbt);
void orc_sketch_csr_f32(const int64_t* row_ptr, const int32_t* col, const float* val, int64_t m, int64_t n,
                        const double* b, int64_t d, uint64_t seed, double* At, int64_t ldat, double* bt);
void orc_round_f64_to_f32(const double* in, float* out, int64_t count);
void orc_round_f64_to_bf16(const double* in, uint16_t* out, int64_t count);
void orc_round_f64_to_f16(const double* in, uint16_t* out, int64_t count);
void orc_round_f32_to_bf16(const float* in, uint16_t* out, int64_t count);
void orc_round_f32_to_f16(const float* in, uint16_t* out, int64_t count);
void orc_row_norms2(const double* At, int64_t d, int64_t n, int64_t ldat, double* nu2);
int orc_mwrk(const double* At, int64_t d, int64_t n, int64_t ldat, const double* bt, const double* x0,
             const double* xref, double tol, int64_t maxit, int stop_mode, double* x, int64_t* iters,
             int64_t* trace_idx, double* trace_err2, double* trace_r);
int orc_rgrk(const double* At, int64_t d, int64_t n, int64_t ldat, const double* bt, const double* x0,
             const double* xref, double tol, int64_t maxit, int stop_mode, double theta, uint64_t sel_seed,
             double* x, int64_t* iters, int64_t* trace_idx, double* trace_err2, double* trace_r);
int orc_rk(const double* At, int64_t d, int64_t n, int64_t ldat, const double* bt, const double* x0,
           const double* xref, double tol, int64_t maxit, uint64_t sel_seed, double* x, int64_t* iters,
           int64_t* trace_idx, double* trace_err2, double* trace_r);
void orc_uniform_stream(uint64_t sel_seed, int64_t first, int64_t count, double* out);

static uint64_t lcg = 12345u;
static double unif(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * 0x1p-53 - 0.5;
}

int main(void)
{
    enum { M = 300, N = 7, D = 40, K = 60, NNZ = 900 };
    double* A = malloc(sizeof(double) * M * N);
    float* Af = malloc(sizeof(float) * M * N);
    double* xs = malloc(sizeof(double) * N);
    double* b = malloc(sizeof(double) * M);
    for (int i = 0; i < M * N; ++i) { A[i] = unif(); Af[i] = (float)A[i]; }
    for (int c = 0; c < N; ++c) xs[c] = unif();
    for (int i = 0; i < M; ++i) {
        double s = 0.0;
        for (int c = 0; c < N; ++c) s += A[i * N + c] * xs[c];
        b[i] = s;
    }
    uint64_t words[16];
    orc_splitmix64_stream(7, 16, words);
    (void)orc_splitmix64_mix(words[3]);
    uint32_t* bucket = malloc(sizeof(uint32_t) * M);
    int8_t* sign = malloc(M);
    uint32_t* perm = malloc(sizeof(uint32_t) * M);
    uint32_t* ptr = malloc(sizeof(uint32_t) * (D + 1));
    orc_hash(3, M, D, bucket, sign);
    orc_bucket_sort(bucket, M, D, perm, ptr);
    double* At = malloc(sizeof(double) * D * N);
    double* bt = malloc(sizeof(double) * D);
    orc_sketch_dense_f64(A, M, N, N, b, 1, 1, D, 3, At, N, bt, 1);
    orc_sketch_dense_f32(Af, M, N, N, b, 1, 1, D, 3, At, N, bt, 1);
    orc_sketch_dense_f64(A, M, N, N, NULL, 0, 1, D, 3, At, N, NULL, 1);
    /* CSR: three stored entries per row */
    int64_t* rp = malloc(sizeof(int64_t) * (M + 1));
    int32_t* col = malloc(sizeof(int32_t) * NNZ);
    float* val = malloc(sizeof(float) * NNZ);
    for (int i = 0; i <= M; ++i) rp[i] = 3 * (int64_t)i;
    for (int p = 0; p < NNZ; ++p) { col[p] = (p % 3) * 2; val[p] = (float)unif(); }
    orc_sketch_csr_f32(rp, col, val, M, N, b, D, 5, At, N, bt);
    float* f = malloc(sizeof(float) * D * N);
    uint16_t* h = malloc(sizeof(uint16_t) * D * N);
    orc_round_f64_to_f32(At, f, D * N);
    orc_round_f64_to_bf16(At, h, D * N);
    orc_round_f64_to_f16(At, h, D * N);
    orc_round_f32_to_bf16(f, h, D * N);
    orc_round_f32_to_f16(f, h, D * N);
    double* nu2 = malloc(sizeof(double) * D);
    orc_row_norms2(At, D, N, N, nu2);
    orc_sketch_dense_f64(A, M, N, N, b, 1, 1, D, 3, At, N, bt, 1);
    double* x = malloc(sizeof(double) * N);
    int64_t iters = 0;
    int64_t* tidx = malloc(sizeof(int64_t) * (K + 1));
    double* terr = malloc(sizeof(double) * (K + 1));
    double* tr = malloc(sizeof(double) * (K + 1));
    int st = 0;
    st |= orc_mwrk(At, D, N, N, bt, NULL, xs, 0.0, K, 0, x, &iters, tidx, terr, tr) > 1;
    st |= orc_mwrk(At, D, N, N, bt, x, NULL, 1e-12, K, 1, x, &iters, NULL, NULL, NULL) > 1;
    st |= orc_rgrk(At, D, N, N, bt, NULL, xs, 0.0, K, 0, 0.5, 9, x, &iters, tidx, terr, tr) > 1;
    st |= orc_rgrk(At, D, N, N, bt, NULL, NULL, 1e-12, K, 1, 0.0, 9, x, &iters, NULL, NULL, NULL) > 1;
    st |= orc_rk(At, D, N, N, bt, NULL, xs, 0.0, K, 9, x, &iters, tidx, terr, tr) > 1;
    double u[32];
    orc_uniform_stream(4, 100, 32, u);
    free(A); free(Af); free(xs); free(b); free(bucket); free(sign); free(perm); free(ptr); free(At); free(bt);
    free(rp); free(col); free(val); free(f); free(h); free(nu2); free(x); free(tidx); free(terr); free(tr);
    if (st) { printf("unexpected status\n"); return 1; }
    printf("ok\n");
    return 0;
}
