/*
 * csk_oracle.c -- plain, slow, sequential FP64 CPU oracle for the count
 * sketch Kaczmarz (CSK) method of Zhang & Li, "A Count Sketch Kaczmarz
 * Method For Solving Large Overdetermined Linear Systems" (arXiv 2004.02480).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or constant generator with
 * the HIP library; the two are written independently from the paper (and,
 * for the hash, from the published definition of SplitMix64).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math), so
 * every floating-point operation below is one IEEE-754 binary64 operation in
 * the order written.  Two loops may run on several threads (orc_set_threads;
 * one thread unless asked): the sketch over ranges of buckets and the
 * residual of the MWRK loop over rows.  Each thread still computes whole
 * entries in the written order (a bucket entry's sum over ascending rows, a
 * residual's sum over ascending columns), so every result is bitwise the
 * single-thread one.
 *
 * What each function follows:
 *   orc_hash             Definition 1 (count sketch transform S = Phi D): the
 *                        map h:[m]->[d] and the diagonal signs D.  The paper
 *                        only fixes their distribution; the concrete generator
 *                        is the SplitMix64 output function (Steele, Lea &
 *                        Flood, OOPSLA 2014) applied to a counter.
 *   orc_bucket_sort      the stable grouping of rows by h(i) (the nonzero
 *                        pattern of Phi, one entry per column).
 *   orc_sketch_*         Algorithm 1, "Initialize": At = S A, bt = S b, summed
 *                        per sketch row in ascending original row index.
 *   orc_row_norms2       the denominators ||At^(i)||_2^2 of Algorithm 1.
 *   orc_mwrk             the loop of Algorithm 1 (greedy selection of the row
 *                        with the largest weighted residual, then projection
 *                        onto that row), with the stopping rule of Section 3.
 *   orc_rgrk, orc_rk     the randomized selection rules the introduction puts
 *                        Algorithm 1's loop among (relaxed greedy randomized
 *                        Kaczmarz, with greedy randomized Kaczmarz at
 *                        theta = 1/2; randomized Kaczmarz), compared against
 *                        in Section 3; written from their published
 *                        definitions (Bai & Wu; Strohmer & Vershynin).
 *   orc_round_*          precision reduction of a finished FP64 sketch (not in
 *                        the paper; round-to-nearest-even, two steps).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - indices are 0-based;
 *   - rows of At whose norm is zero (empty buckets) are excluded from the
 *     argmax; if every row is zero the solve reports DEGENERATE;
 *   - argmax ties go to the lowest index;
 *   - the stopping test is evaluated at the top of iteration k, before the
 *     k-th projection, so the iteration count equals the projections applied.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Status values returned by orc_mwrk.  They carry the same meaning (and, by
 * deliberate interface agreement, the same numbers) as the library's status
 * codes, but are defined here on their own. */
#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_ERR_INVALID_ARG 2
#define ORC_ERR_NONFINITE 6
#define ORC_ERR_DEGENERATE 7

#define ORC_STOP_REL_ERR 0
#define ORC_STOP_REL_RESID 1

/* ------------------------------------------------------------------------ */
/* Definition 1: the random map h and the random signs D.                    */
/* ------------------------------------------------------------------------ */

/* SplitMix64 output function, from its published definition: two
 * xor-shift-multiply rounds and a final xor-shift on the 64-bit state. */
uint64_t orc_splitmix64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* The SplitMix64 generator advances its state by the odd constant gamma
 * (the 64-bit golden ratio) before every output.  The i-th output (0-based)
 * of a generator seeded with `seed` is therefore mix(seed + (i+1)*gamma);
 * that word is the random draw attached to input row i. */
static uint64_t orc_row_word(uint64_t seed, uint64_t i)
{
    const uint64_t gamma = 0x9E3779B97F4A7C15ULL;
    return orc_splitmix64_mix(seed + (i + 1u) * gamma);
}

/* Bucket h(i) in [0,d): the high 32 bits of the word, scaled to [0,d) by a
 * 32x32->64 multiply and a shift (each bucket receives either floor or ceil
 * of 2^32/d of the 2^32 high-word values, so h(i)=j has probability 1/d up
 * to d/2^32).  Sign D_ii: -1 if the low bit of the word is set, else +1. */
static uint32_t orc_bucket_of(uint64_t w, uint64_t d)
{
    return (uint32_t)(((w >> 32) * d) >> 32);
}

static int orc_sign_of(uint64_t w)
{
    return (w & 1u) ? -1 : 1;
}

/* h and D for rows 0..m-1. */
void orc_hash(uint64_t seed, int64_t m, int64_t d, uint32_t* bucket, int8_t* sign)
{
    for (int64_t i = 0; i < m; ++i) {
        uint64_t w = orc_row_word(seed, (uint64_t)i);
        if (bucket) bucket[i] = orc_bucket_of(w, (uint64_t)d);
        if (sign) sign[i] = (int8_t)orc_sign_of(w);
    }
}

/* Plain sequential SplitMix64 stream (state += gamma; output mix(state)),
 * used by the tests to check that the counter form above is that stream. */
void orc_splitmix64_stream(uint64_t seed, int64_t count, uint64_t* out)
{
    uint64_t state = seed;
    for (int64_t k = 0; k < count; ++k) {
        state += 0x9E3779B97F4A7C15ULL;
        out[k] = orc_splitmix64_mix(state);
    }
}

/* Stable counting sort of rows by bucket: ptr[j] is the first slot of bucket
 * j (ptr[d] = m) and perm[ptr[j] .. ptr[j+1]) lists the rows with h(i)=j in
 * ascending i. */
void orc_bucket_sort(const uint32_t* bucket, int64_t m, int64_t d, uint32_t* perm, uint32_t* ptr)
{
    uint32_t* next = (uint32_t*)calloc((size_t)d + 1, sizeof(uint32_t));
    for (int64_t j = 0; j <= d; ++j) ptr[j] = 0;
    for (int64_t i = 0; i < m; ++i) ptr[bucket[i] + 1] += 1;
    for (int64_t j = 0; j < d; ++j) ptr[j + 1] += ptr[j];
    for (int64_t j = 0; j < d; ++j) next[j] = ptr[j];
    for (int64_t i = 0; i < m; ++i) perm[next[bucket[i]]++] = (uint32_t)i;
    free(next);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1, Initialize: At = S A and bt = S b.                           */
/* ------------------------------------------------------------------------ */

/* Dense A (row-major, m x n, leading dimension lda), FP64.  Row i of A is
 * added, with sign s(i), into row h(i) of At; rows are visited in ascending
 * i, so each entry of At is the sequential FP64 sum, from +0.0, of the signed
 * entries of its bucket in ascending row order.  B (m x nrhs, leading
 * dimension ldb) is sketched the same way into Bt (d x nrhs).  Either of
 * A/At or B/Bt may be NULL. */
/* The rows of At (and Bt) are split into ranges of buckets, one per loop
 * index g; range g visits every row i in ascending order and adds the rows
 * that land in it.  With one thread this is the plain loop over i. */
#define ORC_SKETCH_RANGES 64

void orc_sketch_dense_f64(const double* A, int64_t m, int64_t n, int64_t lda,
                          const double* B, int64_t nrhs, int64_t ldb,
                          int64_t d, uint64_t seed,
                          double* At, int64_t ldat, double* Bt, int64_t ldbt)
{
    if (At)
        for (int64_t j = 0; j < d; ++j)
            for (int64_t c = 0; c < n; ++c) At[j * ldat + c] = 0.0;
    if (Bt)
        for (int64_t j = 0; j < d; ++j)
            for (int64_t c = 0; c < nrhs; ++c) Bt[j * ldbt + c] = 0.0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < ORC_SKETCH_RANGES; ++g) {
        const int64_t j0 = d * g / ORC_SKETCH_RANGES, j1 = d * (g + 1) / ORC_SKETCH_RANGES;
        for (int64_t i = 0; i < m; ++i) {
            uint64_t w = orc_row_word(seed, (uint64_t)i);
            int64_t h = (int64_t)orc_bucket_of(w, (uint64_t)d);
            if (h < j0 || h >= j1) continue;
            double s = (double)orc_sign_of(w);
            if (A && At)
                for (int64_t c = 0; c < n; ++c) At[h * ldat + c] = At[h * ldat + c] + s * A[i * lda + c];
            if (B && Bt)
                for (int64_t c = 0; c < nrhs; ++c) Bt[h * ldbt + c] = Bt[h * ldbt + c] + s * B[i * ldb + c];
        }
    }
}

/* Same, with an FP32 A: each entry is widened exactly to FP64 first. */
void orc_sketch_dense_f32(const float* A, int64_t m, int64_t n, int64_t lda,
                          const double* B, int64_t nrhs, int64_t ldb,
                          int64_t d, uint64_t seed,
                          double* At, int64_t ldat, double* Bt, int64_t ldbt)
{
    if (At)
        for (int64_t j = 0; j < d; ++j)
            for (int64_t c = 0; c < n; ++c) At[j * ldat + c] = 0.0;
    if (Bt)
        for (int64_t j = 0; j < d; ++j)
            for (int64_t c = 0; c < nrhs; ++c) Bt[j * ldbt + c] = 0.0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < ORC_SKETCH_RANGES; ++g) {
        const int64_t j0 = d * g / ORC_SKETCH_RANGES, j1 = d * (g + 1) / ORC_SKETCH_RANGES;
        for (int64_t i = 0; i < m; ++i) {
            uint64_t w = orc_row_word(seed, (uint64_t)i);
            int64_t h = (int64_t)orc_bucket_of(w, (uint64_t)d);
            if (h < j0 || h >= j1) continue;
            double s = (double)orc_sign_of(w);
            if (A && At)
                for (int64_t c = 0; c < n; ++c)
                    At[h * ldat + c] = At[h * ldat + c] + s * (double)A[i * lda + c];
            if (B && Bt)
                for (int64_t c = 0; c < nrhs; ++c) Bt[h * ldbt + c] = Bt[h * ldbt + c] + s * B[i * ldb + c];
        }
    }
}

/* CSR A (row_ptr[m+1], col[nnz], FP32 values): the same sketch, touching only
 * stored entries.  Within a row the column indices are distinct, so every
 * (bucket, column) entry still receives its terms in ascending row order; the
 * skipped zeros would only have added signed zeros, which change no sum. */
void orc_sketch_csr_f32(const int64_t* row_ptr, const int32_t* col, const float* val,
                        int64_t m, int64_t n, const double* b, int64_t d, uint64_t seed,
                        double* At, int64_t ldat, double* bt)
{
    for (int64_t j = 0; j < d; ++j) {
        for (int64_t c = 0; c < n; ++c) At[j * ldat + c] = 0.0;
        if (bt) bt[j] = 0.0;
    }
    for (int64_t i = 0; i < m; ++i) {
        uint64_t w = orc_row_word(seed, (uint64_t)i);
        int64_t h = (int64_t)orc_bucket_of(w, (uint64_t)d);
        double s = (double)orc_sign_of(w);
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int64_t c = col[p];
            At[h * ldat + c] = At[h * ldat + c] + s * (double)val[p];
        }
        if (b && bt) bt[h] = bt[h] + s * b[i];
    }
}

/* The sketched residual through the original system: S (b - A x) for a CSR
 * A (Definition 1's S applied to the residual of A x = b).  It equals
 * bt - At x of the sketch in exact arithmetic, since S is linear; the mixed
 * precision loop on the sketch of a sparse A can take its exact residual
 * this way.  y_i = b_i - (sum over row i's stored entries, in stored order
 * from zero, of val * x_col); r_h(i) accumulates D_ii y_i in ascending row
 * order. */
void orc_sketch_residual_csr(const int64_t* row_ptr, const int32_t* col, const float* val, int64_t m,
                             const double* b, const double* x, int64_t d, uint64_t seed, double* r)
{
    for (int64_t j = 0; j < d; ++j) r[j] = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) s = s + (double)val[p] * x[col[p]];
        double y = b[i] - s;
        uint64_t w = orc_row_word(seed, (uint64_t)i);
        int64_t h = (int64_t)orc_bucket_of(w, (uint64_t)d);
        r[h] = r[h] + (double)orc_sign_of(w) * y;
    }
}

/* ------------------------------------------------------------------------ */
/* Precision reduction of the finished sketch (not part of the paper).       */
/* ------------------------------------------------------------------------ */

/* FP64 -> FP32: the C conversion, which under the default rounding mode is
 * IEEE-754 round-to-nearest-even (C99 Annex F). */
void orc_round_f64_to_f32(const double* in, float* out, int64_t count)
{
    for (int64_t k = 0; k < count; ++k) out[k] = (float)in[k];
}

static uint32_t orc_f32_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    return u;
}

/* FP32 -> bfloat16 (1-8-7), round to nearest, ties to even, on the bit
 * pattern: bfloat16 is the top half of the FP32 encoding, so add just under
 * half an ulp of the kept part (plus one if the kept part is odd) and drop
 * the low 16 bits.  A carry out of the mantissa moves into the exponent,
 * which is the correct rounding, including overflow to infinity.  NaNs stay
 * NaN (quiet bit forced). */
static uint16_t orc_f32_to_bf16(float f)
{
    uint32_t u = orc_f32_bits(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x0040u);
    uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

/* FP32 -> IEEE binary16 (1-5-10), round to nearest, ties to even, including
 * gradual underflow.  binary16 normals have unbiased exponent -14..15; the
 * smallest subnormal is 2^-24; the largest finite value is 65504 and every
 * value from 65520 up rounds to infinity. */
static uint16_t orc_f32_to_f16(float f)
{
    uint32_t u = orc_f32_bits(f);
    uint16_t sign = (uint16_t)((u >> 16) & 0x8000u);
    uint32_t a = u & 0x7FFFFFFFu;
    if (a > 0x7F800000u) return (uint16_t)(sign | 0x7E00u);          /* NaN */
    if (a >= 0x477FF000u) return (uint16_t)(sign | 0x7C00u);         /* >= 65520: inf */
    int32_t e = (int32_t)(a >> 23) - 127;                            /* unbiased exponent */
    uint32_t mant = a & 0x7FFFFFu;
    if (e >= -14) {                                                  /* binary16 normal */
        uint32_t h = ((uint32_t)(e + 15) << 10) | (mant >> 13);
        uint32_t rem = mant & 0x1FFFu;
        if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) h += 1u;  /* carry is correct */
        return (uint16_t)(sign | h);
    }
    if (e < -25) return sign;                                        /* below half of 2^-24 */
    /* value = M * 2^(e-23) with the implicit bit; in units of 2^-24 that is
     * M * 2^(e+1), i.e. M shifted right by -(e+1) (14..24 places). */
    uint32_t M = mant | 0x800000u;
    uint32_t shift = (uint32_t)(-(e + 1));
    uint32_t q = M >> shift;
    uint32_t rem = M & ((1u << shift) - 1u);
    uint32_t half = 1u << (shift - 1u);
    if (rem > half || (rem == half && (q & 1u))) q += 1u;
    return (uint16_t)(sign | q);
}

/* FP64 -> FP32 -> bfloat16 and FP64 -> FP32 -> binary16 (two RNE steps). */
void orc_round_f64_to_bf16(const double* in, uint16_t* out, int64_t count)
{
    for (int64_t k = 0; k < count; ++k) out[k] = orc_f32_to_bf16((float)in[k]);
}

void orc_round_f64_to_f16(const double* in, uint16_t* out, int64_t count)
{
    for (int64_t k = 0; k < count; ++k) out[k] = orc_f32_to_f16((float)in[k]);
}

void orc_round_f32_to_bf16(const float* in, uint16_t* out, int64_t count)
{
    for (int64_t k = 0; k < count; ++k) out[k] = orc_f32_to_bf16(in[k]);
}

void orc_round_f32_to_f16(const float* in, uint16_t* out, int64_t count)
{
    for (int64_t k = 0; k < count; ++k) out[k] = orc_f32_to_f16(in[k]);
}

/* Threads for the two parallel loops (values < 1 mean 1); returns the
 * count in effect (1 when built without OpenMP). */
int orc_set_threads(int t)
{
#ifdef _OPENMP
    omp_set_num_threads(t < 1 ? 1 : t);
    return omp_get_max_threads();
#else
    (void)t;
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1, loop.                                                        */
/* ------------------------------------------------------------------------ */

/* nu2[i] = ||At^(i)||_2^2, summed over columns in ascending order. */
void orc_row_norms2(const double* At, int64_t d, int64_t n, int64_t ldat, double* nu2)
{
    for (int64_t i = 0; i < d; ++i) {
        double s = 0.0;
        for (int64_t c = 0; c < n; ++c) s = s + At[i * ldat + c] * At[i * ldat + c];
        nu2[i] = s;
    }
}

/* Maximal weighted residual Kaczmarz on (At, bt), d x n, from x0 (NULL: the
 * zero vector, as in the experiments of Section 3).
 *
 * Iteration k:
 *   1. stopping test on x_k:
 *        stop_mode REL_ERR:   RES = ||x_k - xref||^2 / ||xref||^2 <= tol^2
 *                             (Section 3's relative solution error; tol is on
 *                             the unsquared relative error; if ||xref|| = 0
 *                             the absolute ||x_k||^2 <= tol^2 is used);
 *        stop_mode REL_RESID: ||bt - At x_k||^2 <= tol^2 ||bt||^2;
 *      then, if k == maxit, stop with NOT_CONVERGED;
 *   2. r_i = bt_i - At^(i) x_k, each dot product summed in column order;
 *   3. i_k = the lowest index attaining max |r_i| / ||At^(i)|| over rows with
 *      nonzero norm (a NaN or infinite weighted residual -> NONFINITE; no
 *      row with nonzero norm -> DEGENERATE);
 *   4. x_{k+1} = x_k + (r_{i_k} / ||At^(i_k)||^2) At^(i_k)^T.
 *
 * Outputs: x (n), *iters = number of projections applied.  Optional traces
 * (NULL to skip), each with room for maxit+1 entries:
 *   trace_idx[k]   = i_k,
 *   trace_err2[k]  = ||x_k - xref||^2 (needs xref),
 *   trace_r[k]     = r_{i_k}. */
int orc_mwrk(const double* At, int64_t d, int64_t n, int64_t ldat, const double* bt,
             const double* x0, const double* xref, double tol, int64_t maxit, int stop_mode,
             double* x, int64_t* iters, int64_t* trace_idx, double* trace_err2, double* trace_r)
{
    if (d < 1 || n < 1 || ldat < n || maxit < 0) return ORC_ERR_INVALID_ARG;
    if (stop_mode == ORC_STOP_REL_ERR && xref == NULL) return ORC_ERR_INVALID_ARG;

    double* nu2 = (double*)malloc(sizeof(double) * (size_t)d);
    double* nu = (double*)malloc(sizeof(double) * (size_t)d);
    double* r = (double*)malloc(sizeof(double) * (size_t)d);
    orc_row_norms2(At, d, n, ldat, nu2);
    for (int64_t i = 0; i < d; ++i) nu[i] = sqrt(nu2[i]);

    for (int64_t c = 0; c < n; ++c) x[c] = x0 ? x0[c] : 0.0;

    double xref2 = 0.0, bt2 = 0.0;
    if (xref)
        for (int64_t c = 0; c < n; ++c) xref2 = xref2 + xref[c] * xref[c];
    for (int64_t i = 0; i < d; ++i) bt2 = bt2 + bt[i] * bt[i];

    int status = ORC_NOT_CONVERGED;
    int64_t k = 0;
    for (;; ++k) {
        double err2 = 0.0;
        if (xref) {
            for (int64_t c = 0; c < n; ++c) {
                double e = x[c] - xref[c];
                err2 = err2 + e * e;
            }
            if (trace_err2) trace_err2[k] = err2;
        }
        /* step 2 (computed before the test so the residual mode can use it) */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < d; ++i) {
            double dot = 0.0;
            for (int64_t c = 0; c < n; ++c) dot = dot + At[i * ldat + c] * x[c];
            r[i] = bt[i] - dot;
        }
        double r2 = 0.0;
        for (int64_t i = 0; i < d; ++i) r2 = r2 + r[i] * r[i];
        /* step 1 */
        if (stop_mode == ORC_STOP_REL_ERR) {
            if (xref2 > 0.0 ? (err2 / xref2 <= tol * tol) : (err2 <= tol * tol)) { status = ORC_OK; break; }
        } else {
            if (r2 <= tol * tol * bt2) { status = ORC_OK; break; }
        }
        if (k == maxit) { status = ORC_NOT_CONVERGED; break; }
        /* step 3 */
        int64_t best = -1;
        double best_score = 0.0;
        int nonfinite = 0;
        for (int64_t i = 0; i < d; ++i) {
            if (!(nu[i] > 0.0)) {
                if (isnan(nu[i])) nonfinite = 1;
                continue;
            }
            double score = fabs(r[i]) / nu[i];
            if (!isfinite(score)) { nonfinite = 1; break; }
            if (best < 0 || score > best_score) { best = i; best_score = score; }
        }
        if (nonfinite) { status = ORC_ERR_NONFINITE; break; }
        if (best < 0) { status = ORC_ERR_DEGENERATE; break; }
        if (trace_idx) trace_idx[k] = best;
        if (trace_r) trace_r[k] = r[best];
        /* step 4 */
        double alpha = r[best] / nu2[best];
        for (int64_t c = 0; c < n; ++c) x[c] = x[c] + alpha * At[best * ldat + c];
    }
    *iters = k;
    free(nu2);
    free(nu);
    free(r);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Randomized row selection: the relaxed greedy randomized Kaczmarz rule     */
/* (Bai & Wu; its parameter theta = 1/2 gives their greedy randomized rule   */
/* and theta = 1 the maximal weighted residual rule of Algorithm 1) and the  */
/* randomized Kaczmarz rule of Strohmer & Vershynin.  The introduction       */
/* places Algorithm 1's loop in this family and Section 3 compares against   */
/* its members.  The stopping test and the projection are those of orc_mwrk; */
/* only the choice of i_k differs, and its random numbers come from a        */
/* SplitMix64 counter stream of the caller's selection seed.                 */
/* ------------------------------------------------------------------------ */

/* The k-th (0-based) uniform of the selection stream: the top 52 bits of the
 * k-th SplitMix64 output plus one half, times 2^-52.  Every operation is
 * exact, and the value lies strictly inside (0, 1). */
static double orc_uniform(uint64_t seed, uint64_t k)
{
    uint64_t w = orc_row_word(seed, k);
    return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

/* Shared by the two rules: the relative-error or residual stop test of
 * orc_mwrk on x_k.  r (d) must hold bt - At x_k when stop_mode is REL_RESID. */
static int orc_stop_met(int stop_mode, double err2, double xref2, double r2, double bt2, double tol)
{
    if (stop_mode == ORC_STOP_REL_ERR)
        return xref2 > 0.0 ? (err2 / xref2 <= tol * tol) : (err2 <= tol * tol);
    return r2 <= tol * tol * bt2;
}

/* Relaxed greedy randomized Kaczmarz on (At, bt), d x n, from x0 (NULL: 0).
 *
 * Iteration k (stop test first, exactly as in orc_mwrk):
 *   1. r_i = bt_i - At^(i) x_k (column order), R = ||r||^2 (row order);
 *      F = ||At||_F^2 = sum of the squared row norms (row order, once);
 *   2. M = max of r_i^2 / ||At^(i)||^2 over rows of nonzero norm (none:
 *      DEGENERATE; a NaN or infinite value: NONFINITE);
 *   3. the working set: rows of nonzero norm with
 *        |r_i|^2 >= eps_k R ||At^(i)||^2,  eps_k = theta M / R + (1 - theta) / F,
 *      tested in the equivalent form r_i^2 / ||At^(i)||^2 >= t_k with
 *      t_k = theta M + (1 - theta) (R / F) (multiply eps_k by R, divide by
 *      the row's squared norm).  In exact arithmetic t_k <= M, because M is
 *      at least R / F, the norm-weighted mean of the scores; t_k is capped at
 *      M so that rounding never empties the set;
 *   4. i_k is drawn from the set with probability r_i^2 over the sum of r_j^2
 *      in the set: with E_i = -log(u_i), u_i the (k d + i)-th uniform of the
 *      selection stream (a unit exponential per row), i_k is the member with
 *      the largest r_i^2 / E_i, the lowest index on ties (the smallest of
 *      independent exponential clocks with rates r_i^2 falls on row i with
 *      probability r_i^2 over their sum; Efraimidis & Spirakis);
 *   5. x_{k+1} = x_k + (r_{i_k} / ||At^(i_k)||^2) At^(i_k)^T.
 * theta must lie in [0, 1].  Traces as in orc_mwrk. */
int orc_rgrk(const double* At, int64_t d, int64_t n, int64_t ldat, const double* bt,
             const double* x0, const double* xref, double tol, int64_t maxit, int stop_mode,
             double theta, uint64_t sel_seed,
             double* x, int64_t* iters, int64_t* trace_idx, double* trace_err2, double* trace_r)
{
    if (d < 1 || n < 1 || ldat < n || maxit < 0) return ORC_ERR_INVALID_ARG;
    if (!(theta >= 0.0 && theta <= 1.0)) return ORC_ERR_INVALID_ARG;
    if (stop_mode == ORC_STOP_REL_ERR && xref == NULL) return ORC_ERR_INVALID_ARG;

    double* nu2 = (double*)malloc(sizeof(double) * (size_t)d);
    double* r = (double*)malloc(sizeof(double) * (size_t)d);
    orc_row_norms2(At, d, n, ldat, nu2);
    double fro2 = 0.0;
    for (int64_t i = 0; i < d; ++i) fro2 = fro2 + nu2[i];

    for (int64_t c = 0; c < n; ++c) x[c] = x0 ? x0[c] : 0.0;
    double xref2 = 0.0, bt2 = 0.0;
    if (xref)
        for (int64_t c = 0; c < n; ++c) xref2 = xref2 + xref[c] * xref[c];
    for (int64_t i = 0; i < d; ++i) bt2 = bt2 + bt[i] * bt[i];

    int status = ORC_NOT_CONVERGED;
    int64_t k = 0;
    for (;; ++k) {
        double err2 = 0.0;
        if (xref) {
            for (int64_t c = 0; c < n; ++c) {
                double e = x[c] - xref[c];
                err2 = err2 + e * e;
            }
            if (trace_err2) trace_err2[k] = err2;
        }
        double r2 = 0.0;
        for (int64_t i = 0; i < d; ++i) {
            double dot = 0.0;
            for (int64_t c = 0; c < n; ++c) dot = dot + At[i * ldat + c] * x[c];
            r[i] = bt[i] - dot;
            r2 = r2 + r[i] * r[i];
        }
        if (orc_stop_met(stop_mode, err2, xref2, r2, bt2, tol)) { status = ORC_OK; break; }
        if (k == maxit) { status = ORC_NOT_CONVERGED; break; }

        /* step 2 */
        int found = 0, nonfinite = 0;
        double M = 0.0;
        for (int64_t i = 0; i < d; ++i) {
            if (!(nu2[i] > 0.0)) {
                if (isnan(nu2[i])) nonfinite = 1;
                continue;
            }
            double s = (r[i] * r[i]) / nu2[i];
            if (!isfinite(s)) { nonfinite = 1; break; }
            if (!found || s > M) M = s;
            found = 1;
        }
        if (nonfinite) { status = ORC_ERR_NONFINITE; break; }
        if (!found) { status = ORC_ERR_DEGENERATE; break; }
        /* step 3 */
        double t = theta * M + (1.0 - theta) * (r2 / fro2);
        if (t > M) t = M;
        /* step 4 */
        int64_t best = -1;
        double best_key = 0.0;
        for (int64_t i = 0; i < d; ++i) {
            if (!(nu2[i] > 0.0)) continue;
            if (!((r[i] * r[i]) / nu2[i] >= t)) continue;
            double e = -log(orc_uniform(sel_seed, (uint64_t)k * (uint64_t)d + (uint64_t)i));
            double key = (r[i] * r[i]) / e;
            if (best < 0 || key > best_key) { best = i; best_key = key; }
        }
        if (trace_idx) trace_idx[k] = best;
        if (trace_r) trace_r[k] = r[best];
        /* step 5 */
        double alpha = r[best] / nu2[best];
        for (int64_t c = 0; c < n; ++c) x[c] = x[c] + alpha * At[best * ldat + c];
    }
    *iters = k;
    free(nu2);
    free(r);
    return status;
}

/* Randomized Kaczmarz on (At, bt): each iteration draws row i with
 * probability ||At^(i)||^2 / ||At||_F^2, independently of x, and projects
 * onto it.  The draw inverts the cumulative distribution: C_i = sum of the
 * squared norms of rows 0..i (in index order, once), t_k = u_k C_{d-1} with
 * u_k the k-th uniform of the selection stream, and i_k the smallest i with
 * C_i > t_k (rows of zero norm never qualify; C_{d-1} = 0: DEGENERATE).
 * Only the selected row's residual r_{i_k} = bt_i - At^(i) x_k is formed, so
 * the stop test is the relative error (stop_mode REL_ERR) alone; the other
 * arguments and the traces are as in orc_mwrk. */
int orc_rk(const double* At, int64_t d, int64_t n, int64_t ldat, const double* bt,
           const double* x0, const double* xref, double tol, int64_t maxit, uint64_t sel_seed,
           double* x, int64_t* iters, int64_t* trace_idx, double* trace_err2, double* trace_r)
{
    if (d < 1 || n < 1 || ldat < n || maxit < 0 || xref == NULL) return ORC_ERR_INVALID_ARG;

    double* nu2 = (double*)malloc(sizeof(double) * (size_t)d);
    double* cum = (double*)malloc(sizeof(double) * (size_t)d);
    orc_row_norms2(At, d, n, ldat, nu2);
    double acc = 0.0;
    for (int64_t i = 0; i < d; ++i) {
        acc = acc + nu2[i];
        cum[i] = acc;
    }
    for (int64_t c = 0; c < n; ++c) x[c] = x0 ? x0[c] : 0.0;
    double xref2 = 0.0;
    for (int64_t c = 0; c < n; ++c) xref2 = xref2 + xref[c] * xref[c];

    int status = ORC_NOT_CONVERGED;
    int64_t k = 0;
    for (;; ++k) {
        double err2 = 0.0;
        for (int64_t c = 0; c < n; ++c) {
            double e = x[c] - xref[c];
            err2 = err2 + e * e;
        }
        if (trace_err2) trace_err2[k] = err2;
        if (orc_stop_met(ORC_STOP_REL_ERR, err2, xref2, 0.0, 0.0, tol)) { status = ORC_OK; break; }
        if (k == maxit) { status = ORC_NOT_CONVERGED; break; }
        if (!isfinite(cum[d - 1])) { status = ORC_ERR_NONFINITE; break; }
        if (!(cum[d - 1] > 0.0)) { status = ORC_ERR_DEGENERATE; break; }
        double t = orc_uniform(sel_seed, (uint64_t)k) * cum[d - 1];
        int64_t i = 0;
        while (!(cum[i] > t)) ++i;  /* terminates: t < cum[d-1] */
        double dot = 0.0;
        for (int64_t c = 0; c < n; ++c) dot = dot + At[i * ldat + c] * x[c];
        double ri = bt[i] - dot;
        if (!isfinite(ri)) { status = ORC_ERR_NONFINITE; break; }
        if (trace_idx) trace_idx[k] = i;
        if (trace_r) trace_r[k] = ri;
        double alpha = ri / nu2[i];
        for (int64_t c = 0; c < n; ++c) x[c] = x[c] + alpha * At[i * ldat + c];
    }
    *iters = k;
    free(nu2);
    free(cum);
    return status;
}

/* The uniforms themselves, for the tests of the draws. */
void orc_uniform_stream(uint64_t sel_seed, int64_t first, int64_t count, double* out)
{
    for (int64_t k = 0; k < count; ++k) out[k] = orc_uniform(sel_seed, (uint64_t)(first + k));
}
