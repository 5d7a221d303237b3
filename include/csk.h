/*
 * csk.h -- C ABI of libcsk, the MI355X (gfx950) implementation of the count
 * sketch Kaczmarz (CSK) method of Zhang & Li, "A Count Sketch Kaczmarz
 * Method For Solving Large Overdetermined Linear Systems" (arXiv 2004.02480).
 *
 * The method (Algorithm 1 of the paper) solves a consistent overdetermined
 * system A x = b, A in R^{m x n}, m >> n (Section 1, eq. (1)) in two steps:
 *   1. Initialize: draw a count sketch transform S = Phi D in R^{d x m}
 *      (Definition 1: a random map h:[m]->[d] and random signs D_ii = +-1)
 *      and form At = S A (d x n) and bt = S b (d);
 *   2. Loop: i_k = argmax_i |bt_i - At^(i) x_k| / ||At^(i)||_2, then
 *      x_{k+1} = x_k + (bt_{i_k} - At^(i_k) x_k) / ||At^(i_k)||^2 At^(i_k)^T,
 *      until the stopping rule of Section 3 holds.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers are DEVICE pointers unless marked (host).  Matrices are
 *    row-major with an explicit leading dimension (elements between row
 *    starts, >= the row length).  Indices are 0-based.
 *  - The caller owns every buffer.  The library allocates no device memory
 *    on these paths: scratch space is the caller's workspace `ws` of
 *    `ws_bytes` bytes (size from the matching *_workspace_size query; the
 *    pointer must be 256-byte aligned).  Nothing is retained past the
 *    stream-ordered work.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call is asynchronous: it validates its arguments on the host,
 *    enqueues kernels on `stream` and returns.  A CSK_ERR_* return from the
 *    call itself means nothing was enqueued (argument errors) or a launch
 *    failed (CSK_ERR_DEVICE).  Outcomes decided on the device (converged,
 *    not converged, non-finite data, degenerate sketch, cancelled) are
 *    written to a csk_solve_result in device memory.
 *  - Calls are reentrant; concurrent calls must use distinct workspaces.
 *  - Determinism: for fixed inputs, sizes and launch configuration every
 *    output is bitwise reproducible run to run.
 *
 * The hash (the concrete random generator behind Definition 1)
 * ------------------------------------------------------------
 * The paper fixes only the distribution of h and D.  This library draws,
 * for input row i (0-based) and a 64-bit seed, the word
 *     w_i = M(seed + (i+1) * 0x9E3779B97F4A7C15)      (mod 2^64)
 * where M is the SplitMix64 output function (Steele, Lea & Flood, OOPSLA
 * 2014): z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27;
 * z *= 0x94D049BB133111EB; z ^= z>>31.  (w_i is the (i+1)-th output of a
 * SplitMix64 generator seeded with `seed`.)  Then
 *     h(i) = ((w_i >> 32) * d) >> 32           (bucket in [0, d))
 *     D_ii = -1 if (w_i & 1) else +1.
 *
 * Sketch summation order (what makes At bit-exact)
 * ------------------------------------------------
 * At[j][c] is the sequential FP64 sum, starting at +0.0, of D_ii * A[i][c]
 * over the rows i with h(i) = j taken in ASCENDING i.  FP32 input is widened
 * exactly first.  Low-precision copies are rounded from that FP64 value in
 * two round-to-nearest-even steps: FP64 -> FP32 -> (BF16 | FP16).
 */
#ifndef CSK_H
#define CSK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
typedef int32_t csk_status;
#define CSK_OK 0               /* converged / call succeeded                  */
#define CSK_NOT_CONVERGED 1    /* maxit projections applied; x is valid       */
#define CSK_ERR_INVALID_ARG 2  /* bad size, pointer, leading dimension, mode  */
#define CSK_ERR_UNSUPPORTED 3  /* dtype or shape combination not built        */
#define CSK_ERR_DEVICE 4       /* a HIP call failed (message: csk_last_error) */
#define CSK_ERR_WORKSPACE 5    /* ws_bytes smaller than the query's answer    */
#define CSK_ERR_NONFINITE 6    /* a weighted residual was NaN or infinite     */
#define CSK_ERR_DEGENERATE 7   /* every row of At has zero norm               */
#define CSK_CANCELLED 8        /* the cancel word became nonzero              */

/* ---- element types ----------------------------------------------------- */
typedef int32_t csk_dtype;
#define CSK_F64 0
#define CSK_F32 1
#define CSK_F16 2   /* IEEE binary16 */
#define CSK_BF16 3  /* bfloat16 (1-8-7) */

/* ---- stopping rules ---------------------------------------------------- */
/* CSK_STOP_REL_ERR: Section 3's relative solution error
 *   RES = ||x_k - x_ref||^2 / ||x_ref||^2 <= tol^2  (tol on the unsquared
 *   relative error; if ||x_ref|| = 0, ||x_k||^2 <= tol^2).  Needs x_ref.
 * CSK_STOP_REL_RESID: ||bt - At x_k||_2 <= tol ||bt||_2 (sketched residual;
 *   a project choice for callers without a reference solution).
 * Both are tested at the top of iteration k, before the k-th projection, so
 * `iters` counts the projections applied. */
#define CSK_STOP_REL_ERR 0
#define CSK_STOP_REL_RESID 1

typedef struct csk_solve_opts {
    double tol;              /* see the stopping rules above                     */
    int64_t maxit;           /* at most this many projections (>= 0)             */
    int32_t stop_mode;       /* CSK_STOP_REL_ERR or CSK_STOP_REL_RESID            */
    int32_t refresh_every;   /* mixed precision: exact FP64 residual every K
                                iterations (0 -> 64)                             */
    const double* x_ref;     /* n, device; required for CSK_STOP_REL_ERR         */
    const volatile int32_t* cancel; /* nullable; host-mapped pinned or device
                                word polled every check_every iterations; a
                                nonzero value ends the solve with CSK_CANCELLED */
    int32_t check_every;     /* cancel poll interval (0 -> 256)                  */
    int32_t grid;            /* persistent grid size; 0 -> automatic             */
    int32_t block;           /* threads per workgroup; 0 -> automatic            */
    int32_t single_wg;       /* -1 auto, 0 force grid path, 1 force one WG       */
    int64_t* trace_idx;      /* nullable, device, at least maxit entries: the
                                solve writes trace_idx[k] = i_k, the row it
                                projects onto at iteration k, for every k <
                                iters (Algorithm 1's selected index; entries
                                from iters on are left as they were).  Read by
                                csk_solve, csk_solve_csr, csk_solve_rgrk and
                                csk_solve_rk; the batched and multi-RHS calls
                                ignore it.                                       */
} csk_solve_opts;

/* Written by the device at the end of a solve (device memory). */
typedef struct csk_solve_result {
    int64_t iters;           /* projections applied                               */
    int32_t status;          /* CSK_OK, CSK_NOT_CONVERGED, CSK_ERR_NONFINITE,
                                CSK_ERR_DEGENERATE or CSK_CANCELLED               */
    int32_t fp64_fallback;   /* mixed precision: 1 if the solve finished in
                                plain FP64 iterations after stagnating            */
    double final_measure;    /* the stop measure at exit: RES (REL_ERR) or
                                ||r||^2/||bt||^2 (REL_RESID)                      */
    int64_t refreshes;       /* mixed precision: exact residual refreshes         */
} csk_solve_result;

/* Static text for a status code. */
const char* csk_status_string(csk_status s);
/* Text of the last host-side failure on the calling thread ("" if none). */
const char* csk_last_error(void);
/* ABI version (major*10000 + minor*100 + patch). */
int32_t csk_version(void);

/* ---- A1: the hash alone (Definition 1) --------------------------------- *
 * bucket[i] = h(i) and sign[i] = D_ii for i in [0, m).  Either output may be
 * NULL.  Requires m >= 1, 1 <= d < 2^31.                                     */
csk_status csk_hash(uint64_t seed, int64_t m, int64_t d, uint32_t* bucket, int8_t* sign,
                    void* stream);

/* ---- A1-A5: the dense sketch (Algorithm 1, Initialize) ----------------- *
 * Computes At = S A and Bt = S B for the A (m x n, dtype a_dtype in {F64,
 * F32}, leading dimension lda) and optional B (m x nrhs FP64, leading
 * dimension ldb; nrhs = 1 for the vector b of Algorithm 1).
 * Outputs (each nullable, at least one of At64 / At_lp non-NULL):
 *   At64   d x n FP64, leading dimension ldat64;
 *   At_lp  d x n in lp_dtype (F32, F16 or BF16), leading dimension ldat_lp,
 *          the two-step RNE rounding of the FP64 sketch;
 *   Bt     d x nrhs FP64, leading dimension ldbt (required when B is given);
 *   nu2    d FP64: ||At64^(j)||^2, the squared norm of the FP64 row (zero for
 *          empty buckets), computed from the FP64 sums even if At64 is NULL;
 *   perm   m u32: rows grouped by bucket, ascending within a bucket;
 *   ptr    d+1 u32: bucket j owns perm[ptr[j] .. ptr[j+1]), ptr[d] = m.
 * Requires 1 <= m < 2^31, n >= 1, 1 <= d < 2^31, lda >= n.  The paper asks
 * for d < m; that is recommended, not enforced (the sketch stays defined).
 * Memory: when A (or B) starts on 16 bytes and its leading dimension times
 * the element size is a multiple of 16, rows are read in whole 16-byte
 * vectors, so the bytes of the last row up to the end of the vector holding
 * its last column are read (their values are ignored); a buffer of m * lda
 * elements always suffices.  Otherwise rows are read element by element.   */
csk_status csk_sketch_workspace_size(int64_t m, int64_t n, int64_t d, int64_t nrhs, size_t* bytes /*host*/);
csk_status csk_sketch(const void* A, csk_dtype a_dtype, int64_t m, int64_t n, int64_t lda,
                      const double* B, int64_t nrhs, int64_t ldb,
                      int64_t d, uint64_t seed,
                      double* At64, int64_t ldat64,
                      void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp,
                      double* Bt, int64_t ldbt,
                      double* nu2, uint32_t* perm, uint32_t* ptr,
                      void* ws, size_t ws_bytes, void* stream);

/* ---- A10: the sketch of a CSR matrix ------------------------------------ *
 * A given as row_ptr (m+1, int64, row_ptr[0] = 0, nondecreasing), col (nnz,
 * int32 in [0, n), distinct within a row) and val (nnz, FP32).  Same outputs
 * and summation order as csk_sketch (each dense entry of At is the ascending-
 * row sum of the stored entries that land on it; absent entries add nothing).
 * b (m FP64) and bt (d FP64) are nullable together.                          */
csk_status csk_sketch_csr_workspace_size(int64_t m, int64_t n, int64_t d, size_t* bytes /*host*/);
csk_status csk_sketch_csr(const int64_t* row_ptr, const int32_t* col, const float* val,
                          int64_t m, int64_t n, int64_t nnz, const double* b,
                          int64_t d, uint64_t seed,
                          double* At64, int64_t ldat64,
                          void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp,
                          double* bt, double* nu2,
                          void* ws, size_t ws_bytes, void* stream);

/* ---- A10, sparse result: the sketch of a CSR matrix as a CSR matrix ---- *
 * Same input contract as csk_sketch_csr (Definition 1 and Algorithm 1,
 * Initialize).  Row j of At holds the union of the stored columns of the
 * rows hashed to bucket j, in ascending column order, each value the
 * ascending-row FP64 sum of the signed stored entries landing on it (bitwise
 * the entry csk_sketch_csr writes densely; a sum that cancels to zero stays
 * stored).  Outputs (device): at_row_ptr (d + 1 int64, at_row_ptr[0] = 0,
 * at_row_ptr[d] = nnz(At) <= nnz), at_col (int32) and at_val (FP64), each
 * with room for nnz entries (the caller cannot know nnz(At) before the call;
 * read at_row_ptr[d] after it).  nu2 (nullable): squared row norms, bitwise
 * those of csk_sketch_csr.  b and bt are nullable together.
 * Requires 1 <= m, d < 2^31, 1 <= n <= 131072, nnz < 2^32 - 1.            */
csk_status csk_sketch_csr_sparse_workspace_size(int64_t m, int64_t n, int64_t d, size_t* bytes /*host*/);
csk_status csk_sketch_csr_sparse(const int64_t* row_ptr, const int32_t* col, const float* val,
                                 int64_t m, int64_t n, int64_t nnz, const double* b,
                                 int64_t d, uint64_t seed,
                                 int64_t* at_row_ptr, int32_t* at_col, double* at_val,
                                 double* bt, double* nu2,
                                 void* ws, size_t ws_bytes, void* stream);

/* ---- A6/A7: the MWRK loop on the sketched system (Algorithm 1, loop) ---- *
 * at_dtype = F64: At is the FP64 sketch (At64 may be NULL or equal to At);
 *   plain FP64 iterations.
 * at_dtype in {F32, F16, BF16}: mixed precision.  At is the low-precision
 *   sketch and At64 (required) the FP64 one.  Every refresh_every iterations
 *   the exact residual r_ref = bt - At64 x is recomputed in FP64 and x_ref
 *   saved; in between r = r_ref - At * (x - x_ref) with FP32 accumulation.
 *   Selection weights and projections use the FP64 row and nu2.  If the
 *   exact stop measure fails to decrease over two refresh windows the solve
 *   continues with plain FP64 iterations (result.fp64_fallback = 1).
 * nu2: d FP64 squared row norms of At64 (nullable: computed into ws).
 * x0: n FP64 start (nullable: zero, as in Section 3).  x: n FP64 output.
 * Rows of zero norm are never selected; ties go to the lowest row index.
 * Requires d >= 1, 1 <= n <= 8192, ldat >= n, d < 2^31.
 * Memory: when At (and At64) start on 16 bytes and ldat * element size is a
 * multiple of 16, rows are read in whole 16-byte vectors, so the bytes of
 * the last row up to the end of the vector holding column n - 1 are read
 * (their values are ignored); a buffer of d * ldat elements always
 * suffices.  Otherwise rows are read element by element.
 * The solve keeps part of At in LDS for its whole duration (as much as fits
 * beside x); nothing of it is written back.                                 */
csk_status csk_solve_workspace_size(int64_t d, int64_t n, csk_dtype at_dtype, size_t* bytes /*host*/);
csk_status csk_solve(const void* At, csk_dtype at_dtype, int64_t ldat,
                     const double* At64, int64_t ldat64,
                     int64_t d, int64_t n, const double* bt, const double* nu2,
                     const double* x0, double* x,
                     const csk_solve_opts* opts /*host*/, csk_solve_result* res,
                     void* ws, size_t ws_bytes, void* stream);

/* ---- A7 for a sparse A: the refresh residual from the CSR A itself ---- *
 * The mixed-precision solve of csk_solve (at_dtype F32, F16 or BF16, At64
 * required for the projections and the FP64 fallback) on the sketch of a
 * CSR matrix, with each refresh residual taken as r_ref = S (b - A x) from
 * the CSR A (row_ptr m + 1 int64, col int32, val FP32, b m FP64, all
 * device; S the count sketch of seed, as csk_sketch_csr used) instead of
 * bt - At64 x: equal in exact arithmetic, it reads about 12 bytes per
 * stored entry of A per refresh where bt - At64 x reads the d x n FP64
 * sketch.  y_i = b_i - sum_e val_e x_col(e) (row i's entries in order,
 * summed from zero in FP64), then r_ref_j = sum over rows i of bucket j in
 * ascending order of D_ii y_i.  The call groups the rows by bucket itself
 * (inside ws).  Other arguments, results and errors as csk_solve;
 * additionally CSK_ERR_INVALID_ARG for an FP64 At, missing CSR arrays or b,
 * or m or d outside [1, 2^31).  ws: csk_solve_csr_refresh_workspace_size
 * bytes, 256-byte aligned.                                                  */
csk_status csk_solve_csr_refresh_workspace_size(int64_t m, int64_t d, int64_t n, size_t* bytes /*host*/);
csk_status csk_solve_csr_refresh(const void* At, csk_dtype at_dtype, int64_t ldat,
                                 const double* At64, int64_t ldat64, int64_t d, int64_t n,
                                 const int64_t* row_ptr, const int32_t* col, const float* val,
                                 int64_t m, const double* b, uint64_t seed,
                                 const double* bt, const double* nu2, const double* x0, double* x,
                                 const csk_solve_opts* opts /*host*/, csk_solve_result* res,
                                 void* ws, size_t ws_bytes, void* stream);

/* ---- csk_solve without a workspace: for callers that cannot allocate ---- *
 * For code that must not call hipMalloc (work recorded under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * solve as csk_solve, same arguments and results, bitwise the same x and
 * result for the same inputs and launch shape, but its workspace (exchange
 * records, the FP64 refresh residual, norms computed when nu2 is NULL) comes
 * from a static device array of CSK_NOALLOC_SCRATCH_BYTES inside the library.
 * The library makes no allocation of any kind on this path.
 * Limit: the workspace csk_solve would need, 16 bytes per row plus 128 bytes
 * per workgroup of the launch, must fit the scratch (d up to about 520000
 * rows); a larger solve returns CSK_ERR_WORKSPACE before anything is
 * enqueued (csk_last_error names the sizes).
 * Each device holds its own copy of the array from the library's load until
 * the process ends; every call on a device shares that copy, and each call
 * clears what it needs cleared, so calls in sequence (on one stream, or
 * ordered by events) are independent.  Calls that may overlap on one device
 * (two streams, or two threads, without ordering) race on the scratch and
 * give undefined results: order them, or use csk_solve with separate
 * workspaces.                                                                */
#define CSK_NOALLOC_SCRATCH_BYTES (8u << 20)
csk_status csk_solve_noalloc(const void* At, csk_dtype at_dtype, int64_t ldat,
                             const double* At64, int64_t ldat64,
                             int64_t d, int64_t n, const double* bt, const double* nu2,
                             const double* x0, double* x,
                             const csk_solve_opts* opts /*host*/, csk_solve_result* res,
                             void* stream);

/* ---- Randomized selection rules on the FP64 sketch --------------------- *
 * The introduction places Algorithm 1's loop in a family of row-selection
 * rules and Section 3 compares it with two of them; these calls run the loop
 * with such a rule in place of the greedy one.  Both take the FP64 At (d x n,
 * leading dimension ldat), bt, nu2 (nullable: computed into ws), x0
 * (nullable: zero), x and opts as csk_solve does (refresh_every, grid and
 * single_wg of opts apply as there; the memory contract on At is csk_solve's),
 * and draw their random numbers from the selection stream of sel_seed: its
 * k-th uniform is (top 52 bits of the k-th SplitMix64 output of sel_seed
 * + 1/2) * 2^-52, strictly inside (0, 1).  Same seed, same inputs and same
 * launch shape give the same result.
 *
 * csk_solve_rgrk: the relaxed greedy randomized rule of Bai & Wu (theta in
 *   [0, 1]; theta = 1/2 is their greedy randomized Kaczmarz, theta = 1 the
 *   greedy rule up to exact ties).  At iteration k, with r = bt - At x_k,
 *   M the largest r_i^2 / ||At^(i)||^2 over rows of nonzero norm,
 *   R = ||r||^2 and F = ||At||_F^2 (the sum of nu2), the working set is
 *   the rows of nonzero norm with r_i^2 / ||At^(i)||^2 >= t_k,
 *   t_k = min(M, theta M + (1 - theta) R / F) (the published test
 *   |r_i|^2 >= eps_k ||r||^2 ||At^(i)||^2 rewritten; the cap keeps the best
 *   row in the set under rounding), and i_k is the member with the largest
 *   r_i^2 / E_i, E_i = -log(uniform k d + i), lowest index on ties: row i
 *   with probability r_i^2 over the members' sum.  Requires 1 <= n <= 8192,
 *   d < 2^31; each workgroup keeps its rows' residuals in LDS (too many rows
 *   per workgroup: CSK_ERR_UNSUPPORTED, ask for a larger grid).
 * csk_solve_rk: randomized Kaczmarz (Strohmer & Vershynin): row i with
 *   probability ||At^(i)||^2 / ||At||_F^2 each iteration, i_k the smallest i
 *   with C_i > u_k C_{d-1}, C the cumulative sums of nu2 and u_k the k-th
 *   uniform (C is summed in 512 segments, so it can differ from one running
 *   sum in index order in the last bits; a row of zero norm is never
 *   drawn).  Only the drawn row's residual is formed, so the
 *   stop mode must be CSK_STOP_REL_ERR (else CSK_ERR_INVALID_ARG).  One
 *   workgroup; requires 1 <= n <= 8192, d < 2^31.                           */
csk_status csk_solve_rgrk_workspace_size(int64_t d, int64_t n, size_t* bytes /*host*/);
csk_status csk_solve_rgrk(const double* At, int64_t ldat, int64_t d, int64_t n,
                          const double* bt, const double* nu2, const double* x0, double* x,
                          double theta, uint64_t sel_seed,
                          const csk_solve_opts* opts /*host*/, csk_solve_result* res,
                          void* ws, size_t ws_bytes, void* stream);
csk_status csk_solve_rk_workspace_size(int64_t d, int64_t n, size_t* bytes /*host*/);
csk_status csk_solve_rk(const double* At, int64_t ldat, int64_t d, int64_t n,
                        const double* bt, const double* nu2, const double* x0, double* x,
                        uint64_t sel_seed,
                        const csk_solve_opts* opts /*host*/, csk_solve_result* res,
                        void* ws, size_t ws_bytes, void* stream);

/* ---- The MWRK loop on a CSR sketch (Algorithm 1, loop) ------------------ *
 * The loop of csk_solve in FP64 with At given as CSR (at_row_ptr d + 1
 * int64 with at_row_ptr[0] = 0 and at_row_ptr[d] = nnz, at_col int32 in
 * [0, n) and distinct within a row, at_val FP64), e.g. from
 * csk_sketch_csr_sparse.  Each iteration reads the nnz stored entries
 * instead of d * n.  nu2: squared row norms (nullable: computed into ws).
 * opts as for csk_solve (refresh_every is ignored: there is no low-precision
 * copy).  A row pointer array inconsistent with nnz ends the solve with
 * result.status = CSK_ERR_INVALID_ARG.
 * Requires 1 <= d < 2^31, 1 <= n <= 16384, nnz < 2^31; the workgroup's
 * share of rows must fit LDS beside x (else CSK_ERR_UNSUPPORTED: ask for
 * more workgroups).  Each workgroup keeps part of its rows' entries in LDS
 * for the whole solve.                                                      */
csk_status csk_solve_csr_workspace_size(int64_t d, int64_t n, int64_t nnz, size_t* bytes /*host*/);
csk_status csk_solve_csr(const int64_t* at_row_ptr, const int32_t* at_col, const double* at_val,
                         int64_t d, int64_t n, int64_t nnz, const double* bt, const double* nu2,
                         const double* x0, double* x,
                         const csk_solve_opts* opts /*host*/, csk_solve_result* res,
                         void* ws, size_t ws_bytes, void* stream);

/* ---- Tuning of the persistent solve's launch shape ---------------------- *
 * csk_tune_solve times trial_iters MWRK iterations (no convergence test) of
 * each candidate launch shape on the given system -- one workgroup while the
 * matrix is small, 64, 128, 192 and one workgroup per CU, each with the
 * lanes-per-row splits whose padded row length is within 25% of the best --
 * and records the fastest in a process-wide cache keyed by (device, d, n,
 * at_dtype, vector rows).  Every later csk_solve of that key that leaves the
 * shape to the library (opts->grid == 0, opts->single_wg == -1) uses it.
 * The timing synchronizes the stream; the workspace holds the trial runs'
 * x and result (csk_tune_solve_workspace_size).  Arguments as csk_solve.
 * csk_tune_lookup reads the cache (grid 0: no entry; vector_rows: whether
 * the rows are 16-byte vectors, i.e. At 16-byte aligned and ldat * element
 * size a multiple of 16); csk_tune_clear empties it.  The cache is guarded
 * by a mutex; all other calls stay reentrant.                               */
typedef struct csk_tune_entry {
    int32_t grid;            /* workgroups (1: single-workgroup kernel)          */
    int32_t lanes_per_row;   /* 4, 16 or 64                                      */
    double us_per_iter;      /* measured microseconds per iteration              */
} csk_tune_entry;
csk_status csk_tune_solve_workspace_size(int64_t d, int64_t n, csk_dtype at_dtype, size_t* bytes /*host*/);
csk_status csk_tune_solve(const void* At, csk_dtype at_dtype, int64_t ldat,
                          const double* At64, int64_t ldat64,
                          int64_t d, int64_t n, const double* bt, const double* nu2,
                          int32_t trial_iters, csk_tune_entry* best /*host, nullable*/,
                          void* ws, size_t ws_bytes, void* stream);
csk_status csk_tune_lookup(int64_t d, int64_t n, csk_dtype at_dtype, int32_t vector_rows,
                           csk_tune_entry* out /*host*/);
void csk_tune_clear(void);

/* ---- A8: many independent systems, sketch + solve in one pass ---------- *
 * Each descriptor (host array) names one system's device buffers.  A is
 * a_dtype (F64 or F32); the solve runs in lp_dtype (F64 = plain, else mixed
 * with an FP64 copy kept in ws) with opts shared by all systems (x_ref in
 * opts is ignored; each system has its own).  res: nsys results (device).  */
typedef struct csk_system_desc {
    const void* A;        /* m x n, leading dimension lda                        */
    const double* b;      /* m                                                   */
    const double* x_ref;  /* n, or NULL (then the system uses CSK_STOP_REL_RESID) */
    double* x;            /* n, output                                           */
    int64_t m, n, lda, d;
    uint64_t seed;
} csk_system_desc;
csk_status csk_solve_batched_workspace_size(const csk_system_desc* sys /*host*/, int32_t nsys,
                                            csk_dtype a_dtype, csk_dtype lp_dtype, size_t* bytes /*host*/);
csk_status csk_solve_batched(const csk_system_desc* sys /*host*/, int32_t nsys,
                             csk_dtype a_dtype, csk_dtype lp_dtype,
                             const csk_solve_opts* opts /*host*/, csk_solve_result* res,
                             void* ws, size_t ws_bytes, void* stream);

/* Where csk_solve_batched keeps system s's sketch (Definition 1 and
 * Algorithm 1, Initialize, applied to that system) inside its workspace,
 * for callers that read the sketch the solve used once the call's work has
 * finished.  Byte offsets count from the start of ws; at64 holds d x n FP64
 * with leading dimension ld64, at_lp (-1 when lp_dtype is F64) d x n in
 * lp_dtype with leading dimension ld_lp, both with zeros past column n; bt
 * and nu2 hold d FP64 each.  Arguments as csk_solve_batched_workspace_size;
 * 0 <= s < nsys.  The layout depends only on the descriptors' sizes and the
 * two dtypes.                                                              */
typedef struct csk_batched_sketch_loc {
    int64_t at64, at_lp, bt, nu2;  /* byte offsets into ws                      */
    int64_t ld64, ld_lp;           /* leading dimensions, in elements            */
} csk_batched_sketch_loc;
csk_status csk_solve_batched_sketch_loc(const csk_system_desc* sys /*host*/, int32_t nsys, csk_dtype a_dtype,
                                        csk_dtype lp_dtype, int32_t s, csk_batched_sketch_loc* out /*host*/);

/* ---- Tuning of the multi-RHS and batched launches; the tune cache on disk *
 * csk_tune_report: what a tuner measured.  `choice` is the fastest
 * candidate and `default_choice` the library's untuned one, in the kernel
 * family's terms (multi-RHS: 16-row tiles per workgroup; batched: the plan
 * variant, see csk_tune_batched); `us` and `default_us` their measured times
 * (multi-RHS: microseconds per iteration; batched: microseconds per call).
 *
 * csk_tune_mrhs times trial_iters iterations (no convergence test) of
 * csk_solve_mrhs on the given system for every row-tile count from the
 * default (the fewest that keep one workgroup per CU) up to 8, and records
 * the fastest for (architecture, d, n, nrhs, lp_dtype); later csk_solve_mrhs
 * calls of that key use it.  Arguments as csk_solve_mrhs; the workspace
 * (csk_tune_mrhs_workspace_size) holds the trial runs' solutions and
 * results.  The timing synchronizes the stream.
 *
 * csk_tune_batched runs csk_solve_batched on the given systems once per
 * plan variant -- 0: the default (the split plan of the modelled iteration
 * counts, longest estimated system first), 1: no system split, 2: splits
 * priced at half the modelled exchange cost (more splitting), 3: at twice
 * it (less), 4: the default split with the systems in the given order --
 * and records the fastest for (architecture, the systems' shapes, a_dtype,
 * lp_dtype); later csk_solve_batched calls of that key use it.  Each run is
 * a full solve (the systems' x and res hold the last one's result);
 * arguments and workspace as csk_solve_batched.
 *
 * The cache of all tuners is process-wide.  csk_tune_save writes it to a
 * text file (architecture-keyed entries, stamped with csk_version());
 * csk_tune_load merges a file's entries (a file of another library version
 * is ignored; *entries, nullable, receives the count read, -1 for none).
 * When the environment variable CSK_TUNE_CACHE names a file, the cache is
 * read from it on first use and written back after every tuning call.      */
typedef struct csk_tune_report {
    int32_t choice, default_choice;
    double us, default_us;
    int32_t candidates;
} csk_tune_report;
csk_status csk_tune_mrhs_workspace_size(int64_t d, int64_t n, int64_t nrhs, size_t* bytes /*host*/);
csk_status csk_tune_mrhs(const void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp,
                         const double* At64, int64_t ldat64, int64_t d, int64_t n,
                         const double* Bt, int64_t nrhs, int64_t ldbt, const double* nu2,
                         int32_t trial_iters, csk_tune_report* report /*host, nullable*/,
                         void* ws, size_t ws_bytes, void* stream);
csk_status csk_tune_batched(const csk_system_desc* sys /*host*/, int32_t nsys,
                            csk_dtype a_dtype, csk_dtype lp_dtype,
                            const csk_solve_opts* opts /*host*/, csk_solve_result* res,
                            csk_tune_report* report /*host, nullable*/,
                            void* ws, size_t ws_bytes, void* stream);
csk_status csk_tune_save(const char* path /*host*/);
csk_status csk_tune_load(const char* path /*host*/, int32_t* entries /*host, nullable*/);

/* ---- A9: one sketch, many right-hand sides ----------------------------- *
 * Runs the loop of Algorithm 1 independently for each column j of Bt (d x
 * nrhs FP64) on the shared At: X[:, j] (n x nrhs, leading dimension ldx)
 * solves At X[:, j] = Bt[:, j].  The residuals of all columns are formed
 * together as R = R_ref - At_lp (X - X_ref) with At_lp in BF16 or F16 on the
 * matrix cores (FP32 accumulation) and an exact FP64 refresh
 * R_ref = Bt - At64 X_ref every refresh_every iterations.  For n <= 512,
 * X - X_ref enters the products as the sum of the projected rows of At_lp
 * (each step's sum formed in FP32 and rounded to lp_dtype); beyond that, as
 * X - X_ref rounded to lp_dtype.  Selection, projections and X use the FP64
 * rows in both cases.  Xref (n x nrhs,
 * leading dimension ldxref) is the reference for CSK_STOP_REL_ERR (per
 * column).  res: nrhs results (device).  Requires n <= 1024.                */
csk_status csk_solve_mrhs_workspace_size(int64_t d, int64_t n, int64_t nrhs, size_t* bytes /*host*/);
csk_status csk_solve_mrhs(const void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp,
                          const double* At64, int64_t ldat64,
                          int64_t d, int64_t n,
                          const double* Bt, int64_t nrhs, int64_t ldbt,
                          const double* nu2,
                          const double* X0, double* X, int64_t ldx,
                          const double* Xref, int64_t ldxref,
                          const csk_solve_opts* opts /*host*/, csk_solve_result* res,
                          void* ws, size_t ws_bytes, void* stream);

/* ---- Algorithm 1 as one HIP graph ---------------------------------------- *
 * csk_pipeline_capture records csk_sketch (A, b -> At64 [, At_lp], bt, nu2;
 * Algorithm 1, Initialize) followed by csk_solve (the loop; mixed precision
 * when At_lp is given, on lp_dtype) on `stream` into a HIP graph, without
 * running them, and instantiates it.  csk_pipeline_launch replays the whole
 * pipeline on a stream: one launch instead of the chain of dependent kernel
 * launches, with every pointer, size and option fixed at capture (update the
 * contents of A, b, x0 and opts->x_ref between launches, never their
 * addresses).  Arguments mean what they mean for csk_sketch (b a vector,
 * nrhs 1) and csk_solve; the two workspaces are those calls' own and must
 * stay allocated, like every other buffer, until the last launch has
 * finished.  `stream` must be a created stream (not the null stream) with
 * no capture in progress; a failure of either call ends the capture and is
 * returned (nothing is recorded or run).  csk_pipeline_destroy releases the
 * graph (NULL is accepted).  Launches of one pipeline that overlap in time
 * race on its buffers.                                                      */
typedef struct csk_pipeline_s* csk_pipeline;
csk_status csk_pipeline_capture(const void* A, csk_dtype a_dtype, int64_t m, int64_t n, int64_t lda,
                                const double* b, int64_t d, uint64_t seed,
                                double* At64, int64_t ldat64,
                                void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp,
                                double* bt, double* nu2, const double* x0, double* x,
                                const csk_solve_opts* opts /*host*/, csk_solve_result* res,
                                void* ws_sketch, size_t ws_sketch_bytes,
                                void* ws_solve, size_t ws_solve_bytes,
                                void* stream, csk_pipeline* out /*host*/);
csk_status csk_pipeline_launch(csk_pipeline p, void* stream);
csk_status csk_pipeline_destroy(csk_pipeline p);

#ifdef __cplusplus
}
#endif
#endif /* CSK_H */
