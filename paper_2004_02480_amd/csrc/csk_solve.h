// csk_solve.h -- internal interface of the MWRK solver (Algorithm 1, loop).
#pragma once

#include "csk_internal.h"

namespace csk {

// One sketched system as the solver sees it.
struct SolveSys {
    const void* At;       // d x n in the working precision (FP64 in plain mode)
    const double* At64;   // d x n FP64 (projections, refreshes)
    const double* bt;     // d
    const double* nu2;    // d, squared norms of the FP64 rows
    const double* x0;     // n or null (zero start)
    const double* xref;   // n or null
    double* x;            // n, output
    double* rref;         // d, exact residual of the last refresh (mixed)
    csk_solve_result* res;
    int64_t ldat, ldat64;
    int32_t d, n;
    int32_t stop_mode;
    int32_t npad;         // LDS length of the operand vectors (>= n, zero-padded)
};

// Mixed precision on the sketch of a CSR matrix: the refresh residual taken
// as r_ref = S (b - A x) from the CSR A itself, in place of bt - At64 x.
// rp/col/val/b: the CSR A (m rows) and b; perm/ptr: the rows grouped by
// bucket, ascending within a bucket (the sketch's grouping for seed); y: m
// doubles of scratch; flags: kRefreshFlags grid-barrier words; self: device
// memory for a copy of this descriptor (the kernel reads it from there).
constexpr int kRefreshFlags = 1024;
struct CsrRef {
    const int64_t* rp;
    const int32_t* col;
    const float* val;
    const double* b;
    const uint32_t* perm;
    const uint32_t* ptr;
    double* y;
    uint32_t* flags;
    int64_t m;
    uint64_t seed;
    CsrRef* self;
};

struct SolvePlan {
    int lpr;        // lanes per row in the residual product
    int vw;         // elements per vector load (1 = scalar path)
    int grid;       // workgroups (1 = single-workgroup path)
    int block;      // threads per workgroup
};

SolvePlan solve_plan(int64_t d, int64_t n, csk_dtype at_dtype, int64_t ldat, const void* At,
                     const csk_solve_opts* o);
size_t solve_ws_bytes(int64_t d, int64_t n, int grid);
// Operand length in LDS for a row of n columns with the given lanes per row.
int64_t solve_npad(int64_t n, csk_dtype at_dtype, int lpr, bool vec);
// Lanes per row used by the batched kernel.
int solve_batch_lpr();

// forced: a launch shape to use instead of the planned one (tuning), or null.
// cref: the refresh from a CSR A (mixed precision only), or null.
csk_status solve_run(const SolveSys& sys, csk_dtype at_dtype, const csk_solve_opts* o,
                     void* ws, size_t ws_bytes, hipStream_t st, const SolvePlan* forced = nullptr,
                     const CsrRef* cref = nullptr);

// The relaxed greedy randomized selection rule (FP64 At64 only; theta in
// [0, 1], selection stream seed sel_seed) in place of the greedy one.
size_t solve_rgrk_ws_bytes(int64_t d, int64_t n, int grid);
csk_status solve_rgrk_run(const SolveSys& sys, const csk_solve_opts* o, double theta, uint64_t sel_seed,
                          void* ws, size_t ws_bytes, hipStream_t st);

// nu2[i] = ||A^(i)||^2 for the d x n FP64 rows of A (leading dimension lda).
csk_status launch_row_norms2(const double* A, int64_t lda, int64_t d, int64_t n, double* nu2, hipStream_t st);

// Randomized Kaczmarz (one workgroup; stop mode REL_ERR; n <= 8192).
size_t solve_rk_ws_bytes(int64_t d);
csk_status solve_rk_run(const double* At, int64_t ldat, int64_t d, int64_t n, const double* bt, const double* nu2,
                        const double* x0, double* x, const csk_solve_opts* o, uint64_t sel_seed,
                        csk_solve_result* res, void* ws, size_t ws_bytes, hipStream_t st);

// Lanes per row with the least padded coverage, vector width of the
// working matrix, and the cache of tuned launch shapes.
int pick_lpr(int64_t n, int64_t per_lane);
int64_t chunk_k_of(csk_dtype t);
int solve_vw(csk_dtype at_dtype, int64_t ldat, const void* At);
void tune_store(int64_t d, int64_t n, csk_dtype at_dtype, int vw, int grid, int lpr, double us);
bool tune_lookup(int64_t d, int64_t n, csk_dtype at_dtype, int vw, int* grid, int* lpr, double* us);
void tune_clear();

// Batched.  Systems are handed out from an atomic queue in `order` (host,
// largest estimated work first); a system whose work is well above the
// average share of one workgroup is split over several workgroups that run
// the grid loop on it with their own exchange records.
constexpr size_t kBatchExchRecords = 4096;  // exchange records for split systems
size_t solve_exch_record_bytes();

struct BatchedPlan {
    const int32_t* order;      // host, nsys: queue position -> system
    const SolveSys* sys;       // host copy of the descriptors
    int64_t npad_max, d_max, n_max;
    int32_t* order_dev;        // nsys
    int32_t* item_off_dev;     // nsys + 1: first work item of each queue position
    int32_t* exch_off_dev;     // nsys: first exchange record of each queue position
    void* exch_dev;            // exch_records records
    size_t exch_records;
    uint32_t* queue_dev;
    int32_t variant;           // plan variant (0 default; see csk_tune_batched)
};

// `sys_dev` is the device array of nsys descriptors (rows 16-byte aligned,
// npad from solve_npad with solve_batch_lpr()).
csk_status solve_batched_run(const SolveSys* sys_dev, int32_t nsys, const BatchedPlan& bp, csk_dtype at_dtype,
                             const csk_solve_opts* o, hipStream_t st);

}  // namespace csk
