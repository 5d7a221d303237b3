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

csk_status solve_run(const SolveSys& sys, csk_dtype at_dtype, const csk_solve_opts* o,
                     void* ws, size_t ws_bytes, hipStream_t st);

// Batched: `sys` is a device array of nsys systems (rows 16-byte aligned,
// npad from solve_npad with solve_batch_lpr()); `order` (device, nsys) lists
// them in the order the work queue hands them out.
csk_status solve_batched_run(const SolveSys* sys_dev, const int32_t* order_dev, int32_t nsys,
                             int64_t npad_max, csk_dtype at_dtype, const csk_solve_opts* o,
                             uint32_t* queue_dev, hipStream_t st);

}  // namespace csk
