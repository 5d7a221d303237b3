// csk_mrhs.h -- internal interface of the multi-right-hand-side solver.
#pragma once

#include "csk_internal.h"

namespace csk {

size_t mrhs_ws_bytes(int64_t d, int64_t n, int64_t nrhs);
csk_status mrhs_run(const void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp, const double* At64, int64_t ldat64,
                    int64_t d, int64_t n, const double* Bt, int64_t nrhs, int64_t ldbt, const double* nu2,
                    const double* X0, double* X, int64_t ldx, const double* Xref, int64_t ldxref,
                    const csk_solve_opts* o, csk_solve_result* res, void* ws, size_t ws_bytes, hipStream_t st,
                    int rt_force = 0);
size_t mrhs_tune_ws_bytes(int64_t d, int64_t n, int64_t nrhs);
csk_status mrhs_tune(const void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp, const double* At64, int64_t ldat64,
                     int64_t d, int64_t n, const double* Bt, int64_t nrhs, int64_t ldbt, const double* nu2,
                     int32_t trial_iters, csk_tune_report* rep, void* ws, size_t ws_bytes, hipStream_t st);

}  // namespace csk
