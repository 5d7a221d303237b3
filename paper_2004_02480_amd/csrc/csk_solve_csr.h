// csk_solve_csr.h -- internal interface of the MWRK loop (Algorithm 1, loop)
// on a sketched matrix stored as CSR.
#pragma once

#include "csk_internal.h"

namespace csk {

struct CsrSolveSys {
    const int64_t* rp;    // d + 1 row offsets, rp[0] = 0, rp[d] = nnz
    const int32_t* col;   // nnz column indices, distinct within a row
    const double* val;    // nnz FP64 values
    const double* bt;     // d
    const double* nu2;    // d squared row norms, or null (computed)
    const double* x0;     // n or null (zero start)
    const double* xref;   // n or null
    double* x;            // n, output
    csk_solve_result* res;
    int64_t nnz;
    int32_t d, n;
    int32_t stop_mode;
    int32_t pad_;
};

int csr_solve_grid(int64_t d, int64_t nnz, const csk_solve_opts* o);
int csr_solve_lpr(int64_t d, int64_t nnz);
size_t csr_solve_ws_bytes(int64_t d, int grid);
csk_status csr_solve_run(const CsrSolveSys& sys, const csk_solve_opts* o, void* ws, size_t ws_bytes,
                         hipStream_t st);

}  // namespace csk
