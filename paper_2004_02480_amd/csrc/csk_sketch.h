// csk_sketch.h -- internal interface of the sketch pipeline (Algorithm 1,
// Initialize): At = S A, Bt = S B for one or many systems at once.
#pragma once

#include "csk_internal.h"

namespace csk {

// One system of a sketch batch.  All offsets index the batch-wide arrays:
// rows of every system form one global row space (perm), buckets one global
// bucket space (cnt, ptr), and segmented-sum work items one task space.
struct SketchSys {
    const void* A;        // m x n, leading dimension lda (a_dtype)
    const double* B;      // m x nrhs FP64, leading dimension ldb, or null
    double* At64;         // d x n, ldat64, or null
    void* Atlp;           // d x n in lp dtype, ldatlp, or null
    double* Bt;           // d x nrhs, ldbt (when B)
    double* nu2;          // d, or null
    int64_t lda, ldb, ldat64, ldatlp, ldbt;
    int64_t m;
    int64_t row_off;      // first global row
    int64_t bkt_off;      // first global bucket
    int64_t task_off;     // first global segsum task
    uint64_t seed;
    int32_t n, d, nrhs, nchunks;
    int32_t zpad;         // write zeros to the row padding (columns n .. ld - 1)
    int32_t pad_;
};

// Host-side description of a batch before it is laid out.
struct SketchJob {
    const void* A;
    const double* B;
    double* At64;
    void* Atlp;
    double* Bt;
    double* nu2;
    int64_t m, n, lda, nrhs, ldb, d, ldat64, ldatlp, ldbt;
    uint64_t seed;
    int32_t zpad;         // the outputs' row padding is the library's own: zero it
};

// Workspace bytes for a batch of `nsys` systems with total rows M, total
// buckets D and total segsum tasks T (see sketch_tasks).
size_t sketch_ws_bytes(int64_t M, int64_t D, int64_t T, int32_t nsys);
int64_t sketch_chunks(int64_t n, csk_dtype a_dtype);

// Runs the whole sketch pipeline for `jobs` (host array) on `stream`, with
// scratch carved from `ws`.  Optional perm/ptr outputs (single-system only).
csk_status sketch_run(const SketchJob* jobs, int32_t nsys, csk_dtype a_dtype, csk_dtype lp_dtype,
                      uint32_t* perm_out, uint32_t* ptr_out,
                      void* ws, size_t ws_bytes, hipStream_t stream);

// CSR sketch (FP32 values), single system: dense outputs, or (sparse) At as
// CSR with FP64 values.  Workspace bytes of either.
size_t sketch_csr_ws_bytes(int64_t m, int64_t d, bool sparse);
// The rows 0..m-1 grouped by bucket (seed, d buckets), ascending within a
// bucket: perm (m) and ptr (d + 1), both inside ws (group_ws_bytes).
size_t group_ws_bytes(int64_t m, int64_t d);
csk_status group_only(int64_t m, int64_t d, uint64_t seed, void* ws, size_t ws_bytes, const uint32_t** perm,
                      const uint32_t** ptr, hipStream_t st);
csk_status sketch_csr_sparse_run(const int64_t* row_ptr, const int32_t* col, const float* val, int64_t m,
                                 int64_t n, const double* b, int64_t d, uint64_t seed, int64_t* at_rp,
                                 int32_t* at_col, double* at_val, double* bt, double* nu2, void* ws, size_t ws_bytes,
                                 hipStream_t st);
csk_status sketch_csr_run(const int64_t* row_ptr, const int32_t* col, const float* val, int64_t m, int64_t n,
                          int64_t nnz, const double* b, int64_t d, uint64_t seed, double* At64, int64_t ldat64,
                          void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp, double* bt, double* nu2,
                          void* ws, size_t ws_bytes, hipStream_t st);

}  // namespace csk
