// csk_api.hip -- the extern "C" boundary of libcsk (declared in csk.h):
// argument validation, workspace layout and the launch sequence of each
// entry point.  All compute happens in the kernels of sketch.hip,
// sketch_csr.hip, solve.hip and mrhs.hip.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "csk_sketch.h"
#include "csk_solve.h"
#include "csk_solve_csr.h"
#include "csk_mrhs.h"
#include "csk_tune.h"

namespace csk {

namespace {
thread_local char g_err[512] = {0};
}

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

csk_status hip_fail(hipError_t e, const char* what)
{
    set_error("%s: %s", what, hipGetErrorString(e));
    return CSK_ERR_DEVICE;
}

int device_cu_count()
{
    static std::mutex mu;
    static std::vector<int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
        cache[dev] = cus;
    }
    return cache[dev];
}

int device_max_lds()
{
    static std::mutex mu;
    static std::vector<int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int b = 0;
        if (hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || b < 65536)
            b = 65536;
        cache[dev] = b;
    }
    return cache[dev];
}

// ---- kernels local to the boundary --------------------------------------
namespace {

__global__ void k_hash_rows(uint64_t seed, int64_t m, uint32_t d, uint32_t* bucket, int8_t* sign)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t w = draw_word(seed, static_cast<uint64_t>(i));
        if (bucket) bucket[i] = draw_bucket(w, d);
        if (sign) sign[i] = (w & 1ull) ? int8_t(-1) : int8_t(1);
    }
}

struct SysPack {
    SolveSys s[24];
};

__global__ void k_store_solve_descs(SysPack pack, int count, SolveSys* dst)
{
    if ((int)threadIdx.x < count) dst[threadIdx.x] = pack.s[threadIdx.x];
}

struct OrderPack {
    int32_t v[512];
};

__global__ void k_store_order(OrderPack pack, int count, int32_t* dst)
{
    for (int k = threadIdx.x; k < count; k += blockDim.x) dst[k] = pack.v[k];
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

}  // namespace

csk_status upload_i32(const int32_t* host, int64_t count, int32_t* dev, hipStream_t st)
{
    for (int64_t k = 0; k < count; k += 512) {
        OrderPack pack;
        const int cnt = (int)std::min<int64_t>(512, count - k);
        for (int q = 0; q < cnt; ++q) pack.v[q] = host[k + q];
        k_store_order<<<1, 256, 0, st>>>(pack, cnt, dev + k);
        CSK_LAUNCH_CHECK("k_store_order");
    }
    return CSK_OK;
}

namespace {

bool lp_ok(csk_dtype t) { return t == CSK_F32 || t == CSK_F16 || t == CSK_BF16; }

constexpr int64_t kMaxN = 8192;

csk_status check_opts(const csk_solve_opts* o)
{
    if (!o) { set_error("opts is NULL"); return CSK_ERR_INVALID_ARG; }
    if (!(o->tol >= 0.0)) { set_error("tol must be >= 0"); return CSK_ERR_INVALID_ARG; }
    if (o->maxit < 0) { set_error("maxit must be >= 0"); return CSK_ERR_INVALID_ARG; }
    if (o->stop_mode != CSK_STOP_REL_ERR && o->stop_mode != CSK_STOP_REL_RESID) {
        set_error("unknown stop_mode %d", o->stop_mode);
        return CSK_ERR_INVALID_ARG;
    }
    if (o->refresh_every < 0 || o->check_every < 0 || o->grid < 0) {
        set_error("refresh_every, check_every and grid must be >= 0");
        return CSK_ERR_INVALID_ARG;
    }
    if (o->grid > 65536) { set_error("grid too large"); return CSK_ERR_INVALID_ARG; }
    return CSK_OK;
}

// Batched layout: per system, a block of the workspace holding its sketch
// (low-precision and FP64 copies with rows padded to 64 bytes), bt, nu2 and
// the refresh residual.
struct BatchLayout {
    std::vector<int64_t> off_lp, off_64, off_bt, off_nu2, off_rref, ld_lp, ld_64;
    size_t data_bytes = 0;
};

BatchLayout batch_layout(const csk_system_desc* sys, int32_t nsys, csk_dtype lp_dtype)
{
    BatchLayout L;
    const size_t lpsz = dtype_size(lp_dtype);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~size_t(255);
        const size_t at = off;
        off += bytes;
        return (int64_t)at;
    };
    for (int s = 0; s < nsys; ++s) {
        const int64_t n = sys[s].n, d = sys[s].d;
        const int64_t ld64 = (n + 7) & ~int64_t(7);
        const int64_t ldlp = (n + 31) & ~int64_t(31);
        L.ld_64.push_back(ld64);
        L.ld_lp.push_back(ldlp);
        L.off_64.push_back(take((size_t)d * ld64 * 8));
        L.off_lp.push_back(lp_dtype == CSK_F64 ? -1 : take((size_t)d * ldlp * lpsz));
        L.off_bt.push_back(take((size_t)d * 8));
        L.off_nu2.push_back(take((size_t)d * 8));
        L.off_rref.push_back(take((size_t)d * 8));
    }
    L.data_bytes = (off + 255) & ~size_t(255);
    return L;
}

csk_status check_batch(const csk_system_desc* sys, int32_t nsys, csk_dtype a_dtype, csk_dtype lp_dtype)
{
    if (!sys || nsys < 1) { set_error("need at least one system"); return CSK_ERR_INVALID_ARG; }
    if (a_dtype != CSK_F64 && a_dtype != CSK_F32) { set_error("A must be F64 or F32"); return CSK_ERR_UNSUPPORTED; }
    if (lp_dtype != CSK_F64 && !lp_ok(lp_dtype)) { set_error("bad lp_dtype"); return CSK_ERR_UNSUPPORTED; }
    for (int s = 0; s < nsys; ++s) {
        const csk_system_desc& D = sys[s];
        if (!D.A || !D.b || !D.x) { set_error("system %d: A, b and x are required", s); return CSK_ERR_INVALID_ARG; }
        if (D.m < 1 || D.n < 1 || D.d < 1 || D.lda < D.n || D.m > INT32_MAX || D.d > INT32_MAX) {
            set_error("system %d: bad sizes (m=%lld n=%lld d=%lld lda=%lld)", s, (long long)D.m, (long long)D.n,
                      (long long)D.d, (long long)D.lda);
            return CSK_ERR_INVALID_ARG;
        }
        if (D.n > kMaxN) { set_error("system %d: n=%lld exceeds %lld", s, (long long)D.n, (long long)kMaxN); return CSK_ERR_UNSUPPORTED; }
    }
    return CSK_OK;
}

}  // namespace
}  // namespace csk

using namespace csk;

extern "C" {

const char* csk_status_string(csk_status s)
{
    switch (s) {
    case CSK_OK: return "CSK_OK";
    case CSK_NOT_CONVERGED: return "CSK_NOT_CONVERGED";
    case CSK_ERR_INVALID_ARG: return "CSK_ERR_INVALID_ARG";
    case CSK_ERR_UNSUPPORTED: return "CSK_ERR_UNSUPPORTED";
    case CSK_ERR_DEVICE: return "CSK_ERR_DEVICE";
    case CSK_ERR_WORKSPACE: return "CSK_ERR_WORKSPACE";
    case CSK_ERR_NONFINITE: return "CSK_ERR_NONFINITE";
    case CSK_ERR_DEGENERATE: return "CSK_ERR_DEGENERATE";
    case CSK_CANCELLED: return "CSK_CANCELLED";
    default: return "CSK_UNKNOWN_STATUS";
    }
}

const char* csk_last_error(void) { return g_err; }

int32_t csk_version(void) { return 10100; }

csk_status csk_hash(uint64_t seed, int64_t m, int64_t d, uint32_t* bucket, int8_t* sign, void* stream)
{
    g_err[0] = 0;
    if (m < 1 || d < 1 || d > INT32_MAX) { set_error("need m >= 1 and 1 <= d < 2^31"); return CSK_ERR_INVALID_ARG; }
    if (!bucket && !sign) return CSK_OK;
    const int grid = (int)std::min<int64_t>((m + 255) / 256, 16384);
    k_hash_rows<<<grid, 256, 0, as_stream(stream)>>>(seed, m, (uint32_t)d, bucket, sign);
    CSK_LAUNCH_CHECK("k_hash_rows");
    return CSK_OK;
}

csk_status csk_sketch_workspace_size(int64_t m, int64_t n, int64_t d, int64_t nrhs, size_t* bytes)
{
    g_err[0] = 0;
    if (!bytes || m < 1 || n < 1 || d < 1 || nrhs < 0) { set_error("bad sizes"); return CSK_ERR_INVALID_ARG; }
    const int64_t T = d * std::max(sketch_chunks(n, CSK_F64), sketch_chunks(std::max<int64_t>(nrhs, 1), CSK_F64));
    *bytes = sketch_ws_bytes(m, d, T, 1);
    return CSK_OK;
}

csk_status csk_sketch(const void* A, csk_dtype a_dtype, int64_t m, int64_t n, int64_t lda,
                      const double* B, int64_t nrhs, int64_t ldb, int64_t d, uint64_t seed,
                      double* At64, int64_t ldat64, void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp,
                      double* Bt, int64_t ldbt, double* nu2, uint32_t* perm, uint32_t* ptr,
                      void* ws, size_t ws_bytes, void* stream)
{
    g_err[0] = 0;
    if (!A) { set_error("A is NULL"); return CSK_ERR_INVALID_ARG; }
    if (a_dtype != CSK_F64 && a_dtype != CSK_F32) { set_error("A must be F64 or F32"); return CSK_ERR_UNSUPPORTED; }
    if (m < 1 || n < 1 || d < 1 || m > INT32_MAX || d > INT32_MAX || n > INT32_MAX) {
        set_error("need 1 <= m, d < 2^31 and n >= 1");
        return CSK_ERR_INVALID_ARG;
    }
    if (lda < n) { set_error("lda < n"); return CSK_ERR_INVALID_ARG; }
    if (!At64 && !At_lp) { set_error("one of At64 / At_lp is required"); return CSK_ERR_INVALID_ARG; }
    if (At64 && ldat64 < n) { set_error("ldat64 < n"); return CSK_ERR_INVALID_ARG; }
    if (At_lp && !lp_ok(lp_dtype)) { set_error("lp_dtype must be F32, F16 or BF16"); return CSK_ERR_UNSUPPORTED; }
    if (At_lp && ldat_lp < n) { set_error("ldat_lp < n"); return CSK_ERR_INVALID_ARG; }
    if (B) {
        if (nrhs < 1 || ldb < nrhs || !Bt || ldbt < nrhs) { set_error("bad B / Bt arguments"); return CSK_ERR_INVALID_ARG; }
    }
    if (!ws) { set_error("workspace is NULL"); return CSK_ERR_INVALID_ARG; }
    if (reinterpret_cast<uintptr_t>(ws) & 255u) { set_error("workspace must be 256-byte aligned"); return CSK_ERR_INVALID_ARG; }
    size_t need = 0;
    csk_sketch_workspace_size(m, n, d, B ? nrhs : 0, &need);
    if (ws_bytes < need) { set_error("workspace: need %zu bytes, got %zu", need, ws_bytes); return CSK_ERR_WORKSPACE; }
    SketchJob J{};
    J.A = A;
    J.B = B;
    J.At64 = At64;
    J.Atlp = At_lp;
    J.Bt = Bt;
    J.nu2 = nu2;
    J.m = m;
    J.n = n;
    J.lda = lda;
    J.nrhs = B ? nrhs : 0;
    J.ldb = ldb;
    J.d = d;
    J.ldat64 = ldat64;
    J.ldatlp = ldat_lp;
    J.ldbt = ldbt;
    J.seed = seed;
    return sketch_run(&J, 1, a_dtype, At_lp ? lp_dtype : (csk_dtype)0, perm, ptr, ws, ws_bytes, as_stream(stream));
}

csk_status csk_sketch_csr_workspace_size(int64_t m, int64_t n, int64_t d, size_t* bytes)
{
    g_err[0] = 0;
    if (!bytes || m < 1 || n < 1 || d < 1) { set_error("bad sizes"); return CSK_ERR_INVALID_ARG; }
    *bytes = sketch_csr_ws_bytes(m, d, false);
    return CSK_OK;
}

csk_status csk_sketch_csr(const int64_t* row_ptr, const int32_t* col, const float* val, int64_t m, int64_t n,
                          int64_t nnz, const double* b, int64_t d, uint64_t seed, double* At64, int64_t ldat64,
                          void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp, double* bt, double* nu2, void* ws,
                          size_t ws_bytes, void* stream)
{
    g_err[0] = 0;
    if (!row_ptr || (nnz > 0 && (!col || !val))) { set_error("row_ptr / col / val required"); return CSK_ERR_INVALID_ARG; }
    if (m < 1 || n < 1 || d < 1 || nnz < 0 || m > INT32_MAX || d > INT32_MAX || n > INT32_MAX) {
        set_error("need 1 <= m, d < 2^31, n >= 1, nnz >= 0");
        return CSK_ERR_INVALID_ARG;
    }
    if (!At64 && !At_lp) { set_error("one of At64 / At_lp is required"); return CSK_ERR_INVALID_ARG; }
    if (At64 && ldat64 < n) { set_error("ldat64 < n"); return CSK_ERR_INVALID_ARG; }
    if (At_lp && (!lp_ok(lp_dtype) || ldat_lp < n)) { set_error("bad At_lp arguments"); return CSK_ERR_INVALID_ARG; }
    if ((b == nullptr) != (bt == nullptr)) { set_error("b and bt go together"); return CSK_ERR_INVALID_ARG; }
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) { set_error("workspace NULL or unaligned"); return CSK_ERR_INVALID_ARG; }
    size_t need = 0;
    csk_sketch_csr_workspace_size(m, n, d, &need);
    if (ws_bytes < need) { set_error("workspace: need %zu bytes, got %zu", need, ws_bytes); return CSK_ERR_WORKSPACE; }
    return sketch_csr_run(row_ptr, col, val, m, n, nnz, b, d, seed, At64, ldat64, At_lp,
                          At_lp ? lp_dtype : (csk_dtype)0, ldat_lp, bt, nu2, ws, ws_bytes, as_stream(stream));
}

constexpr int64_t kMaxCsrSketchN = 131072;  // LDS bitmap of the distinct-column count
constexpr int64_t kMaxCsrSolveN = 16384;    // x in LDS, 16-bit resident column indices

csk_status csk_sketch_csr_sparse_workspace_size(int64_t m, int64_t n, int64_t d, size_t* bytes)
{
    g_err[0] = 0;
    if (!bytes || m < 1 || n < 1 || d < 1) { set_error("bad sizes"); return CSK_ERR_INVALID_ARG; }
    *bytes = sketch_csr_ws_bytes(m, d, true);
    return CSK_OK;
}

csk_status csk_sketch_csr_sparse(const int64_t* row_ptr, const int32_t* col, const float* val, int64_t m,
                                 int64_t n, int64_t nnz, const double* b, int64_t d, uint64_t seed,
                                 int64_t* at_row_ptr, int32_t* at_col, double* at_val, double* bt, double* nu2,
                                 void* ws, size_t ws_bytes, void* stream)
{
    g_err[0] = 0;
    if (!row_ptr || (nnz > 0 && (!col || !val))) { set_error("row_ptr / col / val required"); return CSK_ERR_INVALID_ARG; }
    if (m < 1 || n < 1 || d < 1 || nnz < 0 || m > INT32_MAX || d > INT32_MAX || nnz >= (int64_t)UINT32_MAX) {
        set_error("need 1 <= m, d < 2^31, n >= 1, 0 <= nnz < 2^32 - 1");
        return CSK_ERR_INVALID_ARG;
    }
    if (n > kMaxCsrSketchN) { set_error("n=%lld exceeds %lld", (long long)n, (long long)kMaxCsrSketchN); return CSK_ERR_UNSUPPORTED; }
    if (!at_row_ptr || (nnz > 0 && (!at_col || !at_val))) { set_error("at_row_ptr / at_col / at_val required"); return CSK_ERR_INVALID_ARG; }
    if ((b == nullptr) != (bt == nullptr)) { set_error("b and bt go together"); return CSK_ERR_INVALID_ARG; }
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) { set_error("workspace NULL or unaligned"); return CSK_ERR_INVALID_ARG; }
    size_t need = 0;
    csk_sketch_csr_sparse_workspace_size(m, n, d, &need);
    if (ws_bytes < need) { set_error("workspace: need %zu bytes, got %zu", need, ws_bytes); return CSK_ERR_WORKSPACE; }
    return sketch_csr_sparse_run(row_ptr, col, val, m, n, b, d, seed, at_row_ptr, at_col, at_val, bt, nu2, ws,
                                 ws_bytes, as_stream(stream));
}

csk_status csk_solve_csr_workspace_size(int64_t d, int64_t n, int64_t nnz, size_t* bytes)
{
    g_err[0] = 0;
    if (!bytes || d < 1 || n < 1 || nnz < 0) { set_error("bad sizes"); return CSK_ERR_INVALID_ARG; }
    *bytes = csr_solve_ws_bytes(d, 65536);
    return CSK_OK;
}

csk_status csk_solve_csr(const int64_t* at_row_ptr, const int32_t* at_col, const double* at_val, int64_t d,
                         int64_t n, int64_t nnz, const double* bt, const double* nu2, const double* x0, double* x,
                         const csk_solve_opts* opts, csk_solve_result* res, void* ws, size_t ws_bytes, void* stream)
{
    g_err[0] = 0;
    csk_status st = check_opts(opts);
    if (st != CSK_OK) return st;
    if (d < 1 || n < 1 || d > INT32_MAX || nnz < 0 || nnz > INT32_MAX) {
        set_error("need 1 <= d < 2^31, n >= 1, 0 <= nnz < 2^31");
        return CSK_ERR_INVALID_ARG;
    }
    if (n > kMaxCsrSolveN) { set_error("n=%lld exceeds %lld", (long long)n, (long long)kMaxCsrSolveN); return CSK_ERR_UNSUPPORTED; }
    if (!at_row_ptr || (nnz > 0 && (!at_col || !at_val))) { set_error("at_row_ptr / at_col / at_val required"); return CSK_ERR_INVALID_ARG; }
    if (!bt || !x || !res) { set_error("bt, x and res are required"); return CSK_ERR_INVALID_ARG; }
    if (opts->stop_mode == CSK_STOP_REL_ERR && !opts->x_ref) {
        set_error("CSK_STOP_REL_ERR needs opts->x_ref");
        return CSK_ERR_INVALID_ARG;
    }
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) { set_error("workspace NULL or unaligned"); return CSK_ERR_INVALID_ARG; }
    const int grid = csr_solve_grid(d, nnz, opts);
    if (ws_bytes < csr_solve_ws_bytes(d, grid)) {
        set_error("workspace: need %zu bytes, got %zu", csr_solve_ws_bytes(d, grid), ws_bytes);
        return CSK_ERR_WORKSPACE;
    }
    CsrSolveSys S{};
    S.rp = at_row_ptr;
    S.col = at_col;
    S.val = at_val;
    S.bt = bt;
    S.nu2 = nu2;
    S.x0 = x0;
    S.xref = opts->x_ref;
    S.x = x;
    S.res = res;
    S.nnz = nnz;
    S.d = (int32_t)d;
    S.n = (int32_t)n;
    S.stop_mode = opts->stop_mode;
    return csr_solve_run(S, opts, ws, ws_bytes, as_stream(stream));
}

csk_status csk_solve_workspace_size(int64_t d, int64_t n, csk_dtype at_dtype, size_t* bytes)
{
    g_err[0] = 0;
    if (!bytes || d < 1 || n < 1 || dtype_size(at_dtype) == 0) { set_error("bad sizes"); return CSK_ERR_INVALID_ARG; }
    *bytes = solve_ws_bytes(d, n, 65536);
    return CSK_OK;
}

namespace {

// Argument checks and launch of csk_solve and csk_solve_noalloc.  `ws` is
// the caller's workspace, or with from_scratch the library's static one
// (then ws_bytes is its size and a shortfall reports the scratch limit).
csk_status solve_entry(const void* At, csk_dtype at_dtype, int64_t ldat, const double* At64, int64_t ldat64,
                       int64_t d, int64_t n, const double* bt, const double* nu2, const double* x0, double* x,
                       const csk_solve_opts* opts, csk_solve_result* res, void* ws, size_t ws_bytes, void* stream,
                       bool from_scratch, const CsrRef* cref = nullptr)
{
    g_err[0] = 0;
    csk_status st = check_opts(opts);
    if (st != CSK_OK) return st;
    if (d < 1 || n < 1 || d > INT32_MAX) { set_error("need 1 <= d < 2^31, n >= 1"); return CSK_ERR_INVALID_ARG; }
    if (n > kMaxN) { set_error("n=%lld exceeds %lld", (long long)n, (long long)kMaxN); return CSK_ERR_UNSUPPORTED; }
    if (!bt || !x || !res) { set_error("bt, x and res are required"); return CSK_ERR_INVALID_ARG; }
    if (at_dtype == CSK_F64) {
        if (!At && !At64) { set_error("At is NULL"); return CSK_ERR_INVALID_ARG; }
        if (!At64) { At64 = static_cast<const double*>(At); ldat64 = ldat; }
        if (!At) { At = At64; ldat = ldat64; }
        if (ldat < n || ldat64 < n) { set_error("ldat < n"); return CSK_ERR_INVALID_ARG; }
    } else if (lp_ok(at_dtype)) {
        if (!At || !At64) { set_error("mixed precision needs At and At64"); return CSK_ERR_INVALID_ARG; }
        if (ldat < n || ldat64 < n) { set_error("leading dimension < n"); return CSK_ERR_INVALID_ARG; }
    } else {
        set_error("unknown dtype %d", at_dtype);
        return CSK_ERR_UNSUPPORTED;
    }
    if (opts->stop_mode == CSK_STOP_REL_ERR && !opts->x_ref) {
        set_error("CSK_STOP_REL_ERR needs opts->x_ref");
        return CSK_ERR_INVALID_ARG;
    }
    const SolvePlan plan = solve_plan(d, n, at_dtype, ldat, At, opts);
    const size_t need = solve_ws_bytes(d, n, plan.grid);
    if (from_scratch && need > ws_bytes) {
        set_error("csk_solve_noalloc: this solve needs %zu bytes of scratch, the library's static scratch holds %zu "
                  "(d = %lld too large; use csk_solve with a workspace)",
                  need, ws_bytes, (long long)d);
        return CSK_ERR_WORKSPACE;
    }
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) { set_error("workspace NULL or unaligned"); return CSK_ERR_INVALID_ARG; }
    if (ws_bytes < need) {
        set_error("workspace: need %zu bytes, got %zu", need, ws_bytes);
        return CSK_ERR_WORKSPACE;
    }
    SolveSys S{};
    S.At = At;
    S.At64 = At64;
    S.bt = bt;
    S.nu2 = nu2;
    S.x0 = x0;
    S.xref = opts->x_ref;
    S.x = x;
    S.res = res;
    S.ldat = ldat;
    S.ldat64 = ldat64;
    S.d = (int32_t)d;
    S.n = (int32_t)n;
    S.stop_mode = opts->stop_mode;
    return solve_run(S, at_dtype, opts, ws, ws_bytes, as_stream(stream), nullptr, cref);
}

// Workspace of csk_solve_csr_refresh: the bucket grouping, y (m doubles),
// the refresh's grid-barrier flags, the device copy of its descriptor, then
// the solve's own.
struct CsrRefreshLayout {
    size_t group, y, flags, ref, solve, total;
};
static CsrRefreshLayout csr_refresh_layout(int64_t m, int64_t d, int64_t n)
{
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    CsrRefreshLayout L{};
    L.group = up(group_ws_bytes(m, d));
    L.y = up((size_t)m * 8);
    L.flags = up((size_t)kRefreshFlags * 4);
    L.ref = up(sizeof(CsrRef));
    L.solve = solve_ws_bytes(d, n, 65536);
    L.total = L.group + L.y + L.flags + L.ref + L.solve;
    return L;
}

}  // namespace

csk_status csk_solve_csr_refresh_workspace_size(int64_t m, int64_t d, int64_t n, size_t* bytes)
{
    g_err[0] = 0;
    if (!bytes || m < 1 || d < 1 || n < 1) { set_error("bad sizes"); return CSK_ERR_INVALID_ARG; }
    *bytes = csr_refresh_layout(m, d, n).total;
    return CSK_OK;
}

csk_status csk_solve_csr_refresh(const void* At, csk_dtype at_dtype, int64_t ldat, const double* At64,
                                 int64_t ldat64, int64_t d, int64_t n, const int64_t* row_ptr, const int32_t* col,
                                 const float* val, int64_t m, const double* b, uint64_t seed, const double* bt,
                                 const double* nu2, const double* x0, double* x, const csk_solve_opts* opts,
                                 csk_solve_result* res, void* ws, size_t ws_bytes, void* stream)
{
    g_err[0] = 0;
    if (!lp_ok(at_dtype)) { set_error("the refresh from a CSR A needs a low-precision At"); return CSK_ERR_INVALID_ARG; }
    if (!row_ptr || !col || !val || !b) { set_error("row_ptr, col, val and b are required"); return CSK_ERR_INVALID_ARG; }
    if (m < 1 || m > INT32_MAX || d < 1 || d > INT32_MAX) { set_error("need 1 <= m, d < 2^31"); return CSK_ERR_INVALID_ARG; }
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) { set_error("workspace NULL or unaligned"); return CSK_ERR_INVALID_ARG; }
    const CsrRefreshLayout L = csr_refresh_layout(m, d, n);
    if (ws_bytes < L.total) {
        set_error("workspace: need %zu bytes, got %zu", L.total, ws_bytes);
        return CSK_ERR_WORKSPACE;
    }
    char* base = static_cast<char*>(ws);
    CsrRef R{};
    R.rp = row_ptr;
    R.col = col;
    R.val = val;
    R.b = b;
    R.y = reinterpret_cast<double*>(base + L.group);
    R.flags = reinterpret_cast<uint32_t*>(base + L.group + L.y);
    R.m = m;
    R.seed = seed;
    R.self = reinterpret_cast<CsrRef*>(base + L.group + L.y + L.flags);
    csk_status st = group_only(m, d, seed, base, L.group, &R.perm, &R.ptr, as_stream(stream));
    if (st != CSK_OK) return st;
    return solve_entry(At, at_dtype, ldat, At64, ldat64, d, n, bt, nu2, x0, x, opts, res,
                       base + L.group + L.y + L.flags + L.ref, L.solve, stream, false, &R);
}

csk_status csk_solve(const void* At, csk_dtype at_dtype, int64_t ldat, const double* At64, int64_t ldat64,
                     int64_t d, int64_t n, const double* bt, const double* nu2, const double* x0, double* x,
                     const csk_solve_opts* opts, csk_solve_result* res, void* ws, size_t ws_bytes, void* stream)
{
    return solve_entry(At, at_dtype, ldat, At64, ldat64, d, n, bt, nu2, x0, x, opts, res, ws, ws_bytes, stream,
                       false);
}

// ---- csk_solve without a workspace argument ---------------------------------
// The solve's workspace (exchange records, r_ref, computed norms) comes from
// one static device array.  In host code `scratch` names a host-side stand-in,
// not device memory: only the address hipGetSymbolAddress returns for the
// current device is ever passed to a kernel.  Each device holds its own copy
// of the array until the process ends; calls on one device share it.

static __device__ __align__(256) unsigned char scratch[CSK_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// The current device's copy of `scratch`, looked up once per device.
csk_status scratch_of_current_device(void** out)
{
    int dev = 0;
    const hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) return hip_fail(ge, "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices) {
        set_error("csk_solve_noalloc: device %d beyond the %d the library tracks", dev, kMaxScratchDevices);
        return CSK_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return CSK_OK;
}

}  // namespace

csk_status csk_solve_noalloc(const void* At, csk_dtype at_dtype, int64_t ldat, const double* At64, int64_t ldat64,
                             int64_t d, int64_t n, const double* bt, const double* nu2, const double* x0, double* x,
                             const csk_solve_opts* opts, csk_solve_result* res, void* stream)
{
    g_err[0] = 0;
    void* ws = nullptr;
    const csk_status e = scratch_of_current_device(&ws);
    if (e != CSK_OK) return e;
    return solve_entry(At, at_dtype, ldat, At64, ldat64, d, n, bt, nu2, x0, x, opts, res, ws,
                       (size_t)CSK_NOALLOC_SCRATCH_BYTES, stream, true);
}

// ---- Algorithm 1 as one HIP graph -------------------------------------------

struct csk_pipeline_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

csk_status csk_pipeline_capture(const void* A, csk_dtype a_dtype, int64_t m, int64_t n, int64_t lda, const double* b,
                                int64_t d, uint64_t seed, double* At64, int64_t ldat64, void* At_lp,
                                csk_dtype lp_dtype, int64_t ldat_lp, double* bt, double* nu2, const double* x0,
                                double* x, const csk_solve_opts* opts, csk_solve_result* res, void* ws_sketch,
                                size_t ws_sketch_bytes, void* ws_solve, size_t ws_solve_bytes, void* stream,
                                csk_pipeline* out)
{
    g_err[0] = 0;
    if (!out) { set_error("out is NULL"); return CSK_ERR_INVALID_ARG; }
    *out = nullptr;
    if (!stream) { set_error("capture needs a created stream, not the null stream"); return CSK_ERR_INVALID_ARG; }
    if (!b || !bt || !nu2 || !At64) { set_error("b, bt, nu2 and At64 are required"); return CSK_ERR_INVALID_ARG; }
    csk_status st = check_opts(opts);
    if (st != CSK_OK) return st;
    hipStream_t hs = as_stream(stream);
    CSK_HIP(hipStreamBeginCapture(hs, hipStreamCaptureModeThreadLocal));
    st = csk_sketch(A, a_dtype, m, n, lda, b, 1, 1, d, seed, At64, ldat64, At_lp, At_lp ? lp_dtype : CSK_F64,
                    ldat_lp, bt, 1, nu2, nullptr, nullptr, ws_sketch, ws_sketch_bytes, stream);
    if (st == CSK_OK)
        st = csk_solve(At_lp ? At_lp : At64, At_lp ? lp_dtype : CSK_F64, At_lp ? ldat_lp : ldat64, At64, ldat64, d, n,
                       bt, nu2, x0, x, opts, res, ws_solve, ws_solve_bytes, stream);
    hipGraph_t graph = nullptr;
    const hipError_t he = hipStreamEndCapture(hs, &graph);
    if (st != CSK_OK || he != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (st != CSK_OK) return st;  // the failing call's message stays
        return hip_fail(he, "hipStreamEndCapture");
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(ie, "hipGraphInstantiate");
    }
    *out = new csk_pipeline_s{graph, exec};
    return CSK_OK;
}

csk_status csk_pipeline_launch(csk_pipeline p, void* stream)
{
    g_err[0] = 0;
    if (!p) { set_error("pipeline is NULL"); return CSK_ERR_INVALID_ARG; }
    CSK_HIP(hipGraphLaunch(p->exec, as_stream(stream)));
    return CSK_OK;
}

csk_status csk_pipeline_destroy(csk_pipeline p)
{
    g_err[0] = 0;
    if (!p) return CSK_OK;
    const hipError_t e1 = hipGraphExecDestroy(p->exec);
    const hipError_t e2 = hipGraphDestroy(p->graph);
    delete p;
    if (e1 != hipSuccess) return hip_fail(e1, "hipGraphExecDestroy");
    if (e2 != hipSuccess) return hip_fail(e2, "hipGraphDestroy");
    return CSK_OK;
}

// ---- randomized selection rules ----------------------------------------------

namespace {
csk_status check_fp64_solve(const double* At, int64_t ldat, int64_t d, int64_t n, const double* bt, double* x,
                            const csk_solve_opts* opts, csk_solve_result* res, const void* ws)
{
    csk_status st = check_opts(opts);
    if (st != CSK_OK) return st;
    if (d < 1 || n < 1 || d > INT32_MAX) { set_error("need 1 <= d < 2^31, n >= 1"); return CSK_ERR_INVALID_ARG; }
    if (n > kMaxN) { set_error("n=%lld exceeds %lld", (long long)n, (long long)kMaxN); return CSK_ERR_UNSUPPORTED; }
    if (!At || !bt || !x || !res) { set_error("At, bt, x and res are required"); return CSK_ERR_INVALID_ARG; }
    if (ldat < n) { set_error("ldat < n"); return CSK_ERR_INVALID_ARG; }
    if (opts->stop_mode == CSK_STOP_REL_ERR && !opts->x_ref) {
        set_error("CSK_STOP_REL_ERR needs opts->x_ref");
        return CSK_ERR_INVALID_ARG;
    }
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) { set_error("workspace NULL or unaligned"); return CSK_ERR_INVALID_ARG; }
    return CSK_OK;
}
}  // namespace

csk_status csk_solve_rgrk_workspace_size(int64_t d, int64_t n, size_t* bytes)
{
    g_err[0] = 0;
    if (!bytes || d < 1 || n < 1) { set_error("bad sizes"); return CSK_ERR_INVALID_ARG; }
    *bytes = solve_rgrk_ws_bytes(d, n, 65536);
    return CSK_OK;
}

csk_status csk_solve_rgrk(const double* At, int64_t ldat, int64_t d, int64_t n, const double* bt, const double* nu2,
                          const double* x0, double* x, double theta, uint64_t sel_seed, const csk_solve_opts* opts,
                          csk_solve_result* res, void* ws, size_t ws_bytes, void* stream)
{
    g_err[0] = 0;
    csk_status st = check_fp64_solve(At, ldat, d, n, bt, x, opts, res, ws);
    if (st != CSK_OK) return st;
    if (!(theta >= 0.0 && theta <= 1.0)) { set_error("theta must lie in [0, 1]"); return CSK_ERR_INVALID_ARG; }
    const SolvePlan plan = solve_plan(d, n, CSK_F64, ldat, At, opts);
    if (ws_bytes < solve_rgrk_ws_bytes(d, n, plan.grid)) {
        set_error("workspace: need %zu bytes, got %zu", solve_rgrk_ws_bytes(d, n, plan.grid), ws_bytes);
        return CSK_ERR_WORKSPACE;
    }
    SolveSys S{};
    S.At = At;
    S.At64 = At;
    S.bt = bt;
    S.nu2 = nu2;
    S.x0 = x0;
    S.xref = opts->x_ref;
    S.x = x;
    S.res = res;
    S.ldat = ldat;
    S.ldat64 = ldat;
    S.d = (int32_t)d;
    S.n = (int32_t)n;
    S.stop_mode = opts->stop_mode;
    return solve_rgrk_run(S, opts, theta, sel_seed, ws, ws_bytes, as_stream(stream));
}

csk_status csk_solve_rk_workspace_size(int64_t d, int64_t n, size_t* bytes)
{
    g_err[0] = 0;
    if (!bytes || d < 1 || n < 1) { set_error("bad sizes"); return CSK_ERR_INVALID_ARG; }
    *bytes = solve_rk_ws_bytes(d);
    return CSK_OK;
}

csk_status csk_solve_rk(const double* At, int64_t ldat, int64_t d, int64_t n, const double* bt, const double* nu2,
                        const double* x0, double* x, uint64_t sel_seed, const csk_solve_opts* opts,
                        csk_solve_result* res, void* ws, size_t ws_bytes, void* stream)
{
    g_err[0] = 0;
    csk_status st = check_fp64_solve(At, ldat, d, n, bt, x, opts, res, ws);
    if (st != CSK_OK) return st;
    if (opts->stop_mode != CSK_STOP_REL_ERR) {
        set_error("randomized Kaczmarz forms one residual per iteration: stop_mode must be CSK_STOP_REL_ERR");
        return CSK_ERR_INVALID_ARG;
    }
    if (ws_bytes < solve_rk_ws_bytes(d)) {
        set_error("workspace: need %zu bytes, got %zu", solve_rk_ws_bytes(d), ws_bytes);
        return CSK_ERR_WORKSPACE;
    }
    return solve_rk_run(At, ldat, d, n, bt, nu2, x0, x, opts, sel_seed, res, ws, ws_bytes, as_stream(stream));
}

// ---- tuning of the persistent solve's launch shape --------------------------

csk_status csk_tune_solve_workspace_size(int64_t d, int64_t n, csk_dtype at_dtype, size_t* bytes)
{
    g_err[0] = 0;
    if (!bytes || d < 1 || n < 1 || dtype_size(at_dtype) == 0) { set_error("bad sizes"); return CSK_ERR_INVALID_ARG; }
    Carve c(nullptr);
    c.take<char>(solve_ws_bytes(d, n, 65536));
    c.take<double>(n);                 // x of the trial runs
    c.take<csk_solve_result>(1);
    *bytes = c.bytes();
    return CSK_OK;
}

csk_status csk_tune_solve(const void* At, csk_dtype at_dtype, int64_t ldat, const double* At64, int64_t ldat64,
                          int64_t d, int64_t n, const double* bt, const double* nu2, int32_t trial_iters,
                          csk_tune_entry* best, void* ws, size_t ws_bytes, void* stream)
{
    g_err[0] = 0;
    if (d < 1 || n < 1 || d > INT32_MAX) { set_error("need 1 <= d < 2^31, n >= 1"); return CSK_ERR_INVALID_ARG; }
    if (n > kMaxN) { set_error("n=%lld exceeds %lld", (long long)n, (long long)kMaxN); return CSK_ERR_UNSUPPORTED; }
    if (!bt) { set_error("bt is required"); return CSK_ERR_INVALID_ARG; }
    if (trial_iters < 1 || trial_iters > 1000000) { set_error("trial_iters out of range"); return CSK_ERR_INVALID_ARG; }
    if (at_dtype == CSK_F64) {
        if (!At && !At64) { set_error("At is NULL"); return CSK_ERR_INVALID_ARG; }
        if (!At64) { At64 = static_cast<const double*>(At); ldat64 = ldat; }
        if (!At) { At = At64; ldat = ldat64; }
    } else if (lp_ok(at_dtype)) {
        if (!At || !At64) { set_error("mixed precision needs At and At64"); return CSK_ERR_INVALID_ARG; }
    } else {
        set_error("unknown dtype %d", at_dtype);
        return CSK_ERR_UNSUPPORTED;
    }
    if (ldat < n || ldat64 < n) { set_error("leading dimension < n"); return CSK_ERR_INVALID_ARG; }
    size_t need = 0;
    csk_tune_solve_workspace_size(d, n, at_dtype, &need);
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) { set_error("workspace NULL or unaligned"); return CSK_ERR_INVALID_ARG; }
    if (ws_bytes < need) { set_error("workspace: need %zu bytes, got %zu", need, ws_bytes); return CSK_ERR_WORKSPACE; }
    Carve c(ws);
    void* sws = c.take<char>(solve_ws_bytes(d, n, 65536));
    double* x = c.take<double>(n);
    csk_solve_result* res = c.take<csk_solve_result>(1);
    hipStream_t stm = as_stream(stream);

    // Candidates: one workgroup (while the matrix is small), then 64, 128,
    // 192 and one per CU, each with the lanes-per-row splits whose padded
    // row length is within 25% of the best.
    const int cus = device_cu_count();
    const int64_t gmax = std::min<int64_t>(cus, std::max<int64_t>(1, (d + 15) / 16));
    std::vector<int> grids;
    if (d * n * (int64_t)dtype_size(at_dtype) <= (int64_t)(4 << 20)) grids.push_back(1);
    for (int g : {64, 128, 192, cus})
        if (g >= 2 && g <= gmax && std::find(grids.begin(), grids.end(), g) == grids.end()) grids.push_back(g);
    if (grids.empty()) grids.push_back((int)std::max<int64_t>(1, gmax));
    const int vw = solve_vw(at_dtype, ldat, At);
    const int vw_eff = (vw > 1 && (reinterpret_cast<uintptr_t>(At64) & 15u) == 0 && (ldat64 * 8) % 16 == 0) ? vw : 1;
    const int64_t per_lane = (int64_t)vw_eff * chunk_k_of(at_dtype);
    int64_t best_cover = INT64_MAX;
    for (int l : {64, 16, 4}) best_cover = std::min(best_cover, (n + l * per_lane - 1) / (l * per_lane) * l * per_lane);
    std::vector<int> lprs;
    for (int l : {64, 16, 4})
        if ((n + l * per_lane - 1) / (l * per_lane) * l * per_lane * 4 <= best_cover * 5) lprs.push_back(l);

    SolveSys S{};
    S.At = At;
    S.At64 = At64;
    S.bt = bt;
    S.nu2 = nu2;
    S.x = x;
    S.res = res;
    S.ldat = ldat;
    S.ldat64 = ldat64;
    S.d = (int32_t)d;
    S.n = (int32_t)n;
    S.stop_mode = CSK_STOP_REL_RESID;
    csk_solve_opts o{};
    o.tol = 0.0;  // never converged: every candidate runs trial_iters iterations
    o.maxit = trial_iters;
    o.stop_mode = CSK_STOP_REL_RESID;
    o.refresh_every = 64;
    o.check_every = 256;
    o.single_wg = -1;

    hipEvent_t e0, e1;
    CSK_HIP(hipEventCreate(&e0));
    CSK_HIP(hipEventCreate(&e1));
    csk_tune_entry pick{0, 0, 0.0};
    csk_status r = CSK_OK;
    for (int g : grids) {
        for (int l : lprs) {
            SolvePlan plan;
            plan.block = 512;
            plan.vw = vw_eff;
            plan.lpr = l;
            plan.grid = g;
            // one untimed run (first launch of the shape), then one timed
            r = solve_run(S, at_dtype, &o, sws, solve_ws_bytes(d, n, 65536), stm, &plan);
            if (r != CSK_OK) break;
            if (hipEventRecord(e0, stm) != hipSuccess) { set_error("hipEventRecord failed"); r = CSK_ERR_DEVICE; break; }
            r = solve_run(S, at_dtype, &o, sws, solve_ws_bytes(d, n, 65536), stm, &plan);
            if (r != CSK_OK) break;
            if (hipEventRecord(e1, stm) != hipSuccess) { set_error("hipEventRecord failed"); r = CSK_ERR_DEVICE; break; }
            if (hipEventSynchronize(e1) != hipSuccess) { set_error("tuning run failed"); r = CSK_ERR_DEVICE; break; }
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                set_error("hipEventElapsedTime failed");
                r = CSK_ERR_DEVICE;
                break;
            }
            const double us = 1e3 * ms / trial_iters;
            if (pick.grid == 0 || us < pick.us_per_iter) pick = csk_tune_entry{g, l, us};
        }
        if (r != CSK_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != CSK_OK) return r;
    tune_store(d, n, at_dtype, vw, pick.grid, pick.lanes_per_row, pick.us_per_iter);
    if (best) *best = pick;
    return CSK_OK;
}

csk_status csk_tune_lookup(int64_t d, int64_t n, csk_dtype at_dtype, int32_t vector_rows, csk_tune_entry* out)
{
    g_err[0] = 0;
    if (!out || d < 1 || n < 1 || dtype_size(at_dtype) == 0) { set_error("bad arguments"); return CSK_ERR_INVALID_ARG; }
    int g = 0, l = 0;
    double us = 0.0;
    const int vw = vector_rows ? 16 / (int)dtype_size(at_dtype) : 1;
    if (tune_lookup(d, n, at_dtype, vw, &g, &l, &us)) *out = csk_tune_entry{g, l, us};
    else *out = csk_tune_entry{0, 0, 0.0};
    return CSK_OK;
}

void csk_tune_clear(void) { tune_clear(); }

csk_status csk_solve_batched_workspace_size(const csk_system_desc* sys, int32_t nsys, csk_dtype a_dtype,
                                            csk_dtype lp_dtype, size_t* bytes)
{
    g_err[0] = 0;
    if (!bytes) { set_error("bytes is NULL"); return CSK_ERR_INVALID_ARG; }
    csk_status st = check_batch(sys, nsys, a_dtype, lp_dtype);
    if (st != CSK_OK) return st;
    const BatchLayout L = batch_layout(sys, nsys, lp_dtype);
    int64_t M = 0, D = 0, T = 0;
    for (int s = 0; s < nsys; ++s) {
        M += sys[s].m;
        D += sys[s].d;
        T += sys[s].d * sketch_chunks(sys[s].n, a_dtype);
    }
    Carve c(nullptr);
    c.take<char>(L.data_bytes);
    c.take<char>(sketch_ws_bytes(M, D, T, nsys));
    c.take<SolveSys>(nsys);
    c.take<int32_t>(nsys);
    c.take<uint32_t>(64);
    c.take<int32_t>(nsys + 1);
    c.take<int32_t>(nsys);
    c.take<char>(kBatchExchRecords * solve_exch_record_bytes());
    *bytes = c.bytes();
    return CSK_OK;
}

csk_status csk_solve_batched_sketch_loc(const csk_system_desc* sys, int32_t nsys, csk_dtype a_dtype,
                                        csk_dtype lp_dtype, int32_t s, csk_batched_sketch_loc* out)
{
    g_err[0] = 0;
    if (!out) { set_error("out is NULL"); return CSK_ERR_INVALID_ARG; }
    csk_status st = check_batch(sys, nsys, a_dtype, lp_dtype);
    if (st != CSK_OK) return st;
    if (s < 0 || s >= nsys) { set_error("system %d outside [0, %d)", s, nsys); return CSK_ERR_INVALID_ARG; }
    // the per-system data block is the workspace's first piece (offset 0)
    const BatchLayout L = batch_layout(sys, nsys, lp_dtype);
    out->at64 = L.off_64[s];
    out->at_lp = L.off_lp[s];
    out->bt = L.off_bt[s];
    out->nu2 = L.off_nu2[s];
    out->ld64 = L.ld_64[s];
    out->ld_lp = L.ld_lp[s];
    return CSK_OK;
}

namespace {

// The systems' shapes as a tune key: count and an FNV-1a hash of every (m, n, d).
std::string batched_tune_key(const csk_system_desc* sys, int32_t nsys, csk_dtype a_dtype, csk_dtype lp_dtype)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= static_cast<uint64_t>(v >> (8 * b)) & 0xFFu;
            h *= 1099511628211ull;
        }
    };
    for (int s = 0; s < nsys; ++s) {
        mix(sys[s].m);
        mix(sys[s].n);
        mix(sys[s].d);
    }
    return tune_key("batched|nsys=%d|shapes=%016llx|a=%d|lp=%d", nsys, (unsigned long long)h, (int)a_dtype, (int)lp_dtype);
}

csk_status batched_entry(const csk_system_desc* sys, int32_t nsys, csk_dtype a_dtype, csk_dtype lp_dtype,
                         const csk_solve_opts* opts, csk_solve_result* res, void* ws, size_t ws_bytes, void* stream,
                         int variant);

}  // namespace

csk_status csk_solve_batched(const csk_system_desc* sys, int32_t nsys, csk_dtype a_dtype, csk_dtype lp_dtype,
                             const csk_solve_opts* opts, csk_solve_result* res, void* ws, size_t ws_bytes,
                             void* stream)
{
    return batched_entry(sys, nsys, a_dtype, lp_dtype, opts, res, ws, ws_bytes, stream, -1);
}

namespace {
csk_status batched_entry(const csk_system_desc* sys, int32_t nsys, csk_dtype a_dtype, csk_dtype lp_dtype,
                         const csk_solve_opts* opts, csk_solve_result* res, void* ws, size_t ws_bytes, void* stream,
                         int variant)
{
    g_err[0] = 0;
    csk_status st = check_opts(opts);
    if (st != CSK_OK) return st;
    st = check_batch(sys, nsys, a_dtype, lp_dtype);
    if (st != CSK_OK) return st;
    if (!res) { set_error("res is NULL"); return CSK_ERR_INVALID_ARG; }
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) { set_error("workspace NULL or unaligned"); return CSK_ERR_INVALID_ARG; }
    size_t need = 0;
    csk_solve_batched_workspace_size(sys, nsys, a_dtype, lp_dtype, &need);
    if (ws_bytes < need) { set_error("workspace: need %zu bytes, got %zu", need, ws_bytes); return CSK_ERR_WORKSPACE; }
    hipStream_t stm = as_stream(stream);

    const BatchLayout L = batch_layout(sys, nsys, lp_dtype);
    int64_t M = 0, D = 0, T = 0, n_max = 0;
    for (int s = 0; s < nsys; ++s) {
        M += sys[s].m;
        D += sys[s].d;
        T += sys[s].d * sketch_chunks(sys[s].n, a_dtype);
        n_max = std::max(n_max, sys[s].n);
    }
    Carve c(ws);
    char* data = c.take<char>(L.data_bytes);
    const size_t sk_bytes = sketch_ws_bytes(M, D, T, nsys);
    char* sk_ws = c.take<char>(sk_bytes);
    SolveSys* d_sys = c.take<SolveSys>(nsys);
    int32_t* d_order = c.take<int32_t>(nsys);
    uint32_t* d_queue = c.take<uint32_t>(64);
    int32_t* d_item_off = c.take<int32_t>(nsys + 1);
    int32_t* d_exch_off = c.take<int32_t>(nsys);
    void* d_exch = c.take<char>(kBatchExchRecords * solve_exch_record_bytes());

    // 1. sketch every system in one pipeline
    std::vector<SketchJob> jobs(nsys);
    for (int s = 0; s < nsys; ++s) {
        SketchJob& J = jobs[s];
        J = SketchJob{};
        J.A = sys[s].A;
        J.B = sys[s].b;
        J.nrhs = 1;
        J.ldb = 1;
        J.m = sys[s].m;
        J.n = sys[s].n;
        J.lda = sys[s].lda;
        J.d = sys[s].d;
        J.seed = sys[s].seed;
        J.At64 = reinterpret_cast<double*>(data + L.off_64[s]);
        J.ldat64 = L.ld_64[s];
        J.Atlp = lp_dtype == CSK_F64 ? nullptr : data + L.off_lp[s];
        J.ldatlp = L.ld_lp[s];
        J.Bt = reinterpret_cast<double*>(data + L.off_bt[s]);
        J.ldbt = 1;
        J.nu2 = reinterpret_cast<double*>(data + L.off_nu2[s]);
        J.zpad = 1;  // the solve then needs no per-element masks
    }
    st = sketch_run(jobs.data(), nsys, a_dtype, lp_dtype == CSK_F64 ? (csk_dtype)0 : lp_dtype, nullptr, nullptr,
                    sk_ws, sk_bytes, stm);
    if (st != CSK_OK) return st;

    // 2. solver descriptors, largest estimated work first
    std::vector<SolveSys> hs(nsys);
    int64_t npad_max = 0, d_max = 0, n_max_s = 0;
    for (int s = 0; s < nsys; ++s) {
        SolveSys& S = hs[s];
        S = SolveSys{};
        S.At64 = jobs[s].At64;
        S.ldat64 = jobs[s].ldat64;
        S.At = lp_dtype == CSK_F64 ? static_cast<const void*>(S.At64) : jobs[s].Atlp;
        S.ldat = lp_dtype == CSK_F64 ? S.ldat64 : jobs[s].ldatlp;
        S.bt = jobs[s].Bt;
        S.nu2 = jobs[s].nu2;
        S.x0 = nullptr;
        S.xref = sys[s].x_ref;
        S.x = sys[s].x;
        S.rref = reinterpret_cast<double*>(data + L.off_rref[s]);
        S.res = res + s;
        S.d = (int32_t)sys[s].d;
        S.n = (int32_t)sys[s].n;
        S.stop_mode = sys[s].x_ref ? CSK_STOP_REL_ERR : CSK_STOP_REL_RESID;
        S.npad = (int32_t)solve_npad(sys[s].n, lp_dtype, solve_batch_lpr(), true);
        npad_max = std::max<int64_t>(npad_max, S.npad);
        d_max = std::max<int64_t>(d_max, S.d);
        n_max_s = std::max<int64_t>(n_max_s, S.n);
    }
    for (int k = 0; k < nsys; k += 24) {
        SysPack pack;
        const int cnt = std::min(24, nsys - k);
        for (int q = 0; q < cnt; ++q) pack.s[q] = hs[k + q];
        k_store_solve_descs<<<1, 64, 0, stm>>>(pack, cnt, d_sys + k);
        CSK_LAUNCH_CHECK("k_store_solve_descs");
    }
    std::vector<int32_t> order(nsys);
    std::iota(order.begin(), order.end(), 0);
    // longest estimated time first: iterations grow like n / (1 - sqrt(n/d))^2
    // (the split plan's model), each streaming d * n elements
    auto est = [&](int32_t i) {
        const double q = std::min(0.9, (double)sys[i].n / (double)sys[i].d);
        return (double)sys[i].d * (double)sys[i].n * (double)sys[i].n / ((1.0 - std::sqrt(q)) * (1.0 - std::sqrt(q)));
    };
    if (variant < 0) {
        TuneRec tr{};
        variant = (tune_get(batched_tune_key(sys, nsys, a_dtype, lp_dtype), &tr) && tr.a >= 0 && tr.a <= 4) ? tr.a : 0;
    }
    if (variant != 4) std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return est(a) > est(b); });
    BatchedPlan bp;
    bp.variant = variant;
    bp.order = order.data();
    bp.sys = hs.data();
    bp.npad_max = npad_max;
    bp.d_max = d_max;
    bp.n_max = n_max_s;
    bp.order_dev = d_order;
    bp.item_off_dev = d_item_off;
    bp.exch_off_dev = d_exch_off;
    bp.exch_dev = d_exch;
    bp.exch_records = kBatchExchRecords;
    bp.queue_dev = d_queue;
    return solve_batched_run(d_sys, nsys, bp, lp_dtype, opts, stm);
}
}  // namespace

csk_status csk_tune_batched(const csk_system_desc* sys, int32_t nsys, csk_dtype a_dtype, csk_dtype lp_dtype,
                            const csk_solve_opts* opts, csk_solve_result* res, csk_tune_report* report, void* ws,
                            size_t ws_bytes, void* stream)
{
    g_err[0] = 0;
    hipStream_t stm = as_stream(stream);
    hipEvent_t e0, e1;
    CSK_HIP(hipEventCreate(&e0));
    CSK_HIP(hipEventCreate(&e1));
    csk_tune_report R{-1, 0, 0.0, 0.0, 0};
    csk_status r = CSK_OK;
    for (int v = 0; v <= 4 && r == CSK_OK; ++v) {
        if (v == 0) {  // one untimed run first (the batch's first launch)
            r = batched_entry(sys, nsys, a_dtype, lp_dtype, opts, res, ws, ws_bytes, stream, 0);
            if (r != CSK_OK) break;
        }
        if (hipEventRecord(e0, stm) != hipSuccess) { set_error("hipEventRecord failed"); r = CSK_ERR_DEVICE; break; }
        r = batched_entry(sys, nsys, a_dtype, lp_dtype, opts, res, ws, ws_bytes, stream, v);
        if (r != CSK_OK) break;
        if (hipEventRecord(e1, stm) != hipSuccess) { set_error("hipEventRecord failed"); r = CSK_ERR_DEVICE; break; }
        if (hipEventSynchronize(e1) != hipSuccess) { set_error("tuning run failed"); r = CSK_ERR_DEVICE; break; }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { set_error("hipEventElapsedTime failed"); r = CSK_ERR_DEVICE; break; }
        const double us = ms * 1e3;
        ++R.candidates;
        if (v == 0) R.default_us = us;
        if (R.choice < 0 || us < R.us) {
            R.choice = v;
            R.us = us;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != CSK_OK) return r;
    tune_put(batched_tune_key(sys, nsys, a_dtype, lp_dtype), TuneRec{R.choice, 0, R.us});
    if (report) *report = R;
    return CSK_OK;
}

csk_status csk_tune_mrhs_workspace_size(int64_t d, int64_t n, int64_t nrhs, size_t* bytes)
{
    g_err[0] = 0;
    if (!bytes || d < 1 || n < 1 || nrhs < 1) { set_error("bad sizes"); return CSK_ERR_INVALID_ARG; }
    *bytes = mrhs_tune_ws_bytes(d, n, nrhs);
    return CSK_OK;
}

csk_status csk_tune_mrhs(const void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp, const double* At64, int64_t ldat64,
                         int64_t d, int64_t n, const double* Bt, int64_t nrhs, int64_t ldbt, const double* nu2,
                         int32_t trial_iters, csk_tune_report* report, void* ws, size_t ws_bytes, void* stream)
{
    g_err[0] = 0;
    if (d < 1 || n < 1 || nrhs < 1 || d > INT32_MAX || n > 1024) { set_error("need 1 <= d < 2^31, 1 <= n <= 1024, nrhs >= 1"); return CSK_ERR_INVALID_ARG; }
    if (!At_lp || !At64 || !Bt || !nu2) { set_error("At_lp, At64, Bt and nu2 are required"); return CSK_ERR_INVALID_ARG; }
    if (lp_dtype != CSK_BF16 && lp_dtype != CSK_F16) { set_error("lp_dtype must be BF16 or F16"); return CSK_ERR_UNSUPPORTED; }
    if (ldat_lp < n || ldat64 < n || ldbt < nrhs) { set_error("leading dimension too small"); return CSK_ERR_INVALID_ARG; }
    if (trial_iters < 1 || trial_iters > 1000000) { set_error("trial_iters out of range"); return CSK_ERR_INVALID_ARG; }
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) { set_error("workspace NULL or unaligned"); return CSK_ERR_INVALID_ARG; }
    return mrhs_tune(At_lp, lp_dtype, ldat_lp, At64, ldat64, d, n, Bt, nrhs, ldbt, nu2, trial_iters, report, ws,
                     ws_bytes, as_stream(stream));
}

csk_status csk_tune_save(const char* path)
{
    g_err[0] = 0;
    if (!path || !*path) { set_error("path is NULL or empty"); return CSK_ERR_INVALID_ARG; }
    if (!tune_save_file(path)) { set_error("cannot write the tune cache to %s", path); return CSK_ERR_INVALID_ARG; }
    return CSK_OK;
}

csk_status csk_tune_load(const char* path, int32_t* entries)
{
    g_err[0] = 0;
    if (!path || !*path) { set_error("path is NULL or empty"); return CSK_ERR_INVALID_ARG; }
    const int k = tune_load_file(path);
    if (entries) *entries = k;
    return CSK_OK;
}

csk_status csk_solve_mrhs_workspace_size(int64_t d, int64_t n, int64_t nrhs, size_t* bytes)
{
    g_err[0] = 0;
    if (!bytes || d < 1 || n < 1 || nrhs < 1) { set_error("bad sizes"); return CSK_ERR_INVALID_ARG; }
    *bytes = mrhs_ws_bytes(d, n, nrhs);
    return CSK_OK;
}

csk_status csk_solve_mrhs(const void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp, const double* At64,
                          int64_t ldat64, int64_t d, int64_t n, const double* Bt, int64_t nrhs, int64_t ldbt,
                          const double* nu2, const double* X0, double* X, int64_t ldx, const double* Xref,
                          int64_t ldxref, const csk_solve_opts* opts, csk_solve_result* res, void* ws,
                          size_t ws_bytes, void* stream)
{
    g_err[0] = 0;
    csk_status st = check_opts(opts);
    if (st != CSK_OK) return st;
    if (lp_dtype != CSK_BF16 && lp_dtype != CSK_F16) { set_error("lp_dtype must be BF16 or F16"); return CSK_ERR_UNSUPPORTED; }
    if (!At_lp || !At64 || !Bt || !X || !res || !nu2) { set_error("At_lp, At64, Bt, nu2, X and res are required"); return CSK_ERR_INVALID_ARG; }
    if (d < 1 || n < 1 || nrhs < 1 || d > INT32_MAX || nrhs > INT32_MAX) { set_error("bad sizes"); return CSK_ERR_INVALID_ARG; }
    if (n > 1024) { set_error("n=%lld exceeds 1024", (long long)n); return CSK_ERR_UNSUPPORTED; }
    if (ldat_lp < n || ldat64 < n || ldbt < nrhs || ldx < nrhs) { set_error("leading dimension too small"); return CSK_ERR_INVALID_ARG; }
    if (opts->stop_mode == CSK_STOP_REL_ERR && (!Xref || ldxref < nrhs)) { set_error("CSK_STOP_REL_ERR needs Xref"); return CSK_ERR_INVALID_ARG; }
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u)) { set_error("workspace NULL or unaligned"); return CSK_ERR_INVALID_ARG; }
    if (ws_bytes < mrhs_ws_bytes(d, n, nrhs)) { set_error("workspace: need %zu bytes, got %zu", mrhs_ws_bytes(d, n, nrhs), ws_bytes); return CSK_ERR_WORKSPACE; }
    return mrhs_run(At_lp, lp_dtype, ldat_lp, At64, ldat64, d, n, Bt, nrhs, ldbt, nu2, X0, X, ldx, Xref, ldxref,
                    opts, res, ws, ws_bytes, as_stream(stream));
}

}  // extern "C"
