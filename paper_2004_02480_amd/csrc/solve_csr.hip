// solve_csr.hip -- Algorithm 1, loop (maximal weighted residual Kaczmarz) on a
// sketched matrix held in CSR form.
//
// The sketch of a sparse A is sparse too: row j of At holds the union of the
// stored columns of the rows hashed to bucket j.  The residual product then
// reads the nnz(At) stored entries instead of all d * n, which at a few
// percent density is an order of magnitude fewer bytes per iteration.
//
// Same persistent design as the dense loop: one workgroup per CU, every
// iteration inside the kernel.  The rows are split into contiguous blocks of
// about equal weight (stored entries plus a fixed cost per row).  A workgroup
// keeps x, its block's row offsets, right-hand sides and squared norms in
// LDS, and as many of its block's stored entries as fit beside them (FP64
// values, 16-bit column indices); the rest of its entries are read from
// memory every iteration, several per lane in flight.  Lane groups of LPR
// lanes share a row.  Candidates, the stop measure and the flags go through
// the tagged-word exchange; the projection touches only the selected row's
// stored columns, and every workgroup applies it to its own copy of x.
#include "csk_grid.h"
#include "csk_solve_csr.h"

#include <algorithm>

namespace csk {
namespace {

constexpr int kNT = 512;
constexpr int kNW = kNT / kWave;
constexpr int kU = 8;                    // streamed entries per lane in flight
constexpr int kUL = 4;                   // resident entries per lane per LDS round
constexpr int kKR = 3;                   // register-resident rows per lane group
constexpr int kJ = 8;                    // register-resident entries per lane and row
constexpr size_t kLdsReserve = 2048;     // static LDS of the kernel, rounded up
enum : uint32_t {
    kFlagBadSplit = 8u,   // a row block larger than planned
    kFlagBadInput = 16u,  // rp[0] != 0 or rp[d] != nnz
};

struct CsrCtl {
    double tol2;
    int64_t maxit;
    const volatile int32_t* cancel;
    XRec* exch;            // [2][grid], tags zero at launch
    int32_t check_every;
    int32_t xslice;        // LDS doubles for the workgroup's slice of x_ref
    int32_t rows_cap;      // rows of the largest block
    int32_t res_cap;       // stored entries kept in LDS per workgroup
    int32_t row_weight;    // split weight of a row, in stored entries
    int32_t pad_;
    int64_t* trace;        // nullable: row projected at each iteration
};

// LDS carve: x, the slice of x_ref, resident values (16-byte aligned), row
// right-hand sides and squared norms, row offsets, resident column indices.
struct CsrLds {
    size_t sx, sxr, lval, lrhs, lnn, lrp, lcol, total;
};

__host__ __device__ inline size_t al_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

__host__ __device__ inline CsrLds csr_lds(int n, int xslice, int rows_cap, int res_cap)
{
    CsrLds o;
    size_t at = 0;
    o.sx = at;
    at += (size_t)n * 8;
    o.sxr = at;
    at += (size_t)xslice * 8;
    at = al_up(at, 16);
    o.lval = at;
    at += (size_t)res_cap * 8;
    o.lrhs = at;
    at += (size_t)rows_cap * 8;
    o.lnn = at;
    at += (size_t)rows_cap * 8;
    o.lrp = at;
    at += (size_t)(rows_cap + 1) * 4;
    o.lcol = at;
    at += (size_t)res_cap * 2;
    o.total = al_up(at, 16);
    return o;
}

// First row of workgroup w's block: the smallest r with
// rp[r] + rw * r >= floor(w * total / G), total = nnz + rw * d, where rw is
// the split weight of a row (the left side grows strictly with r, so the
// blocks tile [0, d) in order).  A block of R rows then has
// rw * (R - 1) < ceil(total / G) + 1, the host's bound on R.
__device__ int split_row(const int64_t* __restrict__ rp, int d, int64_t nnz, int rw, int w, int G)
{
    if (w <= 0) return 0;
    if (w >= G) return d;
    const int64_t total = nnz + (int64_t)rw * d;
    const int64_t t = total / G * w + (total % G) * w / G;
    int lo = 0, hi = d;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rp[mid] + (int64_t)rw * mid >= t) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

template <int LPR, bool GRID>
__global__ __launch_bounds__(kNT) void k_solve_csr(CsrSolveSys S, CsrCtl C)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ GridRed slots[kNW];
    __shared__ GridRed slots2[kNW];  // the exchange's reduction
    __shared__ int s_split[2];
    constexpr int NG = kNT / LPR;
    const int tid = threadIdx.x;
    const int q = tid % LPR;
    const int g = tid / LPR;
    const int wg = GRID ? (int)blockIdx.x : 0;
    const int G = GRID ? (int)gridDim.x : 1;
    const int n = S.n;
    const int d = S.d;
    const CsrLds lay = csr_lds(n, C.xslice, C.rows_cap, C.res_cap);
    double* sx = reinterpret_cast<double*>(smem + lay.sx);
    double* sxr = reinterpret_cast<double*>(smem + lay.sxr);
    double* lval = reinterpret_cast<double*>(smem + lay.lval);
    double* lrhs = reinterpret_cast<double*>(smem + lay.lrhs);
    double* lnn = reinterpret_cast<double*>(smem + lay.lnn);
    int32_t* lrp = reinterpret_cast<int32_t*>(smem + lay.lrp);
    uint16_t* lcol = reinterpret_cast<uint16_t*>(smem + lay.lcol);

    if (tid < 2) s_split[tid] = split_row(S.rp, d, S.nnz, C.row_weight, wg + tid, G);
    __syncthreads();
    const int r0 = s_split[0];
    int r1 = s_split[1];
    // Inconsistent row pointers or a block above the host's bound (which
    // cannot happen with consistent ones) end the solve at its first
    // exchange; the block then reads no entries.
    uint32_t plan_flags = (S.rp[0] != 0 || S.rp[d] != S.nnz) ? kFlagBadInput : 0u;
    if (r1 - r0 > C.rows_cap) plan_flags |= kFlagBadSplit;
    if (plan_flags) r1 = r0;
    const int nr = r1 - r0;
    const int64_t base = S.rp[r0];
    const int nres = (int)min<int64_t>(S.rp[r1] - base, (int64_t)C.res_cap);
    const int cols_per = (n + G - 1) / G;
    const int e0 = min(n, wg * cols_per);
    const int e1 = min(n, e0 + cols_per);

    for (int c = tid; c < n; c += kNT) sx[c] = S.x0 ? S.x0[c] : 0.0;
    if (S.xref)
        for (int c = e0 + tid; c < e1; c += kNT) sxr[c - e0] = S.xref[c];
    for (int i = tid; i <= nr; i += kNT) lrp[i] = (int32_t)(S.rp[r0 + i] - base);
    for (int i = tid; i < nr; i += kNT) {
        lrhs[i] = S.bt[r0 + i];
        lnn[i] = S.nu2[r0 + i];
    }
    for (int p = tid; p < nres; p += kNT) {
        lval[p] = S.val[base + p];
        lcol[p] = static_cast<uint16_t>(S.col[base + p]);
    }
    // ||x_ref||^2 and ||bt||^2, reduced identically by every workgroup
    GridRed q0 = red_identity();
    if (S.xref)
        for (int c = tid; c < n; c += kNT) q0.e2 += S.xref[c] * S.xref[c];
    for (int i = tid; i < d; i += kNT) q0.r2 += S.bt[i] * S.bt[i];
    q0 = block_red<kNT>(q0, slots);  // its barriers also publish the LDS fill
    const double xref2 = q0.e2;
    const double bt2 = q0.r2;
    const double tol2 = C.tol2;
    const bool rel_err = S.stop_mode == CSK_STOP_REL_ERR;
    const double* __restrict__ gval = S.val + base;
    const int32_t* __restrict__ gcol = S.col + base;
    // rsplit: rows [0, rsplit) of the block have all their entries in LDS.
    // Group g holds in registers, for the whole solve, its rows rsplit + g +
    // kr * NG (kr < kKR) from their first entry past the LDS prefix: lane q
    // has entries q + u * LPR (u < kJ); the rest of such a row is streamed.
    // Slots past a row's end hold zero values with column 0.
    int rsplit;
    {
        int lo = 0, hi = nr;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (lrp[mid + 1] > nres) hi = mid;
            else lo = mid + 1;
        }
        rsplit = lo;
    }
    double rv[kKR][kJ];
    int32_t rc[kKR][kJ];
#pragma unroll
    for (int kr = 0; kr < kKR; ++kr) {
        const int lr = rsplit + g + kr * NG;
        const bool on = lr < nr;
        const int s0 = on ? max(lrp[lr], nres) : 0;
        const int e = on ? lrp[lr + 1] : 0;
#pragma unroll
        for (int u = 0; u < kJ; ++u) {
            const int p = s0 + q + u * LPR;
            const bool ok = on && p < e;
            rv[kr][u] = ok ? gval[p] : 0.0;
            rc[kr][u] = ok ? gcol[p] : 0;
        }
    }

    int32_t status = CSK_NOT_CONVERGED;
    double meas = NAN;
    int64_t k = 0;
    for (;; ++k) {
        GridRed loc = red_identity();
        loc.flags = plan_flags;
        // residuals of the block's rows, in three parts: rows whose entries
        // are all in LDS, then each group's kKR rows held in registers (with
        // the LDS part of the row that straddles the resident prefix), then
        // rows beyond those, streamed from memory kU entries per lane at a
        // time (addresses clamped into the row, values masked)
        auto lds_part = [&](int s0, int em, double acc) {
            for (int p0 = s0 + q; p0 < em; p0 += kUL * LPR) {
                double lv[kUL];
                int lc[kUL];
#pragma unroll
                for (int u = 0; u < kUL; ++u) {
                    const int p = min(p0 + u * LPR, em - 1);
                    lv[u] = lval[p];
                    lc[u] = lcol[p];
                }
#pragma unroll
                for (int u = 0; u < kUL; ++u) acc += (p0 + u * LPR < em) ? lv[u] * sx[lc[u]] : 0.0;
            }
            return acc;
        };
        auto stream_part = [&](int ps, int e, double acc) {
            for (int p0 = ps + q; p0 < e; p0 += kU * LPR) {
                double v[kU];
                int32_t cv[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int p = min(p0 + u * LPR, e - 1);
                    v[u] = gval[p];
                    cv[u] = gcol[p];
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) acc += (p0 + u * LPR < e) ? v[u] * sx[cv[u]] : 0.0;
            }
            return acc;
        };
        auto finish = [&](int lr, double acc) {
            const double sum = group_sum_t<double, LPR>(acc);
            const int row = r0 + lr;
            const double r = lrhs[lr] - sum;
            const double nn = lnn[lr];
            if (q == 0) loc.r2 += r * r;
            if (nn > 0.0) {
                const double score = (r * r) / nn;
                if (!isfinite(score)) {
                    loc.flags |= kFlagNonfinite;
                } else if (cand_better(score, (uint32_t)row, loc.score, loc.idx)) {
                    loc.score = score;
                    loc.r = r / nn;
                    loc.idx = (uint32_t)row;
                }
            } else if (isnan(nn)) {
                loc.flags |= kFlagNonfinite;
            }
        };
        for (int lr = g; lr < rsplit; lr += NG) finish(lr, lds_part(lrp[lr], lrp[lr + 1], 0.0));
#pragma unroll
        for (int kr = 0; kr < kKR; ++kr) {
            const int lr = rsplit + g + kr * NG;
            if (lr < nr) {
                const int s0 = lrp[lr], e = lrp[lr + 1];
                double acc = lds_part(s0, min(e, nres), 0.0);
#pragma unroll
                for (int u = 0; u < kJ; ++u) acc += rv[kr][u] * sx[rc[kr][u]];
                finish(lr, stream_part(max(s0, nres) + kJ * LPR, e, acc));
            }
        }
        for (int lr = rsplit + g + kKR * NG; lr < nr; lr += NG)
            finish(lr, stream_part(lrp[lr], lrp[lr + 1], 0.0));
        if (S.xref)
            for (int c = e0 + tid; c < e1; c += kNT) {
                const double ex = sx[c] - sxr[c - e0];
                loc.e2 += ex * ex;
            }
        if (wg == 0 && tid == 0 && C.cancel && (k % C.check_every) == 0 && *C.cancel != 0)
            loc.flags |= kFlagCancel;
        GridRed tot = block_red1<kNT>(loc, slots);
        if constexpr (GRID) tot = exchange<kNT>(tot, C.exch, wg, G, k, slots2, rel_err);

        if (tot.flags & kFlagBadInput) { status = CSK_ERR_INVALID_ARG; break; }
        // stop test on x_k (top of iteration k)
        bool conv;
        if (rel_err) {
            meas = xref2 > 0.0 ? tot.e2 / xref2 : tot.e2;
            conv = xref2 > 0.0 ? (tot.e2 / xref2 <= tol2) : (tot.e2 <= tol2);
        } else {
            meas = bt2 > 0.0 ? tot.r2 / bt2 : tot.r2;
            conv = tot.r2 <= tol2 * bt2;
        }
        if (conv) { status = CSK_OK; break; }
        if (k == C.maxit) { status = CSK_NOT_CONVERGED; break; }
        if (tot.flags & (kFlagTimeout | kFlagBadSplit)) { status = CSK_ERR_DEVICE; break; }
        if (tot.flags & kFlagCancel) { status = CSK_CANCELLED; break; }
        if (tot.flags & kFlagNonfinite) { status = CSK_ERR_NONFINITE; break; }
        if (tot.idx == kNoRow) { status = CSK_ERR_DEGENERATE; break; }
        if (tot.idx >= (uint32_t)d) { status = CSK_ERR_DEVICE; break; }  // never dereference a bad row

        // projection onto row i_k: its stored columns are distinct, so each
        // thread updates its own entries of x
        const double alpha = tot.r;
        if (C.trace && wg == 0 && tid == 0) C.trace[k] = tot.idx;
        const int64_t a0 = S.rp[tot.idx], a1 = S.rp[tot.idx + 1];
        for (int64_t p = a0 + tid; p < a1; p += kNT) {
            const int c = S.col[p];
            sx[c] = sx[c] + alpha * S.val[p];
        }
        __syncthreads();
    }

    if (wg == 0) {
        for (int c = tid; c < n; c += kNT) S.x[c] = sx[c];
        if (tid == 0 && S.res) {
            S.res->iters = k;
            S.res->status = status;
            S.res->fp64_fallback = 0;
            S.res->final_measure = meas;
            S.res->refreshes = 0;
        }
    }
}

// Squared norms of the stored rows, when the caller has none.
__global__ __launch_bounds__(256) void k_csr_norms2(const int64_t* __restrict__ rp, const double* __restrict__ val,
                                                    int d, double* __restrict__ nu2)
{
    const int lane = threadIdx.x & (kWave - 1);
    for (int row = blockIdx.x * 4 + threadIdx.x / kWave; row < d; row += gridDim.x * 4) {
        double s = 0.0;
        for (int64_t p = rp[row] + lane; p < rp[row + 1]; p += kWave) s += val[p] * val[p];
        s = wave_sum(s);
        if (lane == 0) nu2[row] = s;
    }
}

__global__ void k_zero_exch(uint32_t* p, int64_t words)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < words; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = 0u;
}

template <int LPR>
csk_status launch(const CsrSolveSys& S, CsrCtl C, int grid, size_t shm, hipStream_t st)
{
    if (grid <= 1) {
        auto kern = k_solve_csr<LPR, false>;
        CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        kern<<<1, kNT, shm, st>>>(S, C);
        CSK_LAUNCH_CHECK("k_solve_csr");
        return CSK_OK;
    }
    auto kern = k_solve_csr<LPR, true>;
    CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    int per_cu = 0;
    CSK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), kNT, shm));
    const int cap = per_cu * device_cu_count();
    if (grid > cap) {
        set_error("persistent grid of %d workgroups exceeds the %d co-resident ones", grid, cap);
        return CSK_ERR_UNSUPPORTED;
    }
    CsrSolveSys s_arg = S;
    CsrCtl c_arg = C;
    void* args[] = {&s_arg, &c_arg};
    CSK_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(kNT), args,
                                       (unsigned)shm, st));
    return CSK_OK;
}

}  // namespace

int csr_solve_grid(int64_t d, int64_t nnz, const csk_solve_opts* o)
{
    int grid;
    if (o && o->single_wg == 1) grid = 1;
    else if (o && o->grid > 0) grid = o->grid;
    else {
        // one workgroup while the entries fit comfortably in one CU's share
        // of L2, else about 4096 stored entries per workgroup, up to one per CU
        const int64_t want = (nnz + 4095) / 4096;
        grid = (nnz * 12 <= (int64_t)(1 << 20) && !(o && o->single_wg == 0))
                   ? 1
                   : (int)std::max<int64_t>(2, std::min<int64_t>(device_cu_count(), want));
    }
    return (int)std::max<int64_t>(1, std::min<int64_t>(grid, d));
}

// Lanes per row: the narrowest group whose register rows (kJ entries per
// lane) hold a mean row.  A lane group walks its rows one after another, so
// narrow groups keep more rows in flight per workgroup; on the 1e6 x 5000,
// d = 50000 sketch (100 entries per row) 16 lanes take 12.3 us per
// iteration against 14.4 (4 lanes, rows overflowing the registers) and 22.9
// (64 lanes).
int csr_solve_lpr(int64_t d, int64_t nnz)
{
    const int64_t mean = (nnz + d - 1) / std::max<int64_t>(d, 1);
    return mean <= 4 * kJ ? 4 : mean <= 16 * kJ ? 16 : 64;
}

size_t csr_solve_ws_bytes(int64_t d, int grid)
{
    Carve c(nullptr);
    c.take<XRec>(2 * (size_t)std::max(grid, 1));
    c.take<double>(d);  // nu2 when not supplied
    return c.bytes();
}

csk_status csr_solve_run(const CsrSolveSys& sys_in, const csk_solve_opts* o, void* ws, size_t ws_bytes,
                         hipStream_t st)
{
    CsrSolveSys S = sys_in;
    const int grid = csr_solve_grid(S.d, S.nnz, o);
    const int lpr = csr_solve_lpr(S.d, S.nnz);
    Carve c(ws);
    CsrCtl C{};
    C.tol2 = o->tol * o->tol;
    C.maxit = o->maxit;
    C.cancel = o->cancel;
    C.check_every = o->check_every > 0 ? o->check_every : 256;
    C.trace = o->trace_idx;
    C.exch = c.take<XRec>(2 * (size_t)grid);
    double* nu2_ws = c.take<double>(S.d);
    if (c.bytes() > ws_bytes) {
        set_error("solve workspace too small: need %zu bytes, got %zu", c.bytes(), ws_bytes);
        return CSK_ERR_WORKSPACE;
    }
    // LDS plan.  A row weighs as much as the mean row's entries (at least
    // 4), so a block holds at most about twice the mean number of rows
    // (rw * (rows - 1) < ceil(total / G) + 1 bounds rows_cap); the rest of
    // LDS after x, the x_ref slice and the row data holds resident entries
    // (10 bytes each).
    C.row_weight = (int32_t)std::max<int64_t>(4, std::min<int64_t>(1 << 20, (S.nnz + S.d - 1) / S.d));
    const int64_t total = S.nnz + (int64_t)C.row_weight * S.d;
    const int64_t per = (total + grid - 1) / grid;
    C.rows_cap = (int32_t)std::min<int64_t>(S.d, per / C.row_weight + 2);
    C.xslice = S.xref ? (S.n + grid - 1) / grid : 0;
    const size_t cap = (size_t)device_max_lds() - kLdsReserve;
    const size_t fixed = csr_lds(S.n, C.xslice, C.rows_cap, 0).total;
    if (fixed + 64 > cap) {
        set_error("the CSR solve needs %zu bytes of LDS per workgroup before any resident entry "
                  "(n = %d, %d rows per block): use more workgroups", fixed, S.n, C.rows_cap);
        return CSK_ERR_UNSUPPORTED;
    }
    int64_t res = (int64_t)((cap - fixed - 32) / 10) & ~int64_t(7);
    res = std::min<int64_t>(res, (per + 7) & ~int64_t(7));
    C.res_cap = (int32_t)std::max<int64_t>(0, res);
    while (C.res_cap > 0 && csr_lds(S.n, C.xslice, C.rows_cap, C.res_cap).total > cap) C.res_cap -= 8;
    const size_t shm = csr_lds(S.n, C.xslice, C.rows_cap, C.res_cap).total;

    if (S.nu2 == nullptr) {
        k_csr_norms2<<<std::min(4096, (S.d + 3) / 4), 256, 0, st>>>(S.rp, S.val, S.d, nu2_ws);
        CSK_LAUNCH_CHECK("k_csr_norms2");
        S.nu2 = nu2_ws;
    }
    if (grid > 1) {
        const int64_t words = (int64_t)2 * grid * (int64_t)sizeof(XRec) / 4;
        k_zero_exch<<<(int)std::min<int64_t>(64, (words + 255) / 256), 256, 0, st>>>(
            reinterpret_cast<uint32_t*>(C.exch), words);
        CSK_LAUNCH_CHECK("k_zero_exch");
    }
    switch (lpr) {
    case 4: return launch<4>(S, C, grid, shm, st);
    case 16: return launch<16>(S, C, grid, shm, st);
    default: return launch<64>(S, C, grid, shm, st);
    }
}

}  // namespace csk
