// solve.hip -- Algorithm 1, loop: maximal weighted residual Kaczmarz (MWRK)
// on the sketched system (At, bt), as one persistent kernel.
//
// Every iteration k, with no host round trip:
//   1. residual r_i = bt_i - At^(i) x_k for the workgroup's own block of rows
//      (bandwidth-bound: At is streamed once per iteration; x sits in LDS);
//   2. weighted score r_i^2 / ||At^(i)||^2 (the square of the paper's
//      |r_i| / ||At^(i)||, same argmax), best row of the workgroup through
//      wavefront butterflies and LDS;
//   3. (grid path) one grid-wide barrier: each workgroup publishes its best
//      row, partial ||r||^2 and partial ||x - x_ref||^2, then every workgroup
//      reduces all records in the same fixed order, so all agree on i_k and
//      on the stop decision without a second barrier;
//   4. stop test (Section 3's RES, or the sketched residual), then the
//      projection x += (r_{i_k} / ||At^(i_k)||^2) At^(i_k)^T, applied by every
//      workgroup to its own copy of x (each thread owns fixed columns).
// Mixed precision: At is held in FP32/FP16/BF16 and the FP64 sketch At64 is
// kept beside it.  Every `refresh_every` iterations the exact FP64 residual
// r_ref = bt - At64 x is formed and x_ref = x saved; in between the residual
// is r_ref - At (x - x_ref) with FP32 accumulation, so each inner iteration
// streams 2-4x fewer bytes.  Scores and projections use the FP64 rows.
// Small systems run the same loop in one workgroup (no grid barrier); the
// batched kernel hands whole systems to workgroups from an atomic queue.
#include "csk_solve.h"
#include "csk_grid.h"

#include <algorithm>
#include <cmath>

namespace csk {
namespace {

constexpr int kNT = 512;        // threads per workgroup
constexpr int kNW = kNT / kWave;
using Red = GridRed;
constexpr int kCPT = 16;        // owned columns per thread: n <= kNT * kCPT
constexpr int kR = 2;           // rows in flight per lane group


struct tag_f64 { using storage = double; };

struct Ctl {
    double tol2;
    int64_t maxit;
    const volatile int32_t* cancel;
    Red* exch;             // [2][grid]
    uint32_t* barrier;     // arrival counter, zero at launch
    uint32_t* queue;       // batched work queue, zero at launch
    const int32_t* order;  // batched: queue position -> system
    int32_t refresh_every, check_every;
    int32_t nsys;
    int32_t pad_;
};

template <class T, int W>
__device__ __forceinline__ T group_sum_t(T v)
{
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
    return v;
}

// 16-byte vector loads of At, widened to the accumulation type.
template <class Tag> struct Elem;
template <> struct Elem<tag_f64> {
    using S = double; using Acc = double; static constexpr int kVec = 2;
    __device__ static Acc one(const S* p) { return *p; }
    __device__ static void vec(const S* p, Acc* o) { const double2 v = *reinterpret_cast<const double2*>(p); o[0] = v.x; o[1] = v.y; }
};
template <> struct Elem<tag_f32> {
    using S = float; using Acc = float; static constexpr int kVec = 4;
    __device__ static Acc one(const S* p) { return *p; }
    __device__ static void vec(const S* p, Acc* o) { const float4 v = *reinterpret_cast<const float4*>(p); o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w; }
};
template <class Tag> struct Elem16 {
    using S = uint16_t; using Acc = float; static constexpr int kVec = 8;
    __device__ static Acc one(const S* p) { return widen<Tag>(*p); }
    __device__ static void vec(const S* p, Acc* o)
    {
        const uint4 v = *reinterpret_cast<const uint4*>(p);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            o[2 * k] = widen<Tag>(static_cast<uint16_t>(w[k] & 0xFFFFu));
            o[2 * k + 1] = widen<Tag>(static_cast<uint16_t>(w[k] >> 16));
        }
    }
};
template <> struct Elem<tag_f16> : Elem16<tag_f16> {};
template <> struct Elem<tag_bf16> : Elem16<tag_bf16> {};

// Residuals, candidates and partial ||r||^2 for rows [r0, r1) of the
// workgroup.  Lane groups of LPR lanes share a row; kR rows are in flight
// per group.  xs is the operand vector in LDS (x for FP64, x - x_ref in FP32
// for the low-precision product); rhs is bt (exact) or r_ref (inner).  When
// rout is non-null the residuals are stored there (a refresh).
template <class Tag, bool VEC, int LPR>
__device__ __forceinline__ void residual_rows(const typename Elem<Tag>::S* __restrict__ A, int64_t lda,
                                              int n, int r0, int r1,
                                              const typename Elem<Tag>::Acc* __restrict__ xs,
                                              const double* __restrict__ rhs, double* __restrict__ rout,
                                              const double* __restrict__ nu2, Red& loc)
{
    using E = Elem<Tag>;
    using Acc = typename E::Acc;
    constexpr int VW = VEC ? E::kVec : 1;
    constexpr int NG = kNT / LPR;
    const int q = threadIdx.x % LPR;
    const int g = threadIdx.x / LPR;
    constexpr int step = LPR * VW;
    const int K = (n + step - 1) / step;
    for (int base = r0 + g; base < r1; base += NG * kR) {
        Acc acc[kR];
#pragma unroll
        for (int u = 0; u < kR; ++u) acc[u] = Acc(0);
#pragma unroll 4
        for (int k = 0; k < K; ++k) {
            const int col = k * step + q * VW;
            if (col + VW <= n) {
                Acc xv[VW];
#pragma unroll
                for (int e = 0; e < VW; ++e) xv[e] = xs[col + e];
#pragma unroll
                for (int u = 0; u < kR; ++u) {
                    const int row = base + u * NG;
                    if (row < r1) {
                        Acc a[VW];
                        const typename E::S* p = A + (int64_t)row * lda + col;
                        if constexpr (VW == 1) a[0] = E::one(p); else E::vec(p, a);
#pragma unroll
                        for (int e = 0; e < VW; ++e) acc[u] += a[e] * xv[e];
                    }
                }
            } else if (col < n) {
                // ragged end of the row: element loads only
                for (int e = 0; e < n - col; ++e) {
                    const Acc xe = xs[col + e];
#pragma unroll
                    for (int u = 0; u < kR; ++u) {
                        const int row = base + u * NG;
                        if (row < r1) acc[u] += E::one(A + (int64_t)row * lda + col + e) * xe;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kR; ++u) acc[u] = group_sum_t<Acc, LPR>(acc[u]);
#pragma unroll
        for (int u = 0; u < kR; ++u) {
            const int row = base + u * NG;
            if (row < r1) {
                const double r = rhs[row] - static_cast<double>(acc[u]);
                if (rout) rout[row] = r;
                if (q == 0) loc.r2 += r * r;
                const double nn = nu2[row];
                if (nn > 0.0) {
                    const double score = (r * r) / nn;
                    if (!isfinite(score)) loc.flags |= kFlagNonfinite;
                    else if (cand_better(score, (uint32_t)row, loc.score, loc.idx)) {
                        loc.score = score;
                        loc.r = r;
                        loc.idx = (uint32_t)row;
                    }
                } else if (isnan(nn)) {
                    loc.flags |= kFlagNonfinite;
                }
            }
        }
    }
}

template <class Tag, bool VEC, int LPR, bool GRID>
__device__ void solve_loop(const SolveSys& S, const Ctl& C, int wg, int G, char* smem)
{
    constexpr bool MIXED = !std::is_same<Tag, tag_f64>::value;
    using LPS = typename Elem<Tag>::S;
    __shared__ Red slots[kNW];
    __shared__ uint32_t s_ok;

    const int tid = threadIdx.x;
    const int n = S.n;
    const int d = S.d;
    double* sx = reinterpret_cast<double*>(smem);            // x, FP64
    float* sd = reinterpret_cast<float*>(sx + ((n + 1) & ~1)); // x - x_ref, FP32 (mixed)

    const int rows_per = (d + G - 1) / G;
    const int r0 = min(d, wg * rows_per);
    const int r1 = min(d, r0 + rows_per);
    const int cols_per = (n + G - 1) / G;
    const int e0 = min(n, wg * cols_per);
    const int e1 = min(n, e0 + cols_per);

    double xo[kCPT], dl[kCPT];
#pragma unroll
    for (int j = 0; j < kCPT; ++j) {
        const int c = tid + j * kNT;
        xo[j] = 0.0;
        dl[j] = 0.0;
        if (c < n) {
            xo[j] = S.x0 ? S.x0[c] : 0.0;
            sx[c] = xo[j];
            if (MIXED) sd[c] = 0.0f;
        }
    }
    // ||x_ref||^2 and ||bt||^2, reduced identically by every workgroup.
    Red q = red_identity();
    if (S.xref)
        for (int c = tid; c < n; c += kNT) q.e2 += S.xref[c] * S.xref[c];
    for (int i = tid; i < d; i += kNT) q.r2 += S.bt[i] * S.bt[i];
    q = block_red<kNT>(q, slots);
    const double xref2 = q.e2;
    const double bt2 = q.r2;
    const double tol2 = C.tol2;
    const bool rel_err = S.stop_mode == CSK_STOP_REL_ERR;

    bool fp64 = !MIXED;
    bool need_refresh = true;
    int64_t k_ref = 0;
    int64_t nref = 0;
    double hist0 = INFINITY, hist1 = INFINITY;
    int32_t status = CSK_NOT_CONVERGED;
    double meas = NAN;
    uint32_t epoch = 0;
    int64_t k = 0;
    for (;; ++k) {
        const bool refresh = MIXED && !fp64 && (need_refresh || (k - k_ref) >= C.refresh_every);
        const bool exact = !MIXED || fp64 || refresh;
        Red loc = red_identity();
        if (exact) {
            residual_rows<tag_f64, VEC, LPR>(S.At64, S.ldat64, n, r0, r1, sx, S.bt,
                                             refresh ? S.rref : nullptr, S.nu2, loc);
        } else {
            residual_rows<Tag, VEC, LPR>(static_cast<const LPS*>(S.At), S.ldat, n, r0, r1,
                                         reinterpret_cast<const typename Elem<Tag>::Acc*>(sd),
                                         S.rref, nullptr, S.nu2, loc);
        }
        if (S.xref)
            for (int c = e0 + tid; c < e1; c += kNT) {
                const double e = sx[c] - S.xref[c];
                loc.e2 += e * e;
            }
        if (wg == 0 && tid == 0 && C.cancel && (k % C.check_every) == 0 && *C.cancel != 0)
            loc.flags |= kFlagCancel;
        Red tot = block_red<kNT>(loc, slots);
        if constexpr (GRID) {
            Red* rec = C.exch + (size_t)(k & 1) * G;
            if (tid == 0) rec[wg] = tot;
            ++epoch;
            const bool ok = grid_barrier(C.barrier, epoch * (uint32_t)G, &s_ok);
            Red all = red_identity();
            for (int w = tid; w < G; w += kNT) all = red_combine(all, rec[w]);
            tot = block_red<kNT>(all, slots);
            if (!ok) tot.flags |= kFlagTimeout;
        }

        // Stop test on x_k (top of iteration k).
        bool conv;
        if (rel_err) {
            meas = xref2 > 0.0 ? tot.e2 / xref2 : tot.e2;
            conv = xref2 > 0.0 ? (tot.e2 / xref2 <= tol2) : (tot.e2 <= tol2);
        } else {
            const bool hit = tot.r2 <= tol2 * bt2;
            if (exact) meas = bt2 > 0.0 ? tot.r2 / bt2 : tot.r2;
            conv = exact && hit;
            if (MIXED && !exact && hit) need_refresh = true;
        }
        if (conv) { status = CSK_OK; break; }
        if (k == C.maxit) { status = CSK_NOT_CONVERGED; break; }
        if (tot.flags & kFlagTimeout) { status = CSK_ERR_DEVICE; break; }
        if (tot.flags & kFlagCancel) { status = CSK_CANCELLED; break; }
        if (tot.flags & kFlagNonfinite) { status = CSK_ERR_NONFINITE; break; }
        if (tot.idx == kNoRow) { status = CSK_ERR_DEGENERATE; break; }
        if (refresh) {
            ++nref;
            k_ref = k;
            need_refresh = false;
            const double m_now = rel_err ? tot.e2 : tot.r2;
            if (nref >= 3 && !(m_now < hist0)) fp64 = true;  // stagnated over two windows
            hist0 = hist1;
            hist1 = m_now;
        }

        // Projection onto row i_k, on this workgroup's copy of x.
        const int64_t ik = tot.idx;
        const double alpha = tot.r / S.nu2[ik];
        const double* __restrict__ arow = S.At64 + ik * S.ldat64;
#pragma unroll
        for (int j = 0; j < kCPT; ++j) {
            const int c = tid + j * kNT;
            if (c < n) {
                const double a = arow[c];
                xo[j] = xo[j] + alpha * a;
                sx[c] = xo[j];
                if (MIXED) {
                    dl[j] = (refresh ? 0.0 : dl[j]) + alpha * a;
                    sd[c] = static_cast<float>(dl[j]);
                }
            }
        }
        __syncthreads();
    }

    if (wg == 0) {
#pragma unroll
        for (int j = 0; j < kCPT; ++j) {
            const int c = tid + j * kNT;
            if (c < n) S.x[c] = xo[j];
        }
        if (tid == 0 && S.res) {
            S.res->iters = k;
            S.res->status = status;
            S.res->fp64_fallback = (MIXED && fp64) ? 1 : 0;
            S.res->final_measure = meas;
            S.res->refreshes = nref;
        }
    }
}

template <class Tag, bool VEC, int LPR>
__global__ __launch_bounds__(kNT) void k_solve_grid(SolveSys S, Ctl C)
{
    extern __shared__ __align__(16) char smem[];
    solve_loop<Tag, VEC, LPR, true>(S, C, blockIdx.x, gridDim.x, smem);
}

template <class Tag, bool VEC, int LPR>
__global__ __launch_bounds__(kNT) void k_solve_single(SolveSys S, Ctl C)
{
    extern __shared__ __align__(16) char smem[];
    solve_loop<Tag, VEC, LPR, false>(S, C, 0, 1, smem);
}

template <class Tag, bool VEC, int LPR>
__global__ __launch_bounds__(kNT) void k_solve_batched(const SolveSys* __restrict__ sys, Ctl C)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int32_t s_next;
    for (;;) {
        if (threadIdx.x == 0) s_next = static_cast<int32_t>(atomicAdd(C.queue, 1u));
        __syncthreads();
        const int32_t qpos = s_next;
        __syncthreads();
        if (qpos >= C.nsys) break;
        const SolveSys S = sys[C.order[qpos]];
        solve_loop<Tag, VEC, LPR, false>(S, C, 0, 1, smem);
        __syncthreads();
    }
}

__global__ void k_zero_u32(uint32_t* p, int count)
{
    if ((int)threadIdx.x < count) p[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void k_row_norms2(const double* __restrict__ A, int64_t lda, int d, int n,
                                                   double* __restrict__ nu2)
{
    const int lane = threadIdx.x & (kWave - 1);
    for (int64_t i = blockIdx.x * 4 + threadIdx.x / kWave; i < d; i += (int64_t)gridDim.x * 4) {
        double s = 0.0;
        for (int c = lane; c < n; c += kWave) s += A[i * lda + c] * A[i * lda + c];
        s = wave_sum(s);
        if (lane == 0) nu2[i] = s;
    }
}

size_t smem_bytes(int64_t n, bool mixed)
{
    return (size_t)((n + 1) & ~1) * 8 + (mixed ? (size_t)n * 4 : 0) + 16;
}

template <class Tag, bool VEC, int LPR>
csk_status launch_solve(const SolveSys& S, const Ctl& C, int grid, hipStream_t st)
{
    const bool mixed = !std::is_same<Tag, tag_f64>::value;
    const size_t shm = smem_bytes(S.n, mixed);
    if (grid <= 1) {
        auto kern = k_solve_single<Tag, VEC, LPR>;
        CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        kern<<<1, kNT, shm, st>>>(S, C);
        CSK_LAUNCH_CHECK("k_solve_single");
        return CSK_OK;
    }
    auto kern = k_solve_grid<Tag, VEC, LPR>;
    CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    int per_cu = 0;
    CSK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), kNT, shm));
    const int cap = per_cu * device_cu_count();
    if (grid > cap) {
        set_error("persistent grid of %d workgroups exceeds the %d co-resident ones", grid, cap);
        return CSK_ERR_UNSUPPORTED;
    }
    SolveSys s_arg = S;
    Ctl c_arg = C;
    void* args[] = {&s_arg, &c_arg};
    CSK_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(kNT), args,
                                       (unsigned)shm, st));
    return CSK_OK;
}

template <class Tag, bool VEC, int LPR>
csk_status launch_batched(const SolveSys* sys, const Ctl& C, int64_t n_max, hipStream_t st)
{
    const bool mixed = !std::is_same<Tag, tag_f64>::value;
    const size_t shm = smem_bytes(n_max, mixed);
    auto kern = k_solve_batched<Tag, VEC, LPR>;
    CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    int per_cu = 0;
    CSK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), kNT, shm));
    const int grid = std::max(1, std::min(C.nsys, std::max(1, per_cu) * device_cu_count()));
    kern<<<grid, kNT, shm, st>>>(sys, C);
    CSK_LAUNCH_CHECK("k_solve_batched");
    return CSK_OK;
}

template <class Tag>
csk_status dispatch_solve(const SolveSys& S, const Ctl& C, const SolvePlan& p, hipStream_t st)
{
    if (p.vw > 1) {
        if (p.lpr == 16) return launch_solve<Tag, true, 16>(S, C, p.grid, st);
        return launch_solve<Tag, true, 64>(S, C, p.grid, st);
    }
    if (p.lpr == 16) return launch_solve<Tag, false, 16>(S, C, p.grid, st);
    return launch_solve<Tag, false, 64>(S, C, p.grid, st);
}

template <class Tag>
csk_status dispatch_batched(const SolveSys* sys, const Ctl& C, int64_t n_max, bool vec, hipStream_t st)
{
    if (vec) return launch_batched<Tag, true, 16>(sys, C, n_max, st);
    return launch_batched<Tag, false, 16>(sys, C, n_max, st);
}

bool al16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

Ctl make_ctl(const csk_solve_opts* o)
{
    Ctl C{};
    C.tol2 = o->tol * o->tol;
    C.maxit = o->maxit;
    C.cancel = o->cancel;
    C.refresh_every = o->refresh_every > 0 ? o->refresh_every : 64;
    C.check_every = o->check_every > 0 ? o->check_every : 256;
    return C;
}

}  // namespace

SolvePlan solve_plan(int64_t d, int64_t n, csk_dtype at_dtype, int64_t ldat, const void* At,
                     const csk_solve_opts* o)
{
    SolvePlan p;
    p.block = kNT;
    // Lanes per row: 64 when a row spans at least two full wavefront vectors.
    const int64_t vec = 16 / (int64_t)dtype_size(at_dtype);
    p.lpr = (n >= 2 * 64 * std::min<int64_t>(vec, 2)) ? 64 : 16;
    const bool vec_ok = al16(At) && ((ldat * (int64_t)dtype_size(at_dtype)) % 16 == 0);
    p.vw = vec_ok ? (int)vec : 1;
    int grid;
    if (o && o->single_wg == 1) grid = 1;
    else if (o && o->grid > 0) grid = o->grid;
    else if (o && o->single_wg == 0) grid = std::max(2, std::min<int>(device_cu_count(), (int)((d + 15) / 16)));
    else {
        // One workgroup while its rows fit comfortably in one CU's share of
        // L2; otherwise one workgroup per CU, with at least 16 rows each.
        const int64_t bytes = d * n * (int64_t)dtype_size(at_dtype);
        grid = (bytes <= (int64_t)(1 << 20)) ? 1 : std::max(2, std::min<int>(device_cu_count(), (int)((d + 15) / 16)));
    }
    p.grid = std::min<int64_t>(grid, d) < 1 ? 1 : (int)std::min<int64_t>(grid, d);
    return p;
}

size_t solve_ws_bytes(int64_t d, int64_t n, int grid)
{
    (void)n;
    Carve c(nullptr);
    c.take<Red>(2 * (size_t)std::max(grid, 1));
    c.take<uint32_t>(64);
    c.take<double>(d);   // r_ref
    c.take<double>(d);   // nu2 when not supplied
    return c.bytes();
}

csk_status solve_run(const SolveSys& sys_in, csk_dtype at_dtype, const csk_solve_opts* o,
                     void* ws, size_t ws_bytes, hipStream_t st)
{
    SolveSys S = sys_in;
    SolvePlan plan = solve_plan(S.d, S.n, at_dtype, S.ldat, S.At, o);
    // The exact FP64 product shares the vector path, so At64 must qualify too.
    if (plan.vw > 1 && (!al16(S.At64) || (S.ldat64 * 8) % 16 != 0)) plan.vw = 1;

    Carve c(ws);
    Ctl C = make_ctl(o);
    C.exch = c.take<Red>(2 * (size_t)std::max(plan.grid, 1));
    C.barrier = c.take<uint32_t>(64);
    S.rref = c.take<double>(S.d);
    double* nu2_ws = c.take<double>(S.d);
    if (c.bytes() > ws_bytes) {
        set_error("solve workspace too small: need %zu bytes, got %zu", c.bytes(), ws_bytes);
        return CSK_ERR_WORKSPACE;
    }
    if (S.nu2 == nullptr) {
        k_row_norms2<<<std::min(4096, (S.d + 3) / 4), 256, 0, st>>>(S.At64, S.ldat64, S.d, S.n, nu2_ws);
        CSK_LAUNCH_CHECK("k_row_norms2");
        S.nu2 = nu2_ws;
    }
    k_zero_u32<<<1, 64, 0, st>>>(C.barrier, 64);
    CSK_LAUNCH_CHECK("k_zero_u32");
    switch (at_dtype) {
    case CSK_F64: return dispatch_solve<tag_f64>(S, C, plan, st);
    case CSK_F32: return dispatch_solve<tag_f32>(S, C, plan, st);
    case CSK_F16: return dispatch_solve<tag_f16>(S, C, plan, st);
    case CSK_BF16: return dispatch_solve<tag_bf16>(S, C, plan, st);
    default: return CSK_ERR_UNSUPPORTED;
    }
}

csk_status solve_batched_run(const SolveSys* sys_dev, const int32_t* order_dev, int32_t nsys,
                             int64_t n_max, csk_dtype at_dtype, const csk_solve_opts* o,
                             uint32_t* queue_dev, hipStream_t st)
{
    Ctl C = make_ctl(o);
    C.queue = queue_dev;
    C.order = order_dev;
    C.nsys = nsys;
    k_zero_u32<<<1, 64, 0, st>>>(queue_dev, 1);
    CSK_LAUNCH_CHECK("k_zero_u32");
    // Descriptors are laid out by the caller with 16-byte aligned rows.
    const bool vec = true;
    switch (at_dtype) {
    case CSK_F64: return dispatch_batched<tag_f64>(sys_dev, C, n_max, vec, st);
    case CSK_F32: return dispatch_batched<tag_f32>(sys_dev, C, n_max, vec, st);
    case CSK_F16: return dispatch_batched<tag_f16>(sys_dev, C, n_max, vec, st);
    case CSK_BF16: return dispatch_batched<tag_bf16>(sys_dev, C, n_max, vec, st);
    default: return CSK_ERR_UNSUPPORTED;
    }
}

}  // namespace csk
