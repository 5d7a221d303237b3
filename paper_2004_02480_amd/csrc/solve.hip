// solve.hip -- Algorithm 1, loop: maximal weighted residual Kaczmarz (MWRK)
// on the sketched system (At, bt), as one persistent kernel.
//
// Every iteration k, with no host round trip:
//   1. residual r_i = bt_i - At^(i) x_k for the workgroup's own block of rows.
//      The product is bandwidth-bound: At streams through a ring of kD chunks
//      per lane (kK 16-byte vectors each) so enough loads are in flight to
//      cover HBM latency; x sits in LDS.
//   2. weighted score r_i^2 / ||At^(i)||^2 (the square of the paper's
//      |r_i| / ||At^(i)||, same argmax), best row of the workgroup through
//      wavefront butterflies and LDS;
//   3. (grid path) each workgroup publishes its best row (score, step length
//      alpha = r / ||At^(i)||^2, index), partial ||r||^2 and partial
//      ||x - x_ref||^2 in its own record, release-stored with the iteration
//      as tag; every workgroup polls all tags in parallel and reduces the
//      records in the same fixed order, so all agree on i_k and on the stop
//      decision.  No shared read-modify-write counter is contended.
//   4. stop test (Section 3's RES, or the sketched residual), then the
//      projection x += alpha At^(i_k)^T, applied by every workgroup to its
//      own copy of x (each thread owns fixed columns).
// Mixed precision: At is held in FP32/FP16/BF16 and the FP64 sketch At64 is
// kept beside it.  Every `refresh_every` iterations the exact FP64 residual
// r_ref = bt - At64 x is formed and x_ref = x saved; in between the residual
// is r_ref - At (x - x_ref) with FP32 accumulation, so each inner iteration
// streams 2-4x fewer bytes.  Scores and projections use the FP64 rows.
// Small systems run the same loop in one workgroup (no exchange); the
// batched kernel hands whole systems to workgroups from an atomic queue.
#include "csk_grid.h"
#include "csk_solve.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace csk {
namespace {

constexpr int kNT = 512;        // threads per workgroup
constexpr int kNW = kNT / kWave;
constexpr int kCPT = 16;        // owned columns per thread: n <= kNT * kCPT
constexpr int kK = 8;           // 16-byte vectors per lane per chunk (FP64, FP32)
constexpr int kK16 = 4;         // ... for the 16-bit types (8 elements per vector)

using Red = GridRed;            // Red.r carries the step length alpha

struct tag_f64 { using storage = double; };

// Chunks in flight per lane (each chunk holds KK 16-byte vectors): 3 for
// FP64 (8 vectors), 2 for FP32 (8 vectors), 3 for the 16-bit types (4).
template <class Tag> constexpr int ring_depth() { return std::is_same<Tag, tag_f64>::value ? 3 : std::is_same<Tag, tag_f32>::value ? 2 : 3; }
template <class Tag> constexpr int chunk_k() { return sizeof(typename Tag::storage) == 2 ? kK16 : kK; }

// One workgroup's published contribution to an iteration.
struct alignas(64) XRec {
    double score, alpha, r2, e2;
    uint32_t idx, flags;
    uint64_t tag;
};

struct Ctl {
    double tol2;
    int64_t maxit;
    const volatile int32_t* cancel;
    XRec* exch;            // [2][grid], tags zero at launch
    uint32_t* queue;       // batched work queue, zero at launch
    const int32_t* order;  // batched: queue position -> system
    int32_t refresh_every, check_every;
    int32_t nsys;
    int32_t pad_;
};

// Element access.  A chunk slot holds one 16-byte vector per k (VW elements)
// or, on the scalar path, one element in its low bits.
template <class Tag> struct Elem;
template <> struct Elem<tag_f64> {
    using S = double;
    using Acc = double;
    static constexpr int kVec = 2;
    __device__ static double dot(const uint4& v, const double* x, int vw)
    {
        if (vw == 1) return __builtin_bit_cast(double, make_uint2(v.x, v.y)) * x[0];
        const double2 a = __builtin_bit_cast(double2, v);
        return a.x * x[0] + a.y * x[1];
    }
};
template <> struct Elem<tag_f32> {
    using S = float;
    using Acc = float;
    static constexpr int kVec = 4;
    __device__ static float dot(const uint4& v, const float* x, int vw)
    {
        if (vw == 1) return __uint_as_float(v.x) * x[0];
        return __uint_as_float(v.x) * x[0] + __uint_as_float(v.y) * x[1] + __uint_as_float(v.z) * x[2] +
               __uint_as_float(v.w) * x[3];
    }
};
template <class Tag> struct Elem16 {
    using S = uint16_t;
    using Acc = float;
    static constexpr int kVec = 8;
    __device__ static float dot(const uint4& v, const float* x, int vw)
    {
        if (vw == 1) return widen<Tag>(static_cast<uint16_t>(v.x & 0xFFFFu)) * x[0];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s += widen<Tag>(static_cast<uint16_t>(w[k] & 0xFFFFu)) * x[2 * k];
            s += widen<Tag>(static_cast<uint16_t>(w[k] >> 16)) * x[2 * k + 1];
        }
        return s;
    }
};
template <> struct Elem<tag_f16> : Elem16<tag_f16> {};
template <> struct Elem<tag_bf16> : Elem16<tag_bf16> {};

template <class T, int W>
__device__ __forceinline__ T group_sum_t(T v)
{
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
    return v;
}

// The first `cnt` elements at p (cnt <= W) in a 16-byte vector, rest zero;
// element indices are compile-time constants, so nothing leaves registers.
template <class S, int W>
__device__ __forceinline__ uint4 load_partial(const S* p, int cnt)
{
    struct alignas(16) Pack {
        S e[16 / sizeof(S)];
    } t;
#pragma unroll
    for (int e = 0; e < (int)(16 / sizeof(S)); ++e) t.e[e] = (e < W && e < cnt) ? p[e] : S(0);
    return __builtin_bit_cast(uint4, t);
}

// Loads chunk slot `b` (KK vectors of one lane) for (row, seg); `on` false
// (or columns past n) leaves zeros and touches no memory.  For the last
// segment of a row it also fetches that row's right-hand side and squared
// norm, so every load a consumer waits on was issued with its chunk (waits
// on the in-order vector-memory counter then never drain later chunks).
template <class Tag, int VW, int LPR, int KK>
__device__ __forceinline__ void load_chunk(uint4 (&b)[KK], double& rhs_v, double& nu2_v,
                                           const typename Elem<Tag>::S* __restrict__ A, int64_t lda, int n, int row,
                                           int seg, int nseg, int q, bool on, const double* __restrict__ rhs,
                                           const double* __restrict__ nu2)
{
    using S = typename Elem<Tag>::S;
    constexpr int SW = LPR * VW * KK;
    const S* base = A + (int64_t)row * lda;
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
        const int col = seg * SW + (kk * LPR + q) * VW;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (on && col < n) {
            if (col + VW <= n && VW > 1) v = *reinterpret_cast<const uint4*>(base + col);
            else v = load_partial<S, VW>(base + col, n - col);
        }
        b[kk] = v;
    }
    rhs_v = 0.0;
    nu2_v = 0.0;
    if (on && seg == nseg - 1) {
        rhs_v = rhs[row];
        nu2_v = nu2[row];
    }
}

// Residuals, candidates and partial ||r||^2 for rows [r0, r1) of the
// workgroup.  Lane groups of LPR lanes share a row; a row is split into
// nseg segments of LPR*VW*kK columns; the group walks its (row, segment)
// chunks in order with kD chunks in flight.  xs is the operand vector in LDS
// (x for FP64, x - x_ref in FP32 for the low-precision product), zero beyond
// n up to nseg*SW; rhs is bt (exact) or r_ref (inner).  When rout is
// non-null the residuals are stored there (a refresh).
template <class Tag, bool VEC, int LPR, int kD>
__device__ __forceinline__ void stream_rows(const typename Elem<Tag>::S* __restrict__ A, int64_t lda, int n,
                                            int nseg, int r0, int r1, const typename Elem<Tag>::Acc* __restrict__ xs,
                                            const double* __restrict__ rhs, double* __restrict__ rout,
                                            const double* __restrict__ nu2, Red& loc)
{
    using E = Elem<Tag>;
    using Acc = typename E::Acc;
    constexpr int VW = VEC ? E::kVec : 1;
    constexpr int NG = kNT / LPR;
    constexpr int KK = chunk_k<Tag>();
    constexpr int SW = LPR * VW * KK;
    const int q = threadIdx.x % LPR;
    const int g = threadIdx.x / LPR;
    const int span = r1 - r0;
    const int nrows = span > g ? (span - g + NG - 1) / NG : 0;
    const int nchunk = nrows * nseg;
    const int nchunk_max = (span > 0 ? (span + NG - 1) / NG : 0) * nseg;  // group 0 has the most

    uint4 buf[kD][KK];
    double pr[kD], pn[kD];  // right-hand side and squared norm of the slot's row
    int irow = 0, iseg = 0;  // next chunk to load
#pragma unroll
    for (int u = 0; u < kD; ++u) {
        load_chunk<Tag, VW, LPR, KK>(buf[u], pr[u], pn[u], A, lda, n, r0 + g + NG * irow, iseg, nseg, q,
                                     u < nchunk, rhs, nu2);
        if (++iseg == nseg) { iseg = 0; ++irow; }
    }
    int crow = 0, cseg = 0;  // next chunk to consume
    Acc acc = Acc(0);
    for (int c0 = 0; c0 < nchunk_max; c0 += kD) {
#pragma unroll
        for (int u = 0; u < kD; ++u) {
            const int c = c0 + u;
            if (c < nchunk_max) {
                const int cbase = cseg * SW + q * VW;
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) acc += E::dot(buf[u][kk], xs + cbase + kk * LPR * VW, VW);
                if (cseg == nseg - 1) {
                    const Acc s = group_sum_t<Acc, LPR>(acc);
                    acc = Acc(0);
                    if (c < nchunk) {
                        const int row = r0 + g + NG * crow;
                        const double r = pr[u] - static_cast<double>(s);
                        if (rout) rout[row] = r;
                        if (q == 0) loc.r2 += r * r;
                        const double nn = pn[u];
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
                    }
                }
                if (++cseg == nseg) { cseg = 0; ++crow; }
                load_chunk<Tag, VW, LPR, KK>(buf[u], pr[u], pn[u], A, lda, n, r0 + g + NG * irow, iseg, nseg, q,
                                             c + kD < nchunk, rhs, nu2);
                if (++iseg == nseg) { iseg = 0; ++irow; }
            }
        }
    }
}

// Publish this workgroup's record for iteration k and reduce all G records
// (grid path).  Tags start at zero and iteration k writes k + 1, so a stale
// record is never mistaken for a fresh one; two slots alternate by parity.
// All record accesses are device-coherent (write-through stores and loads at
// the coherence point, "sc1"): the writer's field stores are acknowledged
// (explicit wait) before its tag store is issued, and a reader loads the
// fields only after it has seen the tag.  No cache write-back or
// invalidation is needed, so the exchange does not touch L2 contents (where
// the workgroup's rows of At may be resident).
template <class T> __device__ __forceinline__ void coh_store(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T> __device__ __forceinline__ T coh_load(const T* p)
{
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ Red exchange(const Red& mine, XRec* exch, int wg, int G, int64_t k, Red* slots)
{
    XRec* slot = exch + (size_t)(k & 1) * G;
    const uint64_t tagv = static_cast<uint64_t>(k) + 1u;
    if (threadIdx.x == 0) {
        XRec& w = slot[wg];
        coh_store(&w.score, mine.score);
        coh_store(&w.alpha, mine.r);
        coh_store(&w.r2, mine.r2);
        coh_store(&w.e2, mine.e2);
        coh_store(&w.idx, mine.idx);
        coh_store(&w.flags, mine.flags);
        // fields acknowledged at the coherence point before the tag goes out
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        coh_store(&w.tag, tagv);
    }
    bool ok = true;
    Red all = red_identity();
    for (int w = threadIdx.x; w < G; w += kNT) {
        uint32_t spins = 0;
        while (coh_load(&slot[w].tag) != tagv) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kSpinLimit) {
                ok = false;
                break;
            }
        }
        asm volatile("" ::: "memory");
        Red o;
        o.score = coh_load(&slot[w].score);
        o.r = coh_load(&slot[w].alpha);
        o.r2 = coh_load(&slot[w].r2);
        o.e2 = coh_load(&slot[w].e2);
        o.idx = coh_load(&slot[w].idx);
        o.flags = coh_load(&slot[w].flags);
        all = red_combine(all, o);
    }
    if (!ok) all.flags |= kFlagTimeout;
    return block_red<kNT>(all, slots);
}

template <class Tag, bool VEC, int LPR, bool GRID>
__device__ void solve_loop(const SolveSys& S, const Ctl& C, int wg, int G, char* smem)
{
    constexpr bool MIXED = !std::is_same<Tag, tag_f64>::value;
    using LPS = typename Elem<Tag>::S;
    using LAcc = typename Elem<Tag>::Acc;
    constexpr int SW64 = LPR * (VEC ? 2 : 1) * kK;
    constexpr int SWLP = LPR * (VEC ? Elem<Tag>::kVec : 1) * chunk_k<Tag>();
    __shared__ Red slots[kNW];

    const int tid = threadIdx.x;
    const int n = S.n;
    const int d = S.d;
    const int npad = S.npad;
    const int nseg64 = (n + SW64 - 1) / SW64;
    const int nseglp = (n + SWLP - 1) / SWLP;
    double* sx = reinterpret_cast<double*>(smem);           // x, FP64, zero past n
    LAcc* sd = reinterpret_cast<LAcc*>(sx + npad);          // x - x_ref (mixed), zero past n

    const int rows_per = (d + G - 1) / G;
    const int r0 = min(d, wg * rows_per);
    const int r1 = min(d, r0 + rows_per);
    const int cols_per = (n + G - 1) / G;
    const int e0 = min(n, wg * cols_per);
    const int e1 = min(n, e0 + cols_per);

    // x lives in LDS (sx); each thread owns columns tid + j*kNT and is the
    // only writer of them.  Mixed precision keeps x - x_ref for the owned
    // columns in FP64 registers (dl) and its FP32 rounding in LDS (sd).
    double dl[kCPT];
#pragma unroll
    for (int j = 0; j < kCPT; ++j) dl[j] = 0.0;
    for (int c = tid; c < npad; c += kNT) {
        sx[c] = (c < n && S.x0) ? S.x0[c] : 0.0;
        if (MIXED) sd[c] = LAcc(0);
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
    int64_t k = 0;
    for (;; ++k) {
        const bool refresh = MIXED && !fp64 && (need_refresh || (k - k_ref) >= C.refresh_every);
        const bool exact = !MIXED || fp64 || refresh;
        Red loc = red_identity();
        if (exact) {
            // the refresh product of the mixed mode runs once per window: a
            // shallower ring leaves the registers to the working-precision one
            stream_rows<tag_f64, VEC, LPR, MIXED ? 2 : ring_depth<tag_f64>()>(
                S.At64, S.ldat64, n, nseg64, r0, r1, sx, S.bt, refresh ? S.rref : nullptr, S.nu2, loc);
        } else {
            stream_rows<Tag, VEC, LPR, ring_depth<Tag>()>(static_cast<const LPS*>(S.At), S.ldat, n, nseglp, r0, r1,
                                                          sd, S.rref, nullptr, S.nu2, loc);
        }
        if (S.xref)
            for (int c = e0 + tid; c < e1; c += kNT) {
                const double e = sx[c] - S.xref[c];
                loc.e2 += e * e;
            }
        if (wg == 0 && tid == 0 && C.cancel && (k % C.check_every) == 0 && *C.cancel != 0)
            loc.flags |= kFlagCancel;
        Red tot = block_red<kNT>(loc, slots);
        if constexpr (GRID) tot = exchange(tot, C.exch, wg, G, k, slots);

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
        if (tot.idx >= (uint32_t)d) { status = CSK_ERR_DEVICE; break; }  // never dereference a bad row
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
        const double alpha = tot.r;
        const double* __restrict__ arow = S.At64 + (int64_t)tot.idx * S.ldat64;
#pragma unroll
        for (int j = 0; j < kCPT; ++j) {
            const int c = tid + j * kNT;
            if (c < n) {
                const double a = arow[c];
                sx[c] = sx[c] + alpha * a;
                if (MIXED) {
                    dl[j] = (refresh ? 0.0 : dl[j]) + alpha * a;
                    sd[c] = static_cast<LAcc>(dl[j]);
                }
            }
        }
        __syncthreads();
    }

    if (wg == 0) {
        for (int c = tid; c < n; c += kNT) S.x[c] = sx[c];
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

__global__ void k_zero_words(uint32_t* p, int64_t words)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < words; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0u;
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

size_t smem_bytes(int64_t npad, bool mixed)
{
    return (size_t)npad * 8 + (mixed ? (size_t)npad * 4 : 0) + 16;
}

template <class Tag, bool VEC, int LPR>
csk_status launch_solve(const SolveSys& S, const Ctl& C, int grid, hipStream_t st)
{
    const bool mixed = !std::is_same<Tag, tag_f64>::value;
    const size_t shm = smem_bytes(S.npad, mixed);
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

template <class Tag, bool VEC>
csk_status dispatch_lpr(const SolveSys& S, const Ctl& C, const SolvePlan& p, hipStream_t st)
{
    switch (p.lpr) {
    case 4: return launch_solve<Tag, VEC, 4>(S, C, p.grid, st);
    case 16: return launch_solve<Tag, VEC, 16>(S, C, p.grid, st);
    default: return launch_solve<Tag, VEC, 64>(S, C, p.grid, st);
    }
}

template <class Tag>
csk_status dispatch_solve(const SolveSys& S, const Ctl& C, const SolvePlan& p, hipStream_t st)
{
    if (p.vw > 1) return dispatch_lpr<Tag, true>(S, C, p, st);
    return dispatch_lpr<Tag, false>(S, C, p, st);
}

constexpr int kBatchLPR = 16;

template <class Tag>
csk_status launch_batched(const SolveSys* sys, const Ctl& C, int64_t npad_max, hipStream_t st)
{
    const bool mixed = !std::is_same<Tag, tag_f64>::value;
    const size_t shm = smem_bytes(npad_max, mixed);
    auto kern = k_solve_batched<Tag, true, kBatchLPR>;
    CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    int per_cu = 0;
    CSK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), kNT, shm));
    const int grid = std::max(1, std::min(C.nsys, std::max(1, per_cu) * device_cu_count()));
    kern<<<grid, kNT, shm, st>>>(sys, C);
    CSK_LAUNCH_CHECK("k_solve_batched");
    return CSK_OK;
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

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

}  // namespace

int64_t chunk_k_of(csk_dtype t) { return dtype_size(t) == 2 ? kK16 : kK; }

int64_t solve_npad(int64_t n, csk_dtype at_dtype, int lpr, bool vec)
{
    const int64_t vwlp = vec ? 16 / (int64_t)dtype_size(at_dtype) : 1;
    const int64_t sw64 = (int64_t)lpr * (vec ? 2 : 1) * kK;
    const int64_t swlp = (int64_t)lpr * vwlp * chunk_k_of(at_dtype);
    return std::max(round_up(n, sw64), round_up(n, swlp));
}

int solve_batch_lpr() { return kBatchLPR; }

SolvePlan solve_plan(int64_t d, int64_t n, csk_dtype at_dtype, int64_t ldat, const void* At,
                     const csk_solve_opts* o)
{
    SolvePlan p;
    p.block = kNT;
    const int64_t vec = 16 / (int64_t)dtype_size(at_dtype);
    const bool vec_ok = al16(At) && ((ldat * (int64_t)dtype_size(at_dtype)) % 16 == 0);
    p.vw = vec_ok ? (int)vec : 1;
    // Lanes per row: the fewest of {4, 16, 64} whose chunk covers the row.
    const int64_t per_lane = (int64_t)p.vw * chunk_k_of(at_dtype);
    p.lpr = (4 * per_lane >= n) ? 4 : (16 * per_lane >= n) ? 16 : 64;
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
    p.grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, d));
    return p;
}

size_t solve_ws_bytes(int64_t d, int64_t n, int grid)
{
    (void)n;
    Carve c(nullptr);
    c.take<XRec>(2 * (size_t)std::max(grid, 1));
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
    if (plan.vw > 1 && (!al16(S.At64) || (S.ldat64 * 8) % 16 != 0)) {
        plan.vw = 1;
        const int64_t per_lane = chunk_k_of(at_dtype);
        plan.lpr = (4 * per_lane >= S.n) ? 4 : (16 * per_lane >= S.n) ? 16 : 64;
    }
    S.npad = (int32_t)solve_npad(S.n, at_dtype, plan.lpr, plan.vw > 1);

    Carve c(ws);
    Ctl C = make_ctl(o);
    C.exch = c.take<XRec>(2 * (size_t)std::max(plan.grid, 1));
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
    if (plan.grid > 1) {
        const int64_t words = (int64_t)2 * plan.grid * (int64_t)sizeof(XRec) / 4;
        k_zero_words<<<(int)std::min<int64_t>(64, (words + 255) / 256), 256, 0, st>>>(
            reinterpret_cast<uint32_t*>(C.exch), words);
        CSK_LAUNCH_CHECK("k_zero_words");
    }
    switch (at_dtype) {
    case CSK_F64: return dispatch_solve<tag_f64>(S, C, plan, st);
    case CSK_F32: return dispatch_solve<tag_f32>(S, C, plan, st);
    case CSK_F16: return dispatch_solve<tag_f16>(S, C, plan, st);
    case CSK_BF16: return dispatch_solve<tag_bf16>(S, C, plan, st);
    default: return CSK_ERR_UNSUPPORTED;
    }
}

csk_status solve_batched_run(const SolveSys* sys_dev, const int32_t* order_dev, int32_t nsys,
                             int64_t npad_max, csk_dtype at_dtype, const csk_solve_opts* o,
                             uint32_t* queue_dev, hipStream_t st)
{
    Ctl C = make_ctl(o);
    C.queue = queue_dev;
    C.order = order_dev;
    C.nsys = nsys;
    k_zero_words<<<1, 64, 0, st>>>(queue_dev, 1);
    CSK_LAUNCH_CHECK("k_zero_words");
    switch (at_dtype) {
    case CSK_F64: return launch_batched<tag_f64>(sys_dev, C, npad_max, st);
    case CSK_F32: return launch_batched<tag_f32>(sys_dev, C, npad_max, st);
    case CSK_F16: return launch_batched<tag_f16>(sys_dev, C, npad_max, st);
    case CSK_BF16: return launch_batched<tag_bf16>(sys_dev, C, npad_max, st);
    default: return CSK_ERR_UNSUPPORTED;
    }
}

}  // namespace csk
