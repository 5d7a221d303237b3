// solve.hip -- Algorithm 1, loop: maximal weighted residual Kaczmarz (MWRK)
// on the sketched system (At, bt), as one persistent kernel.
//
// Every iteration k, with no host round trip:
//   1. residual r_i = bt_i - At^(i) x_k for the workgroup's own block of rows.
//      The product is bandwidth-bound.  As much of the workgroup's block as
//      LDS holds beside x stays resident there for the whole solve; the rest
//      streams through a ring of kD chunks per lane (kK 16-byte vectors each)
//      so enough loads are in flight to cover HBM latency; x sits in LDS.
//   2. weighted score r_i^2 / ||At^(i)||^2 (the square of the paper's
//      |r_i| / ||At^(i)||, same argmax), best row of the workgroup through
//      wavefront butterflies and LDS;
//   3. (grid path) each workgroup publishes its best row (score, step length
//      alpha = r / ||At^(i)||^2, index), partial ||r||^2 or ||x - x_ref||^2
//      and flags in its own record of device-coherent words, each tagged
//      with the iteration; every workgroup polls all records in parallel and
//      reduces them in the same fixed order, so all agree on i_k and on the
//      stop decision.  No shared read-modify-write counter is contended.
//   4. stop test (Section 3's RES, or the sketched residual), then the
//      projection x += alpha At^(i_k)^T, applied by every workgroup to its
//      own copy of x (each thread owns fixed columns).
// Mixed precision: At is held in FP32/FP16/BF16 and the FP64 sketch At64 is
// kept beside it.  Every `refresh_every` iterations the exact FP64 residual
// r_ref = bt - At64 x is formed and x_ref = x saved; in between the residual
// is r_ref - At (x - x_ref) with FP32 accumulation, so each inner iteration
// streams 2-4x fewer bytes.  For the 16-bit types x - x_ref is also kept in
// LDS in that type (FP16 scaled by a power of two per refresh window), and
// the product uses two-element dot instructions.  Scores and projections
// use the FP64 rows.
// Small systems run the same loop in one workgroup (no exchange); the
// batched kernel hands whole systems to workgroups from an atomic queue.
#include "csk_grid.h"
#include "csk_solve.h"
#include "csk_tune.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <queue>
#include <tuple>
#include <type_traits>
#include <vector>

namespace csk {
namespace {

constexpr int kNT = 512;        // threads per workgroup
constexpr int kNW = kNT / kWave;
constexpr int kK = 8;           // 16-byte vectors per lane per chunk (FP64, FP32)
constexpr int kRegChunks = 4;   // register-resident chunks per lane group (FP64 greedy loop)
constexpr int kK16 = 4;         // ... for the 16-bit types (8 elements per vector)

using Red = GridRed;            // Red.r carries the step length alpha

struct tag_f64 { using storage = double; };

// Chunks in flight per lane (each chunk holds KK 16-byte vectors): 3 for
// FP64 (8 vectors), 2 for FP32 (8 vectors), 3 for the 16-bit types (4).
template <class Tag> constexpr int ring_depth() { return std::is_same<Tag, tag_f64>::value ? 3 : std::is_same<Tag, tag_f32>::value ? 2 : 3; }
template <class Tag> constexpr int chunk_k() { return sizeof(typename Tag::storage) == 2 ? kK16 : kK; }


struct Ctl {
    double tol2;
    int64_t maxit;
    const volatile int32_t* cancel;
    XRec* exch;            // [2][grid], tags zero at launch
    uint32_t* queue;       // batched work queue, zero at launch
    const int32_t* order;  // batched: queue position -> system
    const int32_t* item_off;  // batched: first work item of each queue position (nsys + 1)
    const int32_t* exch_off;  // batched: first exchange record of each queue position
    int32_t refresh_every, check_every;
    int32_t nsys;
    int32_t res_layers;    // LDS-resident chunks per lane group (capacity)
    int32_t xslice;        // LDS doubles for the workgroup's slice of x_ref
    int32_t rres;          // relaxed greedy randomized rule: LDS residuals per workgroup
    double theta;          // ... its relaxation parameter
    uint64_t sel_seed;     // ... and the seed of its selection stream
    int64_t* trace;        // nullable: row projected at each iteration
    const CsrRef* cref;    // mixed precision: refresh from a CSR A (device copy), or null
};

// Element access.  A chunk slot holds one 16-byte vector per k (VW elements)
// or, on the scalar path, one element in its low bits.  `lim` is the number
// of leading elements of the vector that lie inside the row (columns < n of
// a row this lane group owns); the others are treated as zero whatever the
// loaded bits are.
template <class Tag> struct Elem;
template <> struct Elem<tag_f64> {
    using S = double;
    using Acc = double;
    using Op = double;  // element type of the operand vector in LDS
    static constexpr int kVec = 2;
    template <int VW, bool M> __device__ static double dot(const uint4& v, const double* x, int lim)
    {
        if constexpr (VW == 1) {
            const double a = __builtin_bit_cast(double, make_uint2(v.x, v.y));
            return (!M || lim > 0 ? a : 0.0) * x[0];
        } else {
            const double2 a = __builtin_bit_cast(double2, v);
            return (!M || lim > 0 ? a.x : 0.0) * x[0] + (!M || lim > 1 ? a.y : 0.0) * x[1];
        }
    }
};
template <> struct Elem<tag_f32> {
    using S = float;
    using Acc = float;
    using Op = float;
    static constexpr int kVec = 4;
    template <int VW, bool M> __device__ static float dot(const uint4& v, const float* x, int lim)
    {
        if constexpr (VW == 1) return (!M || lim > 0 ? __uint_as_float(v.x) : 0.f) * x[0];
        return (!M || lim > 0 ? __uint_as_float(v.x) : 0.f) * x[0] + (!M || lim > 1 ? __uint_as_float(v.y) : 0.f) * x[1] +
               (!M || lim > 2 ? __uint_as_float(v.z) : 0.f) * x[2] + (!M || lim > 3 ? __uint_as_float(v.w) : 0.f) * x[3];
    }
};
// FP16: the operand copy is x - x_ref times 2^e, with e chosen at each
// refresh so that the window's first step has a scaled norm in [16, 32)
// (FP16's exponent range would lose x - x_ref as the residual shrinks);
// the product is rescaled by 2^-e.  Two-element dot instructions as BF16.
typedef _Float16 f16x2_t __attribute__((ext_vector_type(2)));
template <> struct Elem<tag_f16> {
    using S = uint16_t;
    using Acc = float;
    using Op = uint16_t;
    static constexpr int kVec = 8;
    template <int VW, bool M> __device__ static float dot(const uint4& v, const uint16_t* x, int lim)
    {
        if constexpr (VW == 1) {
            return (!M || lim > 0 ? f16_bits_to_f32(static_cast<uint16_t>(v.x & 0xFFFFu)) : 0.f) *
                   f16_bits_to_f32(x[0]);
        } else if constexpr (!M) {
            const uint4 xv = *reinterpret_cast<const uint4*>(x);
            float s = __builtin_amdgcn_fdot2(__builtin_bit_cast(f16x2_t, v.x), __builtin_bit_cast(f16x2_t, xv.x), 0.f,
                                             false);
            s = __builtin_amdgcn_fdot2(__builtin_bit_cast(f16x2_t, v.y), __builtin_bit_cast(f16x2_t, xv.y), s, false);
            s = __builtin_amdgcn_fdot2(__builtin_bit_cast(f16x2_t, v.z), __builtin_bit_cast(f16x2_t, xv.z), s, false);
            return __builtin_amdgcn_fdot2(__builtin_bit_cast(f16x2_t, v.w), __builtin_bit_cast(f16x2_t, xv.w), s,
                                          false);
        } else {
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s += (lim > 2 * k ? f16_bits_to_f32(static_cast<uint16_t>(w[k] & 0xFFFFu)) : 0.f) *
                     f16_bits_to_f32(x[2 * k]);
                s += (lim > 2 * k + 1 ? f16_bits_to_f32(static_cast<uint16_t>(w[k] >> 16)) : 0.f) *
                     f16_bits_to_f32(x[2 * k + 1]);
            }
            return s;
        }
    }
};
// BF16: the operand (x - x_ref) is kept in LDS rounded to BF16 as well, and
// the unmasked product of a 16-byte vector is four two-element dot
// instructions (BF16 pairs, FP32 accumulation) instead of eight widenings
// and eight FMAs.  Its rounding (relative 2^-9 of x - x_ref) is of the
// order of the BF16 rows' own, and each refresh restarts from the exact
// FP64 residual.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
template <> struct Elem<tag_bf16> {
    using S = uint16_t;
    using Acc = float;
    using Op = uint16_t;
    static constexpr int kVec = 8;
    template <int VW, bool M> __device__ static float dot(const uint4& v, const uint16_t* x, int lim)
    {
        if constexpr (VW == 1) {
            return (!M || lim > 0 ? bf16_bits_to_f32(static_cast<uint16_t>(v.x & 0xFFFFu)) : 0.f) *
                   bf16_bits_to_f32(x[0]);
        } else if constexpr (!M) {
            const uint4 xv = *reinterpret_cast<const uint4*>(x);
            float s = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, v.x),
                                                       __builtin_bit_cast(bf16x2_t, xv.x), 0.f, false);
            s = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, v.y), __builtin_bit_cast(bf16x2_t, xv.y),
                                                s, false);
            s = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, v.z), __builtin_bit_cast(bf16x2_t, xv.z),
                                                s, false);
            return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, v.w),
                                                   __builtin_bit_cast(bf16x2_t, xv.w), s, false);
        } else {
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s += (lim > 2 * k ? bf16_bits_to_f32(static_cast<uint16_t>(w[k] & 0xFFFFu)) : 0.f) *
                     bf16_bits_to_f32(x[2 * k]);
                s += (lim > 2 * k + 1 ? bf16_bits_to_f32(static_cast<uint16_t>(w[k] >> 16)) : 0.f) *
                     bf16_bits_to_f32(x[2 * k + 1]);
            }
            return s;
        }
    }
};
template <class Tag> constexpr bool op16() { return std::is_same<typename Elem<Tag>::Op, uint16_t>::value; }

// Loads chunk slot `b` (KK vectors of one lane) of (row, seg), with the
// row's right-hand side and squared norm.  Every load is issued, from a
// valid address, whatever `on` says: a lane that is off reads the first
// vector of row `rsafe` (all such lanes read the same 16 bytes, one cache
// line), and a vector starting at or past column n reads column 0; the
// caller masks such elements with `lim` (returned: the count of valid
// elements from this lane's first column of the chunk, 0 when off).
// A vector that starts before n may end past it, inside the row's 16-byte
// padded length (the vector path requires 16-byte rows), so it stays inside
// the matrix.  Without branches the compiler never has to merge different
// loads, so waits on the in-order vector-memory counter only ever wait for
// the slot that is consumed.
template <class Tag, int VW, int LPR, int KK>
__device__ __forceinline__ int load_chunk(uint4 (&b)[KK], double& rhs_v, double& nu2_v,
                                          const typename Elem<Tag>::S* __restrict__ A, int64_t lda, int n, int row,
                                          int rsafe, int seg, int q, bool on, const double* __restrict__ rhs,
                                          const double* __restrict__ nu2)
{
    using S = typename Elem<Tag>::S;
    constexpr int SW = LPR * VW * KK;
    const int r = on ? row : rsafe;
    const S* base = A + (int64_t)r * lda;
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
        const int col = seg * SW + (kk * LPR + q) * VW;
        const int cc = (on && col < n) ? col : 0;
        if constexpr (VW > 1) {
            b[kk] = *reinterpret_cast<const uint4*>(base + cc);
        } else if constexpr (sizeof(S) == 8) {
            const uint64_t w = *reinterpret_cast<const uint64_t*>(base + cc);
            b[kk] = make_uint4(static_cast<uint32_t>(w), static_cast<uint32_t>(w >> 32), 0u, 0u);
        } else if constexpr (sizeof(S) == 4) {
            b[kk] = make_uint4(*reinterpret_cast<const uint32_t*>(base + cc), 0u, 0u, 0u);
        } else {
            b[kk] = make_uint4(static_cast<uint32_t>(*reinterpret_cast<const uint16_t*>(base + cc)), 0u, 0u, 0u);
        }
    }
    rhs_v = rhs[r];
    nu2_v = nu2[r];
    return on ? n - (seg * SW + q * VW) : 0;
}

// LDS-resident part of the working matrix.  The first L chunks of every
// lane group's (row, segment) sequence stay in LDS for the whole solve: slot
// (l, kk, tid) holds the thread's own vector kk of chunk l, so the thread
// that fills a slot is the only one that reads it.  Rows whose last segment
// is resident keep their right-hand side and squared norm in LDS as well
// (rhs, nn at group row * NG + group); every lane of the group writes the
// same value there and reads back its own write.
struct ResLds {
    const uint4* chunks;
    const double* rhs;
    const double* nn;
    int L;
};

// The load ring of a streamed walk: kD chunk slots with the right-hand
// side, squared norm and element limit of each (registers).  Its first
// loads are not issued across iterations: they are about a third of an
// iteration's streamed bytes, and with the in-order load counter any later
// wait (exchange polls, the projection's row) would wait for them too.
template <class Tag, int kD> struct Ring {
    uint4 buf[kD][chunk_k<Tag>()];
    double pr[kD], pn[kD];
    int lim[kD];
};

// Register-resident chunks: the RG chunks that follow the LDS-resident ones
// in each lane group's walk, loaded once before the loop and kept in spare
// registers for the whole solve (with their right-hand sides, norms and
// element limits), so the ring streams RG fewer chunks per iteration.
template <class Tag, int RG> struct RegRes {
    uint4 buf[RG > 0 ? RG : 1][chunk_k<Tag>()];
    double pr[RG > 0 ? RG : 1], pn[RG > 0 ? RG : 1];
    int lim[RG > 0 ? RG : 1];
};

// Loads the register chunks: chunks L, L+1, ..., L+RG-1 of each group's walk
// over rows [r0, r1) (those past the group's last chunk are off).
template <class Tag, bool VEC, int LPR, int RG>
__device__ __forceinline__ void fill_regres(RegRes<Tag, RG>& G, const typename Elem<Tag>::S* __restrict__ A,
                                            int64_t lda, int n, int nseg, int r0, int r1,
                                            const double* __restrict__ rhs, const double* __restrict__ nu2, int L)
{
    using E = Elem<Tag>;
    constexpr int VW = VEC ? E::kVec : 1;
    constexpr int NG = kNT / LPR;
    constexpr int KK = chunk_k<Tag>();
    const int q = threadIdx.x % LPR;
    const int g = threadIdx.x / LPR;
    const int span = r1 - r0;
    const int nrows = span > g ? (span - g + NG - 1) / NG : 0;
    const int nchunk = nrows * nseg;
    if (span <= 0) return;  // no rows: nothing to hold (and r0 may be d, past the last row)
#pragma unroll
    for (int u = 0; u < RG; ++u) {
        const int c = L + u;
        const int row = c / nseg, seg = c - (c / nseg) * nseg;
        G.lim[u] = load_chunk<Tag, VW, LPR, KK>(G.buf[u], G.pr[u], G.pn[u], A, lda, n, r0 + g + NG * row, r0, seg, q,
                                                c < nchunk, rhs, nu2);
    }
}

// Issues the ring's first kD loads: chunks L, L+1, ... of each lane group's
// walk over rows [r0, r1) (the first L are LDS- or register-resident).
template <class Tag, bool VEC, int LPR, int kD>
__device__ __forceinline__ void ring_prime(Ring<Tag, kD>& R, const typename Elem<Tag>::S* __restrict__ A,
                                           int64_t lda, int n, int nseg, int r0, int r1,
                                           const double* __restrict__ rhs, const double* __restrict__ nu2, int L,
                                           bool rv)
{
    using E = Elem<Tag>;
    constexpr int VW = VEC ? E::kVec : 1;
    constexpr int NG = kNT / LPR;
    constexpr int KK = chunk_k<Tag>();
    const int q = threadIdx.x % LPR;
    const int g = threadIdx.x / LPR;
    const int span = r1 - r0;
    const int nrows = span > g ? (span - g + NG - 1) / NG : 0;
    const int nchunk = nrows * nseg;
    const int nchunk_max = (span > 0 ? (span + NG - 1) / NG : 0) * nseg;
    const int Lg = min(L, nchunk_max);
    if (nchunk_max - Lg <= 0) return;
    const int R0 = Lg / nseg, Rtot = nchunk_max / nseg;
    int irow = Lg / nseg, iseg = Lg - (Lg / nseg) * nseg;
#pragma unroll
    for (int u = 0; u < kD; ++u) {
        const int prow = rv ? R0 + Rtot - 1 - irow : irow;
        R.lim[u] = load_chunk<Tag, VW, LPR, KK>(R.buf[u], R.pr[u], R.pn[u], A, lda, n, r0 + g + NG * prow, r0, iseg,
                                                q, irow < Rtot && prow * nseg + iseg < nchunk, rhs, nu2);
        if (++iseg == nseg) { iseg = 0; ++irow; }
    }
}

// Residuals, candidates and partial ||r||^2 for rows [r0, r1) of the
// workgroup.  Lane groups of LPR lanes share a row; a row is split into
// nseg segments of LPR*VW*kK columns; the group walks its (row, segment)
// chunks in order: first the LDS-resident ones, then the rest from memory
// with kD chunks in flight (their loads are issued before the resident
// chunks are consumed).  xs is the operand vector in LDS (x for FP64,
// x - x_ref in FP32 for the low-precision product), zero beyond n up to
// nseg*SW; rhs is bt (exact) or r_ref (inner).  When rout is non-null the
// residuals are stored there (a refresh), and for the first nrow_out group
// rows also in the LDS array lrout.  With rev, the streamed rows are walked
// from the last to the first (segments still in order, so every sum is the
// same): alternating the direction every iteration starts each walk on the
// rows the previous one read last, some of which are still in L2.  The FP64
// loop alternates (1.3% faster at A 200000 x 1000, d = 20000); the
// low-precision inner product does not (FP32 measured 2.7% slower).
template <class Tag, bool VEC, int LPR, int kD, bool ROUT, bool M, int RG = 0>
__device__ __forceinline__ void stream_rows(const typename Elem<Tag>::S* __restrict__ A, int64_t lda, int n,
                                            int nseg, int r0, int r1, const typename Elem<Tag>::Op* __restrict__ xs,
                                            const double* __restrict__ rhs, double* __restrict__ rout,
                                            const double* __restrict__ nu2, Red& loc, const ResLds& res,
                                            double* lrout, int nrow_out, double dscale = 1.0, bool rev = false,
                                            const RegRes<Tag, RG>* reg = nullptr)
{
    Ring<Tag, kD> R;
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
    const int Lg = min(res.L, nchunk_max);
    const int Lr = RG > 0 ? min(RG, nchunk_max - Lg) : 0;  // register chunks in use
    const int Ls = Lg + Lr;                   // first streamed chunk
    // The streamed part is padded to whole rounds of the ring so that every
    // slot is consumed and refilled unconditionally (the extra chunks are
    // off: one shared cache line, masked); the compiler then tracks the
    // in-order load counter exactly and waits only for the slot in use.
    const int nstream = nchunk_max - Ls;
    const int nround = (nstream + kD - 1) / kD;
    // reversed walk: streamed group row irow (R0 <= irow < Rtot) reads
    // physical row R0 + Rtot - 1 - irow; only when the resident part ends on
    // a row (padding chunks past Rtot stay off)
    const bool rv = rev && (Ls % nseg) == 0;
    const int R0 = Ls / nseg, Rtot = nchunk_max / nseg;

    auto finish = [&](int crow, Acc s, double pr, double nn) {
        const int row = r0 + g + NG * crow;
        double r;
        if constexpr (std::is_same<Tag, tag_f16>::value) r = pr - static_cast<double>(s) * dscale;  // scaled operand
        else r = pr - static_cast<double>(s);
        if constexpr (ROUT) {
            if (rout) rout[row] = r;
            if (crow < nrow_out) lrout[crow * NG + g] = r;
        }
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

    auto& buf = R.buf;
    auto& pr = R.pr;  // right-hand side and squared norm of the slot's row
    auto& pn = R.pn;
    auto& lim = R.lim;  // valid elements of the slot from this lane's first column
    ring_prime<Tag, VEC, LPR, kD>(R, A, lda, n, nseg, r0, r1, rhs, nu2, Ls, rv);
    int iload = Ls + kD;  // next chunk to load
    int irow = iload / nseg, iseg = iload - (iload / nseg) * nseg;
    int crow = 0, cseg = 0;  // next chunk to consume
    Acc acc = Acc(0);
    for (int c = 0; c < Lg; ++c) {
        const uint4* slot = res.chunks + (size_t)c * KK * kNT + threadIdx.x;
        const int cbase = cseg * SW + q * VW;
        const int l0 = c < nchunk ? n - cbase : 0;
#pragma unroll
        for (int kk = 0; kk < KK; ++kk)
            acc += E::template dot<VW, M>(slot[kk * kNT], xs + cbase + kk * LPR * VW, l0 - kk * LPR * VW);
        if (cseg == nseg - 1) {
            const Acc s = group_sum_t<Acc, LPR>(acc);
            acc = Acc(0);
            if (c < nchunk) finish(crow, s, res.rhs[crow * NG + g], res.nn[crow * NG + g]);
        }
        if (++cseg == nseg) { cseg = 0; ++crow; }
    }
    // the register chunks (chunks Lg .. Ls - 1 of the walk, in order)
    if constexpr (RG > 0) {
#pragma unroll
        for (int u = 0; u < RG; ++u) {
            if (u < Lr) {
                const int c = Lg + u;
                const int cbase = cseg * SW + q * VW;
#pragma unroll
                for (int kk = 0; kk < KK; ++kk)
                    acc += E::template dot<VW, M>(reg->buf[u][kk], xs + cbase + kk * LPR * VW, reg->lim[u] - kk * LPR * VW);
                if (cseg == nseg - 1) {
                    const Acc s = group_sum_t<Acc, LPR>(acc);
                    acc = Acc(0);
                    if (c < nchunk) finish(crow, s, reg->pr[u], reg->pn[u]);
                }
                if (++cseg == nseg) { cseg = 0; ++crow; }
            }
        }
    }
    // consume the next chunk of the ring (group row crow, segment cseg)
    auto consume = [&](const uint4 (&v)[KK], int lm, double p, double nn) {
        const int cbase = cseg * SW + q * VW;
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) acc += E::template dot<VW, M>(v[kk], xs + cbase + kk * LPR * VW, lm - kk * LPR * VW);
        if (cseg == nseg - 1) {
            const Acc s = group_sum_t<Acc, LPR>(acc);
            acc = Acc(0);
            const int pc = rv ? R0 + Rtot - 1 - crow : crow;
            if (crow < Rtot && pc * nseg + cseg < nchunk) finish(pc, s, p, nn);
        }
        if (++cseg == nseg) { cseg = 0; ++crow; }
    };
    // all rounds but the last refill every slot; the last one, a
    // straight-line epilogue, issues no loads that nothing would consume
    for (int rd = 0; rd + 1 < nround; ++rd) {
#pragma unroll
        for (int u = 0; u < kD; ++u) {
            consume(buf[u], lim[u], pr[u], pn[u]);
            const int prow = rv ? R0 + Rtot - 1 - irow : irow;
            lim[u] = load_chunk<Tag, VW, LPR, KK>(buf[u], pr[u], pn[u], A, lda, n, r0 + g + NG * prow, r0, iseg, q,
                                                  irow < Rtot && prow * nseg + iseg < nchunk, rhs, nu2);
            ++iload;
            if (++iseg == nseg) { iseg = 0; ++irow; }
        }
    }
    if (nround > 0) {
#pragma unroll
        for (int u = 0; u < kD; ++u) consume(buf[u], lim[u], pr[u], pn[u]);
    }
}

// Fills the LDS-resident chunks (the first L of each group's sequence) and,
// for rows whose last segment is resident, their right-hand side and norm.
// Elements past n (or of rows the group does not own) are masked when the
// chunks are consumed, so their loaded bits do not matter.
template <class Tag, bool VEC, int LPR>
__device__ void fill_resident(const typename Elem<Tag>::S* __restrict__ A, int64_t lda, int n, int nseg, int r0,
                              int r1, const double* __restrict__ rhs, const double* __restrict__ nu2, uint4* chunks,
                              double* lrhs, double* lnn, int L)
{
    using E = Elem<Tag>;
    constexpr int VW = VEC ? E::kVec : 1;
    constexpr int NG = kNT / LPR;
    constexpr int KK = chunk_k<Tag>();
    const int q = threadIdx.x % LPR;
    const int g = threadIdx.x / LPR;
    const int span = r1 - r0;
    const int nrows = span > g ? (span - g + NG - 1) / NG : 0;
    const int nchunk = nrows * nseg;
    // a workgroup past the last row (r0 = d) holds nothing: none of its
    // chunks is ever read, and row r0 would lie outside the matrix
    if (span <= 0) return;
    for (int c = 0; c < L; ++c) {
        const int crow = c / nseg, seg = c - (c / nseg) * nseg;
        uint4 v[KK];
        double pr, pn;
        load_chunk<Tag, VW, LPR, KK>(v, pr, pn, A, lda, n, r0 + g + NG * crow, r0, seg, q, c < nchunk, rhs, nu2);
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) chunks[((size_t)c * KK + kk) * kNT + threadIdx.x] = v[kk];
        if (seg == nseg - 1) {
            lrhs[crow * NG + g] = pr;
            lnn[crow * NG + g] = pn;
        }
    }
}

// LDS carve of the solve: x (FP64), x - x_ref in the accumulation type
// (mixed), this workgroup's slice of x_ref, the residuals of its rows (the
// relaxed greedy randomized rule), then the resident right-hand sides and
// norms and the resident chunks (16-byte aligned).
struct SolveLds {
    size_t sx, sd, sdb, sxr, sres, lrhs, lnn, chunks, total;
};

__host__ __device__ inline size_t al_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// mixed: x - x_ref in FP32 (4 bytes per element); op16: also its 16-bit copy
__host__ __device__ inline SolveLds solve_lds(int npad, bool mixed, int xslice, int L, int ng, int layer_bytes,
                                              bool op16 = false, int rres = 0)
{
    SolveLds o;
    size_t at = 0;
    o.sx = at;
    at += (size_t)npad * 8;
    o.sd = at;
    at += mixed ? (size_t)npad * 4 : 0;
    at = al_up(at, 16);
    o.sdb = at;
    at += op16 ? (size_t)npad * 2 : 0;
    at = al_up(at, 8);
    o.sxr = at;
    at += (size_t)xslice * 8;
    o.sres = at;
    at += (size_t)rres * 8;
    o.lrhs = at;
    at += (size_t)L * ng * 8;
    o.lnn = at;
    at += (size_t)L * ng * 8;
    at = al_up(at, 16);
    o.chunks = at;
    at += (size_t)L * layer_bytes;
    o.total = at;
    return o;
}

// The relaxed greedy randomized rule's threshold t_k = theta M + (1 - theta)
// (R / F), capped at M, as separate IEEE operations (no fused multiply-add).
__device__ __forceinline__ double rgrk_threshold(double theta, double M, double R, double F)
{
#pragma clang fp contract(off)
    const double t = theta * M + (1.0 - theta) * (R / F);
    return t > M ? M : t;
}

// The candidate of one row from its residual r and squared norm nn (the
// weighted-residual rule; rows of zero norm are never selected).
__device__ __forceinline__ void row_candidate(Red& loc, uint32_t row, double r, double nn)
{
    loc.r2 += r * r;
    if (nn > 0.0) {
        const double score = (r * r) / nn;
        if (!isfinite(score)) {
            loc.flags |= kFlagNonfinite;
        } else if (cand_better(score, row, loc.score, loc.idx)) {
            loc.score = score;
            loc.r = r / nn;
            loc.idx = row;
        }
    } else if (isnan(nn)) {
        loc.flags |= kFlagNonfinite;
    }
}

// The refresh residual of the mixed loop from a CSR A: r_ref = S (b - A x)
// (equal to bt - At x in exact arithmetic, and reading the CSR A, about
// 12 bytes per stored entry, instead of the d x n FP64 sketch).  Every
// workgroup forms y_i = b_i - sum_e val_e x_col(e) for its share of the m
// rows (the row's stored entries in order, summed from zero in FP64) and
// publishes it; after a grid barrier each workgroup sums, for each of its
// rows j of the sketch, D_ii y_i over the rows i of bucket j in ascending
// order (the sketch's order), stores r_ref and the LDS copy of resident
// rows, and forms the candidates as the streamed refresh does.
template <int LPR>
__device__ void refresh_from_csr(const CsrRef& R, const SolveSys& S, const double* __restrict__ sx, int r0, int r1,
                                 int nrow_res, double* lrhs, Red& loc, int wg, int G, uint32_t epoch, uint32_t* s_ok,
                                 bool& ok)
{
    constexpr int NG = kNT / LPR;
    const int64_t per = (R.m + G - 1) / G;
    const int64_t i0 = min(R.m, (int64_t)wg * per), i1 = min(R.m, i0 + per);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kNT) {
        const int64_t e0 = R.rp[i], e1 = R.rp[i + 1];
        double s = 0.0;
        for (int64_t e = e0; e < e1; ++e) s += static_cast<double>(R.val[e]) * sx[R.col[e]];
        coh_store(&R.y[i], R.b[i] - s);
    }
    ok = grid_barrier_flags(R.flags, wg, G, epoch, s_ok) && ok;
    for (int j = r0 + (int)threadIdx.x; j < r1; j += kNT) {
        const uint32_t p0 = R.ptr[j], p1 = R.ptr[j + 1];
        double r = 0.0;
        uint32_t p = p0;
        // four rows' loads in flight, added in order
        for (; p + 4 <= p1; p += 4) {
            uint32_t i[4];
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) i[u] = R.perm[p + u];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = coh_load(&R.y[i[u]]);
#pragma unroll
            for (int u = 0; u < 4; ++u) r += draw_sign(draw_word(R.seed, i[u])) * v[u];
        }
        for (; p < p1; ++p) {
            const uint32_t i = R.perm[p];
            r += draw_sign(draw_word(R.seed, i)) * coh_load(&R.y[i]);
        }
        S.rref[j] = r;
        const int lj = j - r0;
        if (lj / NG < nrow_res) lrhs[(lj / NG) * NG + lj % NG] = r;
        row_candidate(loc, static_cast<uint32_t>(j), r, S.nu2[j]);
    }
}

// SEL 0: the greedy rule of Algorithm 1 (largest weighted residual).
// SEL 1: the relaxed greedy randomized rule (FP64 only): after the first
// reduction (largest score M, ||r||^2 = R, stop measure) every workgroup
// forms its rows' working-set test r_i^2 / ||At^(i)||^2 >= t_k from the
// residuals it kept in LDS, gives each member the key r_i^2 / E_i with E_i
// = -log(u) a unit exponential from the selection stream (position k d + i),
// and a second reduction picks the largest key: row i wins with probability
// r_i^2 over the members' sum.
template <class Tag, bool VEC, int LPR, bool GRID, bool M, int SEL = 0>
__device__ __forceinline__ void solve_loop(const SolveSys& S, const Ctl& C, XRec* exch, int wg, int G, char* smem)
{
    constexpr bool MIXED = !std::is_same<Tag, tag_f64>::value;
    static_assert(SEL == 0 || !MIXED, "the randomized rule runs on the FP64 sketch");
    using LPS = typename Elem<Tag>::S;
    using LAcc = typename Elem<Tag>::Acc;
    constexpr int SW64 = LPR * (VEC ? 2 : 1) * kK;
    constexpr int SWLP = LPR * (VEC ? Elem<Tag>::kVec : 1) * chunk_k<Tag>();
    constexpr int NG = kNT / LPR;
    constexpr int LAYER = kNT * chunk_k<Tag>() * 16;
    __shared__ Red slots[kNW];
    __shared__ Red slots2[kNW];  // the exchange's reduction (one barrier each)
    __shared__ uint32_t s_bar;   // grid barrier of the refresh from a CSR A
    uint32_t csr_epoch = 0;

    const int tid = threadIdx.x;
    const int n = S.n;
    const int d = S.d;
    const int npad = S.npad;
    const int nseg64 = (n + SW64 - 1) / SW64;
    const int nseglp = (n + SWLP - 1) / SWLP;
    const int nseg_res = MIXED ? nseglp : nseg64;  // the stream that uses the resident chunks

    const int rows_per = (d + G - 1) / G;
    const int r0 = min(d, wg * rows_per);
    const int r1 = min(d, r0 + rows_per);
    const int cols_per = (n + G - 1) / G;
    const int e0 = min(n, wg * cols_per);
    const int e1 = min(n, e0 + cols_per);
    // resident chunks: at most what LDS was sized for, and no more than the
    // longest group sequence of this workgroup
    const int gmax_rows = rows_per > 0 ? (rows_per + NG - 1) / NG : 0;
    const int L = min(C.res_layers, gmax_rows * nseg_res);

    constexpr bool OP16 = op16<Tag>();
    const SolveLds lay = solve_lds(npad, MIXED, C.xslice, C.res_layers, NG, LAYER, OP16, SEL ? C.rres : 0);
    double* sx = reinterpret_cast<double*>(smem + lay.sx);   // x, FP64, zero past n
    LAcc* sd = reinterpret_cast<LAcc*>(smem + lay.sd);       // x - x_ref (mixed), zero past n
    uint16_t* sdb = reinterpret_cast<uint16_t*>(smem + lay.sdb);  // its 16-bit copy (OP16)
    double* sxr = reinterpret_cast<double*>(smem + lay.sxr); // x_ref[e0 .. e1)
    double* sres = reinterpret_cast<double*>(smem + lay.sres);  // r_i of rows r0 + j (SEL 1)
    double* lrhs = reinterpret_cast<double*>(smem + lay.lrhs);
    double* lnn = reinterpret_cast<double*>(smem + lay.lnn);
    uint4* lchunks = reinterpret_cast<uint4*>(smem + lay.chunks);
    const ResLds res{lchunks, lrhs, lnn, L};
    const ResLds none{nullptr, nullptr, nullptr, 0};

    // x lives in LDS (sx); each thread owns columns tid + j*kNT and is the
    // only writer of them.  Mixed precision also keeps x - x_ref in the
    // accumulation type (sd): the projections since the last refresh summed
    // in FP32, whose rounding is far below that of the low-precision rows.
    for (int c = tid; c < npad; c += kNT) {
        sx[c] = (c < n && S.x0) ? S.x0[c] : 0.0;
        if (MIXED) sd[c] = LAcc(0);
        if (OP16) sdb[c] = 0;
    }
    if (S.xref && C.xslice > 0)
        for (int c = e0 + tid; c < e1; c += kNT) sxr[c - e0] = S.xref[c];
    if (MIXED)
        fill_resident<Tag, VEC, LPR>(static_cast<const LPS*>(S.At), S.ldat, n, nseglp, r0, r1, S.bt, S.nu2, lchunks,
                                     lrhs, lnn, L);
    else
        fill_resident<tag_f64, VEC, LPR>(S.At64, S.ldat64, n, nseg64, r0, r1, S.bt, S.nu2, lchunks, lrhs, lnn, L);
    const int nrow_res = L / nseg_res;  // group rows whose last segment is resident
    // the FP64 greedy loop over 16-byte rows keeps the chunks after the LDS
    // ones in registers
    constexpr int RG = (!MIXED && SEL == 0 && VEC) ? kRegChunks : 0;
    RegRes<tag_f64, RG> regres;
    if constexpr (RG > 0) fill_regres<tag_f64, VEC, LPR, RG>(regres, S.At64, S.ldat64, n, nseg64, r0, r1, S.bt, S.nu2, L);
    // ||x_ref||^2 and ||bt||^2, reduced identically by every workgroup.
    Red q = red_identity();
    if (S.xref)
        for (int c = tid; c < n; c += kNT) q.e2 += S.xref[c] * S.xref[c];
    for (int i = tid; i < d; i += kNT) q.r2 += S.bt[i] * S.bt[i];
    q = block_red<kNT>(q, slots);
    const double xref2 = q.e2;
    const double bt2 = q.r2;
    double fro2 = 0.0;  // ||At||_F^2 (SEL 1)
    if constexpr (SEL == 1) {
        Red f = red_identity();
        for (int i = tid; i < d; i += kNT) f.r2 += S.nu2[i];
        fro2 = block_red<kNT>(f, slots).r2;
    }
    const double tol2 = C.tol2;
    const bool rel_err = S.stop_mode == CSK_STOP_REL_ERR;

    const typename Elem<Tag>::Op* op_lp;  // the low-precision product's operand
    if constexpr (OP16) op_lp = sdb;
    else op_lp = reinterpret_cast<const typename Elem<Tag>::Op*>(sd);
    float fscale = 1.f;   // FP16 operand: 2^e of the current refresh window
    double dscale = 1.0;  // and 2^-e
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
        if (MIXED && refresh && C.cref) {
            // the refresh residual from the CSR A; every workgroup of the
            // grid (or the one workgroup) takes part
            bool ok = true;
            refresh_from_csr<LPR>(*C.cref, S, sx, r0, r1, nrow_res, lrhs, loc, wg, G, ++csr_epoch, &s_bar, ok);
            if (!ok) loc.flags |= kFlagTimeout;
        } else if (MIXED && refresh) {
            // the refresh product of the mixed mode runs once per window: a
            // shallower ring leaves the registers to the working-precision one
            // (it streams every chunk: the resident ones are low precision)
            stream_rows<tag_f64, VEC, LPR, 2, true, M>(S.At64, S.ldat64, n, nseg64, r0, r1, sx, S.bt, S.rref, S.nu2,
                                                    loc, none, lrhs, nrow_res);
        } else if (MIXED && exact) {
            stream_rows<tag_f64, VEC, LPR, 2, false, M>(S.At64, S.ldat64, n, nseg64, r0, r1, sx, S.bt, nullptr, S.nu2,
                                                     loc, none, nullptr, 0);
        } else if constexpr (!MIXED && SEL == 1) {
            stream_rows<tag_f64, VEC, LPR, ring_depth<tag_f64>(), true, M>(S.At64, S.ldat64, n, nseg64, r0, r1, sx,
                                                                        S.bt, nullptr, S.nu2, loc, res, sres,
                                                                        gmax_rows, 1.0, (k & 1) != 0);
        } else if constexpr (!MIXED) {
            // the register chunks take the registers of all ring slots but
            // one: eight waves per CU with one 8 KB chunk in flight each
            // still cover the Infinity Cache's latency, and every chunk held
            // in registers is one the ring no longer streams
            constexpr int kDg = RG > 0 ? 1 : ring_depth<tag_f64>();
            stream_rows<tag_f64, VEC, LPR, kDg, false, M, RG>(S.At64, S.ldat64, n, nseg64, r0, r1, sx, S.bt, nullptr,
                                                           S.nu2, loc, res, nullptr, 0, 1.0, (k & 1) != 0, &regres);
        } else {
            stream_rows<Tag, VEC, LPR, ring_depth<Tag>(), false, M>(static_cast<const LPS*>(S.At), S.ldat, n, nseglp,
                                                                 r0, r1, op_lp, S.rref, nullptr, S.nu2, loc, res,
                                                                 nullptr, 0, dscale);
        }
        if (S.xref)
            for (int c = e0 + tid; c < e1; c += kNT) {
                const double e = sx[c] - (C.xslice > 0 ? sxr[c - e0] : S.xref[c]);
                loc.e2 += e * e;
            }
        if (wg == 0 && tid == 0 && C.cancel && (k % C.check_every) == 0 && *C.cancel != 0)
            loc.flags |= kFlagCancel;
        Red tot = block_red1<kNT>(loc, slots);
        if constexpr (GRID) tot = exchange<kNT>(tot, exch, wg, G, k, slots2, rel_err, SEL == 1);

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

        double alpha = tot.r;
        uint32_t pick = tot.idx;
        if constexpr (SEL == 1) {
            const double thr = rgrk_threshold(C.theta, tot.score, tot.r2, fro2);
            const uint64_t base = static_cast<uint64_t>(k) * static_cast<uint64_t>(d);
            Red cand = red_identity();
            for (int j = tid; j < r1 - r0; j += kNT) {
                const double nn = S.nu2[r0 + j];
                if (!(nn > 0.0)) continue;
                const double r = sres[j];
                const double w = r * r;
                if (!(w / nn >= thr)) continue;
                const double e = -log(select_uniform(C.sel_seed, base + static_cast<uint64_t>(r0 + j)));
                const double key = w / e;
                if (cand_better(key, static_cast<uint32_t>(r0 + j), cand.score, cand.idx)) {
                    cand.score = key;
                    cand.r = r / nn;
                    cand.idx = static_cast<uint32_t>(r0 + j);
                }
            }
            // slot arrays alternate with the reductions before (one barrier each)
            Red t2 = block_red1<kNT>(cand, GRID ? slots : slots2);
            if constexpr (GRID) t2 = exchange<kNT>(t2, exch + 2 * (size_t)G, wg, G, k, slots2, false);
            if (t2.flags & kFlagTimeout) { status = CSK_ERR_DEVICE; break; }
            if (t2.idx >= (uint32_t)d) { status = CSK_ERR_DEVICE; break; }  // the best row is always a member
            alpha = t2.r;
            pick = t2.idx;
        }

        // Projection onto row i_k, on this workgroup's copy of x.
        if (C.trace && wg == 0 && tid == 0) C.trace[k] = pick;
        const double* __restrict__ arow = S.At64 + (int64_t)pick * S.ldat64;
        if (std::is_same<Tag, tag_f16>::value && refresh) {
            // ||alpha a|| = |r| / ||a|| = sqrt(score), identical in every workgroup
            int ex = 0;
            frexp(sqrt(tot.score), &ex);
            const int e = min(100, max(-100, 5 - ex));
            fscale = ldexpf(1.f, e);
            dscale = ldexp(1.0, -e);
        }
#pragma unroll 2
        for (int c = tid; c < n; c += kNT) {
            const double a = arow[c];
            sx[c] = sx[c] + alpha * a;
            if (MIXED) {
                const LAcc nv = (refresh ? LAcc(0) : sd[c]) + static_cast<LAcc>(alpha * a);
                sd[c] = nv;
                if constexpr (std::is_same<Tag, tag_bf16>::value)
                    sdb[c] = __builtin_bit_cast(uint16_t, static_cast<__bf16>(nv));
                else if constexpr (std::is_same<Tag, tag_f16>::value)
                    sdb[c] = __builtin_bit_cast(uint16_t, static_cast<_Float16>(nv * fscale));
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

// M: per-element masks of the product.  Without them (n a multiple of the
// vector width, vector path) every vector lies wholly before or wholly past
// column n, and one past it multiplies the zero padding of the operand
// vector, so only the discarded sums of lane groups without a row see
// elements that the masks would have removed.
template <class Tag, bool VEC, int LPR, bool M>
__global__ __launch_bounds__(kNT) void k_solve_grid(SolveSys S, Ctl C)
{
    extern __shared__ __align__(16) char smem[];
    solve_loop<Tag, VEC, LPR, true, M>(S, C, C.exch, blockIdx.x, gridDim.x, smem);
}

template <class Tag, bool VEC, int LPR, bool M>
__global__ __launch_bounds__(kNT) void k_solve_single(SolveSys S, Ctl C)
{
    extern __shared__ __align__(16) char smem[];
    solve_loop<Tag, VEC, LPR, false, M>(S, C, nullptr, 0, 1, smem);
}

// The relaxed greedy randomized rule on the FP64 sketch (exchange records:
// two sets of [2][grid]).
template <bool VEC, int LPR, bool M>
__global__ __launch_bounds__(kNT) void k_solve_rgrk_grid(SolveSys S, Ctl C)
{
    extern __shared__ __align__(16) char smem[];
    solve_loop<tag_f64, VEC, LPR, true, M, 1>(S, C, C.exch, blockIdx.x, gridDim.x, smem);
}

template <bool VEC, int LPR, bool M>
__global__ __launch_bounds__(kNT) void k_solve_rgrk_single(SolveSys S, Ctl C)
{
    extern __shared__ __align__(16) char smem[];
    solve_loop<tag_f64, VEC, LPR, false, M, 1>(S, C, nullptr, 0, 1, smem);
}

// The batch's sketches live in the library's own layout, rows padded to 64
// bytes with zeros, so the product needs no per-element masks: a vector
// that straddles column n reads zeros past it.
// Work items in queue order: queue position p owns items
// [item_off[p], item_off[p+1]); a system with one item runs the
// single-workgroup loop, a split one the grid loop over its P items with its
// own exchange records.  The launch is cooperative (every workgroup
// resident) and items are claimed in order, so the parts of a split system
// are always all claimed: only the most recently claimed system can be
// incomplete, and a free workgroup claims its next part.
template <class Tag, bool VEC, int LPR>
__global__ __launch_bounds__(kNT) void k_solve_batched(const SolveSys* __restrict__ sys, Ctl C)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ int32_t s_next;
    const int32_t nitems = C.item_off[C.nsys];
    for (;;) {
        if (threadIdx.x == 0) s_next = static_cast<int32_t>(atomicAdd(C.queue, 1u));
        __syncthreads();
        const int32_t item = s_next;
        __syncthreads();
        if (item >= nitems) break;
        int lo = 0, hi = C.nsys;  // item_off[lo] <= item < item_off[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (C.item_off[mid] <= item) lo = mid;
            else hi = mid;
        }
        const int parts = C.item_off[lo + 1] - C.item_off[lo];
        const SolveSys S = sys[C.order[lo]];
        if (parts == 1)
            solve_loop<Tag, VEC, LPR, false, false>(S, C, nullptr, 0, 1, smem);
        else
            solve_loop<Tag, VEC, LPR, true, false>(S, C, C.exch + C.exch_off[lo], item - C.item_off[lo], parts, smem);
        __syncthreads();
    }
}

// The refresh descriptor into device memory (a kernel, so the call records
// into a captured graph like any other launch).
__global__ void k_store_csr_ref(CsrRef v, CsrRef* dst) { *dst = v; }

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

constexpr int kMaxResLayers = 16;
constexpr size_t kLdsReserve = 2048;  // static LDS of the kernels, rounded up

// Sizes the LDS of a solve launch: the operand vectors, the x_ref slice,
// then as many resident chunk layers as fit (never more than `want`).
template <class Tag, int LPR>
SolveLds plan_lds(int npad, int& xslice, int want, int& layers, int rres = 0)
{
    const bool mixed = !std::is_same<Tag, tag_f64>::value;
    constexpr bool o16 = op16<Tag>();
    constexpr int NG = kNT / LPR;
    constexpr int LAYER = kNT * chunk_k<Tag>() * 16;
    const size_t cap = (size_t)device_max_lds() - kLdsReserve;
    // the x_ref slice is a convenience: without room it is read from memory
    if (xslice > 0 && solve_lds(npad, mixed, xslice, 0, NG, LAYER, o16, rres).total > cap) xslice = 0;
    int L = std::max(0, std::min(want, kMaxResLayers));
    while (L > 0 && solve_lds(npad, mixed, xslice, L, NG, LAYER, o16, rres).total > cap) --L;
    layers = L;
    return solve_lds(npad, mixed, xslice, L, NG, LAYER, o16, rres);
}

template <class Tag, bool VEC, int LPR, bool M, int SEL>
csk_status launch_solve(const SolveSys& S, Ctl C, int grid, hipStream_t st)
{
    constexpr bool mixed = !std::is_same<Tag, tag_f64>::value;
    constexpr int NG = kNT / LPR;
    const int sw = LPR * (VEC ? (mixed ? Elem<Tag>::kVec : 2) : 1) * chunk_k<Tag>();
    const int nseg = (S.n + sw - 1) / sw;
    const int g = std::max(grid, 1);
    const int rows_per = (S.d + g - 1) / g;
    const int want = ((rows_per + NG - 1) / NG) * nseg;
    C.xslice = S.xref ? (S.n + g - 1) / g : 0;
    C.rres = SEL ? ((rows_per + NG - 1) / NG) * NG : 0;
    const SolveLds lay = plan_lds<Tag, LPR>(S.npad, C.xslice, want, C.res_layers, C.rres);
    const size_t shm = lay.total;
    if (shm > (size_t)device_max_lds() - kLdsReserve) {
        set_error("the solve needs %zu bytes of LDS per workgroup (n = %d, or rows per workgroup, too large)", shm,
                  S.n);
        return CSK_ERR_UNSUPPORTED;
    }
    if (grid <= 1) {
        auto kern = k_solve_single<Tag, VEC, LPR, M>;
        if constexpr (SEL == 1) kern = k_solve_rgrk_single<VEC, LPR, M>;
        CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        kern<<<1, kNT, shm, st>>>(S, C);
        CSK_LAUNCH_CHECK("k_solve_single");
        return CSK_OK;
    }
    auto kern = k_solve_grid<Tag, VEC, LPR, M>;
    if constexpr (SEL == 1) kern = k_solve_rgrk_grid<VEC, LPR, M>;
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

template <class Tag, bool VEC, bool M, int SEL>
csk_status dispatch_lpr(const SolveSys& S, const Ctl& C, const SolvePlan& p, hipStream_t st)
{
    switch (p.lpr) {
    case 4: return launch_solve<Tag, VEC, 4, M, SEL>(S, C, p.grid, st);
    case 16: return launch_solve<Tag, VEC, 16, M, SEL>(S, C, p.grid, st);
    default: return launch_solve<Tag, VEC, 64, M, SEL>(S, C, p.grid, st);
    }
}

template <class Tag, int SEL = 0>
csk_status dispatch_solve(const SolveSys& S, const Ctl& C, const SolvePlan& p, hipStream_t st)
{
    // whole vectors: n a multiple of the working type's vector width (and
    // so of FP64's, for the refresh product)
    if (p.vw > 1 && S.n % Elem<Tag>::kVec == 0) return dispatch_lpr<Tag, true, false, SEL>(S, C, p, st);
    if (p.vw > 1) return dispatch_lpr<Tag, true, true, SEL>(S, C, p, st);
    return dispatch_lpr<Tag, false, true, SEL>(S, C, p, st);
}

constexpr int kBatchLPR = 16;

template <class Tag>
csk_status launch_batched(const SolveSys* sys_dev, int32_t nsys, const BatchedPlan& bp, Ctl C, hipStream_t st)
{
    constexpr bool mixed = !std::is_same<Tag, tag_f64>::value;
    constexpr int NG = kNT / kBatchLPR;
    const int sw = kBatchLPR * (mixed ? Elem<Tag>::kVec : 2) * chunk_k<Tag>();
    const int64_t nseg = (bp.n_max + sw - 1) / sw;
    const int want = (int)std::min<int64_t>(kMaxResLayers, ((bp.d_max + NG - 1) / NG) * nseg);
    C.xslice = (int)bp.n_max;
    const SolveLds lay = plan_lds<Tag, kBatchLPR>((int)bp.npad_max, C.xslice, want, C.res_layers);
    const size_t shm = lay.total;
    if (shm > (size_t)device_max_lds() - kLdsReserve) {
        set_error("the batched solve needs %zu bytes of LDS per workgroup (n = %lld too large)", shm,
                  (long long)bp.n_max);
        return CSK_ERR_UNSUPPORTED;
    }
    auto kern = k_solve_batched<Tag, true, kBatchLPR>;
    CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    int per_cu = 0;
    CSK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), kNT, shm));
    const int cap = std::max(1, per_cu) * device_cu_count();

    // Split plan.  A system's time is modelled as its iteration count times
    // a per-iteration cost.  The iterations of the greedy loop on a
    // Gaussian-like sketch grow like n / (1 - sqrt(n/d))^2 (the square of
    // the sketch's condition number times n; fitted on the 512-system
    // workload, log error 0.12), so the longest-running systems are the
    // nearly square ones, not the largest.  The per-iteration cost is a
    // fixed part (about 2 us alone, 6 us when split, for the exchange) plus
    // the system's elements per part at one CU's streaming rate (about
    // 0.18 ns per element in FP32; a CU streams these rows at about
    // 20 GB/s, so splitting scales almost linearly).  Starting from one
    // part each, the system with the longest modelled time gets one more
    // part (at least 32 rows each, at most half the grid) while that
    // shortens the larger of the longest time and the average load per
    // workgroup.
    const double esz = (double)sizeof(typename Elem<Tag>::S);
    const double ce = 0.18e-3 * (esz == 2.0 ? 1.5 : esz == 8.0 ? 1.4 : 1.0);
    // plan variants (tuning): 1 never splits, 2 and 3 price the exchange of
    // a split system at half and twice the modelled cost
    const double split_cost = bp.variant == 2 ? 3.0 : bp.variant == 3 ? 12.0 : 6.0;
    auto model = [&](const SolveSys& S, int parts) {
        const double q = std::min(0.9, (double)S.n / (double)std::max(S.d, 1));
        const double iters = (double)S.n / ((1.0 - std::sqrt(q)) * (1.0 - std::sqrt(q)));
        return iters * ((parts > 1 ? split_cost : 2.0) + ce * (double)S.d * (double)S.n / parts);
    };
    std::vector<int> nparts(nsys, 1);
    std::vector<double> tsys(nsys);
    double total = 0.0;
    std::priority_queue<std::pair<double, int32_t>> heap;
    for (int32_t p = 0; p < nsys; ++p) {
        tsys[p] = model(bp.sys[bp.order[p]], 1);
        total += tsys[p];
        heap.push({tsys[p], p});
    }
    size_t rec = 0;
    while (!heap.empty()) {
        const int32_t p = heap.top().second;
        heap.pop();
        const SolveSys& S = bp.sys[bp.order[p]];
        const int cur = nparts[p];
        const int next = cur + 1;
        const int maxp = bp.variant == 1 ? 1 : std::max(1, std::min(cap / 2, S.d / 32));
        const size_t rec_next = rec - (cur > 1 ? 2 * (size_t)cur : 0) + 2 * (size_t)next;
        if (next > maxp || rec_next > bp.exch_records) break;
        const double t_next = model(S, next);
        const double total_next = total - cur * tsys[p] + next * t_next;
        const double crit_next = std::max(t_next, heap.empty() ? 0.0 : heap.top().first);
        if (std::max(crit_next, total_next / cap) >= std::max(tsys[p], total / cap)) break;
        nparts[p] = next;
        tsys[p] = t_next;
        total = total_next;
        rec = rec_next;
        heap.push({t_next, p});
    }
    std::vector<int32_t> item_off(nsys + 1), exch_off(nsys, 0);
    rec = 0;
    int32_t items = 0;
    for (int32_t p = 0; p < nsys; ++p) {
        const int parts = nparts[p];
        item_off[p] = items;
        exch_off[p] = (int32_t)rec;
        items += parts;
        if (parts > 1) rec += 2 * (size_t)parts;
    }
    item_off[nsys] = items;
    csk_status e = upload_i32(item_off.data(), nsys + 1, bp.item_off_dev, st);
    if (e == CSK_OK) e = upload_i32(exch_off.data(), nsys, bp.exch_off_dev, st);
    if (e != CSK_OK) return e;
    C.item_off = bp.item_off_dev;
    C.exch_off = bp.exch_off_dev;
    C.exch = static_cast<XRec*>(bp.exch_dev);
    if (rec > 0) {
        const int64_t words = (int64_t)rec * (int64_t)sizeof(XRec) / 4;
        k_zero_words<<<(int)std::min<int64_t>(256, (words + 255) / 256), 256, 0, st>>>(
            reinterpret_cast<uint32_t*>(bp.exch_dev), words);
        CSK_LAUNCH_CHECK("k_zero_words");
    }
    const int grid = std::max(1, std::min(items, cap));
    const SolveSys* s_arg = sys_dev;
    Ctl c_arg = C;
    void* args[] = {&s_arg, &c_arg};
    CSK_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(kNT), args,
                                       (unsigned)shm, st));
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
    C.trace = o->trace_idx;
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

// Lanes per row: the one of {64, 16, 4} whose segments cover the row with
// the fewest padded columns (elements past n cost the same work as real
// ones); ties go to the wider group (fewer segments per row).
int pick_lpr(int64_t n, int64_t per_lane)
{
    int best = 64;
    int64_t best_cover = -1;
    for (int lpr : {64, 16, 4}) {
        const int64_t sw = lpr * per_lane;
        const int64_t cover = (n + sw - 1) / sw * sw;
        if (best_cover < 0 || cover < best_cover) {
            best = lpr;
            best_cover = cover;
        }
    }
    return best;
}

// Tuned launch shapes of the persistent solve, keyed by (architecture, d, n,
// working dtype, vector path) in the shared tune store: written by
// csk_tune_solve, read by every default-shaped solve.
namespace {
std::string solve_tune_key(int64_t d, int64_t n, csk_dtype at_dtype, int vw)
{
    return tune_key("solve|d=%lld|n=%lld|dtype=%d|vw=%d", (long long)d, (long long)n, (int)at_dtype, vw);
}
}  // namespace

void tune_store(int64_t d, int64_t n, csk_dtype at_dtype, int vw, int grid, int lpr, double us)
{
    tune_put(solve_tune_key(d, n, at_dtype, vw), TuneRec{grid, lpr, us});
}

bool tune_lookup(int64_t d, int64_t n, csk_dtype at_dtype, int vw, int* grid, int* lpr, double* us)
{
    TuneRec r{};
    if (!tune_get(solve_tune_key(d, n, at_dtype, vw), &r)) return false;
    *grid = r.a;
    *lpr = r.b;
    if (us) *us = r.us;
    return true;
}

void tune_clear() { tune_reset(); }

int solve_vw(csk_dtype at_dtype, int64_t ldat, const void* At)
{
    const int64_t vec = 16 / (int64_t)dtype_size(at_dtype);
    return (al16(At) && ((ldat * (int64_t)dtype_size(at_dtype)) % 16 == 0)) ? (int)vec : 1;
}

SolvePlan solve_plan(int64_t d, int64_t n, csk_dtype at_dtype, int64_t ldat, const void* At,
                     const csk_solve_opts* o)
{
    SolvePlan p;
    p.block = kNT;
    const int64_t vec = 16 / (int64_t)dtype_size(at_dtype);
    const bool vec_ok = al16(At) && ((ldat * (int64_t)dtype_size(at_dtype)) % 16 == 0);
    p.vw = vec_ok ? (int)vec : 1;
    p.lpr = pick_lpr(n, (int64_t)p.vw * chunk_k_of(at_dtype));
    int grid;
    if (o && o->single_wg == 1) grid = 1;
    else if (o && o->grid > 0) grid = o->grid;
    else if (o && o->single_wg == 0) grid = std::max(2, std::min<int>(device_cu_count(), (int)((d + 15) / 16)));
    else {
        // One workgroup while the matrix fits its LDS (no exchange at all);
        // otherwise enough workgroups for each one's rows to stay in LDS
        // (about 64 KB each, at least 8 workgroups, at most one per CU and
        // at least 16 rows each): the exchange grows with the grid (2.4 us
        // at 8 workgroups, 3.8 at 256), the product of resident rows hardly
        // at all.  A 256 KB sketch takes 7.5 us per iteration in one
        // workgroup and 5.6 in eight.
        const int64_t bytes = d * n * (int64_t)dtype_size(at_dtype);
        const int64_t want = std::max<int64_t>(8, (bytes + (64 << 10) - 1) >> 16);
        grid = (bytes <= (int64_t)(96 << 10))
                   ? 1
                   : (int)std::max<int64_t>(2, std::min<int64_t>({(int64_t)device_cu_count(), want, (d + 15) / 16}));
    }
    // a shape from csk_tune_solve replaces the defaults (never an explicit choice)
    if (o && o->grid == 0 && o->single_wg == -1) {
        int tg = 0, tl = 0;
        if (tune_lookup(d, n, at_dtype, p.vw, &tg, &tl, nullptr) && tg >= 1 && tg <= device_cu_count()) {
            grid = tg;
            p.lpr = tl;
        }
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
                     void* ws, size_t ws_bytes, hipStream_t st, const SolvePlan* forced, const CsrRef* cref)
{
    SolveSys S = sys_in;
    SolvePlan plan = forced ? *forced : solve_plan(S.d, S.n, at_dtype, S.ldat, S.At, o);
    // The exact FP64 product shares the vector path, so At64 must qualify too.
    if (plan.vw > 1 && (!al16(S.At64) || (S.ldat64 * 8) % 16 != 0)) {
        plan.vw = 1;
        plan.lpr = pick_lpr(S.n, chunk_k_of(at_dtype));
    }
    S.npad = (int32_t)solve_npad(S.n, at_dtype, plan.lpr, plan.vw > 1);

    Carve c(ws);
    Ctl C = make_ctl(o);
    C.exch = c.take<XRec>(2 * (size_t)std::max(plan.grid, 1));
    S.rref = c.take<double>(S.d);
    double* nu2_ws = c.take<double>(S.d);
    if (cref) {
        if (at_dtype == CSK_F64 || plan.grid > kRefreshFlags) {
            set_error("the refresh from a CSR A needs a low-precision sketch and at most %d workgroups", kRefreshFlags);
            return CSK_ERR_INVALID_ARG;
        }
        if (!cref->self) {
            set_error("the refresh from a CSR A needs a device copy of its descriptor");
            return CSK_ERR_INVALID_ARG;
        }
        k_store_csr_ref<<<1, 1, 0, st>>>(*cref, cref->self);
        CSK_LAUNCH_CHECK("k_store_csr_ref");
        C.cref = cref->self;
        k_zero_words<<<4, 256, 0, st>>>(cref->flags, kRefreshFlags);
        CSK_LAUNCH_CHECK("k_zero_words");
    }
    if (c.bytes() > ws_bytes) {
        set_error("solve workspace too small: need %zu bytes, got %zu", c.bytes(), ws_bytes);
        return CSK_ERR_WORKSPACE;
    }
    if (S.nu2 == nullptr) {
        const csk_status e = launch_row_norms2(S.At64, S.ldat64, S.d, S.n, nu2_ws, st);
        if (e != CSK_OK) return e;
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

size_t solve_rgrk_ws_bytes(int64_t d, int64_t n, int grid)
{
    (void)n;
    Carve c(nullptr);
    c.take<XRec>(4 * (size_t)std::max(grid, 1));
    c.take<double>(d);  // nu2 when not supplied
    return c.bytes();
}

csk_status solve_rgrk_run(const SolveSys& sys_in, const csk_solve_opts* o, double theta, uint64_t sel_seed,
                          void* ws, size_t ws_bytes, hipStream_t st)
{
    SolveSys S = sys_in;
    const SolvePlan plan = solve_plan(S.d, S.n, CSK_F64, S.ldat64, S.At64, o);
    S.npad = (int32_t)solve_npad(S.n, CSK_F64, plan.lpr, plan.vw > 1);
    S.rref = nullptr;
    Carve c(ws);
    Ctl C = make_ctl(o);
    C.theta = theta;
    C.sel_seed = sel_seed;
    C.exch = c.take<XRec>(4 * (size_t)std::max(plan.grid, 1));
    double* nu2_ws = c.take<double>(S.d);
    if (c.bytes() > ws_bytes) {
        set_error("solve workspace too small: need %zu bytes, got %zu", c.bytes(), ws_bytes);
        return CSK_ERR_WORKSPACE;
    }
    if (S.nu2 == nullptr) {
        const csk_status e = launch_row_norms2(S.At64, S.ldat64, S.d, S.n, nu2_ws, st);
        if (e != CSK_OK) return e;
        S.nu2 = nu2_ws;
    }
    if (plan.grid > 1) {
        const int64_t words = (int64_t)4 * plan.grid * (int64_t)sizeof(XRec) / 4;
        k_zero_words<<<(int)std::min<int64_t>(64, (words + 255) / 256), 256, 0, st>>>(
            reinterpret_cast<uint32_t*>(C.exch), words);
        CSK_LAUNCH_CHECK("k_zero_words");
    }
    return dispatch_solve<tag_f64, 1>(S, C, plan, st);
}

size_t solve_exch_record_bytes() { return sizeof(XRec); }

csk_status launch_row_norms2(const double* A, int64_t lda, int64_t d, int64_t n, double* nu2, hipStream_t st)
{
    k_row_norms2<<<(int)std::min<int64_t>(4096, (d + 3) / 4), 256, 0, st>>>(A, lda, (int)d, (int)n, nu2);
    CSK_LAUNCH_CHECK("k_row_norms2");
    return CSK_OK;
}

csk_status solve_batched_run(const SolveSys* sys_dev, int32_t nsys, const BatchedPlan& bp, csk_dtype at_dtype,
                             const csk_solve_opts* o, hipStream_t st)
{
    Ctl C = make_ctl(o);
    C.trace = nullptr;  // one trace cannot describe many systems
    C.queue = bp.queue_dev;
    C.order = bp.order_dev;
    C.nsys = nsys;
    csk_status e = upload_i32(bp.order, nsys, bp.order_dev, st);
    if (e != CSK_OK) return e;
    k_zero_words<<<1, 64, 0, st>>>(bp.queue_dev, 1);
    CSK_LAUNCH_CHECK("k_zero_words");
    switch (at_dtype) {
    case CSK_F64: return launch_batched<tag_f64>(sys_dev, nsys, bp, C, st);
    case CSK_F32: return launch_batched<tag_f32>(sys_dev, nsys, bp, C, st);
    case CSK_F16: return launch_batched<tag_f16>(sys_dev, nsys, bp, C, st);
    case CSK_BF16: return launch_batched<tag_bf16>(sys_dev, nsys, bp, C, st);
    default: return CSK_ERR_UNSUPPORTED;
    }
}

}  // namespace csk
