// mrhs.hip -- one sketch At, many right-hand sides: the loop of Algorithm 1
// run independently for every column j of Bt, with all columns' residuals
// formed together on the matrix cores.
//
// Per iteration (one persistent cooperative launch, two grid barriers).
// Data that crosses workgroups (candidates, Delta, its scale, X for the
// refresh) moves through device-coherent accesses, so the barriers need no
// cache write-back or invalidation and the read-only operands stay in L2:
//   1. residual block R = R_ref - At_lp * Delta for the workgroup's rows and
//      128 columns, with Delta = X - X_ref rounded to BF16/FP16 and the
//      product on v_mfma_f32_16x16x32 (FP32 accumulation); every
//      refresh_every iterations R_ref = Bt - At64 * X exactly, on the FP64
//      matrix cores (v_mfma_f64_16x16x4), and Delta restarts from zero;
//   2. per column, the best row of the block by r^2 / ||At^(i)||^2 (the
//      squared weighted residual of the paper), published to global memory;
//   3. barrier; the owner workgroup of column j reduces the row blocks' bests
//      in fixed order, applies the stop test and the projection
//      X[:, j] += (r / ||At^(i)||^2) At64^(i)^T, and writes Delta[:, j];
//   4. barrier; the run ends when no column is active.
// Scores and projections use the FP64 rows, as in the single-system solver.
#include "csk_grid.h"
#include "csk_mrhs.h"
#include "csk_tune.h"

#include <algorithm>

namespace csk {
namespace {

constexpr int kNT = 512;          // 8 wavefronts
constexpr int kCols = 128;        // columns per workgroup (one 16-column tile per wavefront)
constexpr int kMaxRT = 8;         // 16-row tiles per workgroup
constexpr int kMaxOwned = 8;      // columns owned (reduced and projected) per workgroup
constexpr int kMaxGrid = 4096;    // workgroups (arrival flags of the grid barrier)
// k-steps of the B operand loaded together (fewer when many row tiles
// already hold registers)
template <int RT> constexpr int kb_batch() { return RT <= 5 ? 8 : 4; }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

struct CandRec {
    double score, alpha, r2;  // alpha = r / ||At64^(i)||^2 of the best row
    uint32_t idx, flags;
};

struct MCtl {
    const uint16_t* Alp;      // rows_pad x npad, zero padded
    const double* A64;        // d x n, lda64
    const double* Bt;         // d x R, ldbt
    const double* nu2;        // d
    double* XT;               // Rpad x npad: column j of X is row j
    double* XrT;              // Rpad x npad: X at the last refresh
    const double* XuT;        // Rpad x npad: reference solution, or null
    uint16_t* DT;             // Rpad x npad: Delta in 16-bit
    CandRec* cand;            // RB x Rpad
    const double* colref2;    // Rpad: ||Xref[:, j]||^2
    const double* colbt2;     // Rpad: ||Bt[:, j]||^2
    double* dinv;             // Rpad: 2^-e_j, Delta[:, j] is stored as Delta * 2^e_j
    csk_solve_result* res;    // R
    uint32_t* flags;          // kMaxGrid arrival flags of the grid barrier, zero at launch
    uint32_t* active;
    int32_t* cancel_seen;
    const volatile int32_t* cancel;
    double tol2;
    int64_t maxit;
    int64_t lda64, ldbt;
    int32_t d, n, npad, R, Rpad, RB, CB, refresh_every, check_every, stop_mode;
    int32_t a_lds;            // 1: the workgroup's rows of Alp are staged in LDS
    int32_t a_stride;         // LDS row stride of that tile (npad + 8: no bank conflicts)
};

template <class Tag> struct Mfma;
template <> struct Mfma<tag_bf16> {
    __device__ static f32x4 run(const uint16_t* a, const uint4& b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    }
    __device__ static uint16_t round(double v) { return f64_to_bf16_bits(v); }
};
template <> struct Mfma<tag_f16> {
    __device__ static f32x4 run(const uint16_t* a, const uint4& b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(*reinterpret_cast<const f16x8*>(a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    }
    __device__ static uint16_t round(double v) { return f64_to_f16_bits(v); }
};

// 16 bytes written by other workgroups during the kernel (two coherent
// 8-byte loads).
__device__ __forceinline__ uint4 coh_load16(const uint16_t* p)
{
    const uint64_t lo = coh_load(reinterpret_cast<const uint64_t*>(p));
    const uint64_t hi = coh_load(reinterpret_cast<const uint64_t*>(p) + 1);
    return make_uint4(static_cast<uint32_t>(lo), static_cast<uint32_t>(lo >> 32), static_cast<uint32_t>(hi),
                      static_cast<uint32_t>(hi >> 32));
}

template <class Tag, int RT>
__global__ __launch_bounds__(kNT) void k_mrhs(MCtl C)
{
    constexpr int kKB = kb_batch<RT>();
    __shared__ GridRed slots[kNT / kWave];
    __shared__ uint32_t s_ok;
    __shared__ double s_nu2[RT * 16];
    __shared__ int32_t s_done[kMaxOwned];
    __shared__ double s_scale[kMaxOwned];

    const int tid = threadIdx.x;
    const int G = gridDim.x;
    const int rb = blockIdx.x / C.CB;
    const int cb = blockIdx.x % C.CB;
    const int w = tid / kWave;
    const int lane = tid & (kWave - 1);
    const int lc = lane & 15;          // MFMA lane column / A-row
    const int lg = lane >> 4;          // MFMA lane group
    const int row0 = rb * RT * 16;
    const int mycol = cb * kCols + w * 16 + lc;
    // v_mfma_f64_16x16x4 returns row 4q + lg of its A operand in register q
    // of lane group lg, while the 16-bit products return row 4lg + q there.
    // Loading A-operand row i from row 4(i%4) + i/4 makes both agree.
    const int arow_perm = 4 * (lc & 3) + (lc >> 2);
    const int n = C.n, d = C.d, R = C.R;

    // The low-precision rows of this workgroup stay in LDS for the whole
    // solve when they fit (read-only: Alp was padded before the launch).
    extern __shared__ __align__(16) uint16_t sA[];
    if (C.a_lds) {
        const int chunks = C.npad / 8;
        for (int e = tid; e < RT * 16 * chunks; e += kNT) {
            const int r = e / chunks, c8 = (e - r * chunks) * 8;
            *reinterpret_cast<uint4*>(sA + r * C.a_stride + c8) =
                *reinterpret_cast<const uint4*>(C.Alp + (int64_t)(row0 + r) * C.npad + c8);
        }
    }
    for (int i = tid; i < RT * 16; i += kNT) s_nu2[i] = (row0 + i < d) ? C.nu2[row0 + i] : 0.0;
    if (tid < kMaxOwned) {
        s_done[tid] = 0;
        s_scale[tid] = 1.0;
    }
    __syncthreads();

    double rref[RT][4];
    uint32_t epoch = 0;
    int64_t k_ref = 0, nref = 0;
    for (int64_t k = 0;; ++k) {
        const bool refresh = (k == 0) || (k - k_ref >= C.refresh_every);
        // the current residual is rref - acc: acc = 0 right after a refresh
        f32x4 acc[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (refresh) {
            f64x4 acc64[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) acc64[rt] = f64x4{0.0, 0.0, 0.0, 0.0};
            // both operands of a batch of k-steps are loaded before its
            // products (X coherent, At64 read-only), one round trip a batch
            constexpr int kKB64 = 2;
            for (int kb = 0; kb < n; kb += 4 * kKB64) {
                double bq[kKB64];
                double aq[kKB64][RT];
#pragma unroll
                for (int t = 0; t < kKB64; ++t) {
                    const int kq = kb + 4 * t + lg;
                    bq[t] = (kq < C.npad) ? coh_load(&C.XT[(int64_t)mycol * C.npad + kq]) : 0.0;
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) {
                        const int row = row0 + rt * 16 + arow_perm;
                        aq[t][rt] = (row < d && kq < n) ? C.A64[(int64_t)row * C.lda64 + kq] : 0.0;
                    }
                }
#pragma unroll
                for (int t = 0; t < kKB64; ++t)
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        acc64[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[t][rt], bq[t], acc64[rt], 0, 0, 0);
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = row0 + rt * 16 + 4 * lg + q;
                    rref[rt][q] = (row < d && mycol < R) ? C.Bt[(int64_t)row * C.ldbt + mycol] - acc64[rt][q] : 0.0;
                }
            k_ref = k;
            ++nref;
        } else {
            // Delta's fragments are coherent loads, which the compiler keeps
            // in program order: issue kKB k-steps of them at once, then their
            // products, so a batch costs one round trip rather than kKB.
            const uint16_t* bcol = C.DT + (int64_t)mycol * C.npad + lg * 8;
            for (int kb = 0; kb < C.npad; kb += 32 * kKB) {
                uint4 bq[kKB];
#pragma unroll
                for (int t = 0; t < kKB; ++t)
                    bq[t] = (kb + 32 * t < C.npad) ? coh_load16(bcol + kb + 32 * t) : make_uint4(0, 0, 0, 0);
                if (C.a_lds) {
#pragma unroll
                    for (int t = 0; t < kKB; ++t) {
                        const int kk = kb + 32 * t;
                        if (kk < C.npad) {
#pragma unroll
                            for (int rt = 0; rt < RT; ++rt)
                                acc[rt] = Mfma<Tag>::run(sA + (rt * 16 + lc) * C.a_stride + lg * 8 + kk, bq[t],
                                                         acc[rt]);
                        }
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < kKB; ++t) {
                        const int kk = kb + 32 * t;
                        if (kk < C.npad) {
#pragma unroll
                            for (int rt = 0; rt < RT; ++rt) {
                                const uint16_t* arow =
                                    C.Alp + (int64_t)(row0 + rt * 16 + lc) * C.npad + lg * 8 + kk;
                                acc[rt] = Mfma<Tag>::run(arow, bq[t], acc[rt]);
                            }
                        }
                    }
                }
            }
        }

        // Delta of this column is stored scaled by an exact power of two
        const double dinv = (mycol < R) ? coh_load(&C.dinv[mycol]) : 1.0;
        // best row of this block for column mycol
        GridRed cv = red_identity();
        if (mycol < R) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int lr = rt * 16 + 4 * lg + q;
                    const int row = row0 + lr;
                    if (row < d) {
                        const double r = rref[rt][q] - static_cast<double>(acc[rt][q]) * dinv;
                        cv.r2 += r * r;
                        const double nn = s_nu2[lr];
                        if (nn > 0.0) {
                            const double score = (r * r) / nn;
                            if (!isfinite(score)) cv.flags |= kFlagNonfinite;
                            else if (cand_better(score, (uint32_t)row, cv.score, cv.idx)) {
                                cv.score = score;
                                cv.r = r / nn;  // the step length alpha
                                cv.idx = (uint32_t)row;
                            }
                        } else if (isnan(nn)) {
                            cv.flags |= kFlagNonfinite;
                        }
                    }
                }
        }
        // lanes lc, lc+16, lc+32, lc+48 share a column
#pragma unroll
        for (int off = 16; off < 64; off <<= 1) {
            GridRed o;
            o.score = __shfl_xor(cv.score, off, kWave);
            o.r = __shfl_xor(cv.r, off, kWave);
            o.r2 = __shfl_xor(cv.r2, off, kWave);
            o.e2 = 0.0;
            o.idx = __shfl_xor(cv.idx, off, kWave);
            o.flags = __shfl_xor(cv.flags, off, kWave);
            cv = red_combine(cv, o);
        }
        if (lg == 0 && mycol < R) {
            CandRec* c = &C.cand[(int64_t)rb * C.Rpad + mycol];
            coh_store(&c->score, cv.score);
            coh_store(&c->alpha, cv.r);
            coh_store(&c->r2, cv.r2);
            coh_store(reinterpret_cast<uint64_t*>(&c->idx), (static_cast<uint64_t>(cv.flags) << 32) | cv.idx);
        }
        if (blockIdx.x == 0 && tid == 0 && C.cancel && (k % C.check_every) == 0 && *C.cancel != 0)
            coh_store(C.cancel_seen, int32_t(1));
        ++epoch;
        bool ok = grid_barrier_flags(C.flags, blockIdx.x, G, epoch, &s_ok);

        // owner phase: column j belongs to workgroup j mod G
        const int32_t cancelled = __hip_atomic_load(C.cancel_seen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int t = 0;
        for (int j = blockIdx.x; j < R; j += G, ++t) {
            if (s_done[t]) continue;
            GridRed v = red_identity();
            for (int b = tid; b < C.RB; b += kNT) {
                const CandRec* c = &C.cand[(int64_t)b * C.Rpad + j];
                GridRed o;
                o.score = coh_load(&c->score);
                o.r = coh_load(&c->alpha);
                o.r2 = coh_load(&c->r2);
                o.e2 = 0.0;
                const uint64_t w = coh_load(reinterpret_cast<const uint64_t*>(&c->idx));
                o.idx = static_cast<uint32_t>(w);
                o.flags = static_cast<uint32_t>(w >> 32);
                v = red_combine(v, o);
            }
            double* xj = C.XT + (int64_t)j * C.npad;
            if (C.XuT)
                for (int q = tid; q < n; q += kNT) {
                    const double e = coh_load(&xj[q]) - C.XuT[(int64_t)j * C.npad + q];
                    v.e2 += e * e;
                }
            const GridRed tot = block_red<kNT>(v, slots);
            int32_t status = -1;
            double meas;
            bool conv;
            if (C.stop_mode == CSK_STOP_REL_ERR) {
                const double ref2 = C.colref2[j];
                meas = ref2 > 0.0 ? tot.e2 / ref2 : tot.e2;
                conv = ref2 > 0.0 ? (tot.e2 / ref2 <= C.tol2) : (tot.e2 <= C.tol2);
            } else {
                const double bt2 = C.colbt2[j];
                meas = bt2 > 0.0 ? tot.r2 / bt2 : tot.r2;
                conv = refresh && tot.r2 <= C.tol2 * bt2;
            }
            if (conv) status = CSK_OK;
            else if (k == C.maxit) status = CSK_NOT_CONVERGED;
            else if (!ok) status = CSK_ERR_DEVICE;
            else if (cancelled) status = CSK_CANCELLED;
            else if (tot.flags & kFlagNonfinite) status = CSK_ERR_NONFINITE;
            else if (tot.idx == kNoRow) status = CSK_ERR_DEGENERATE;
            else if (tot.idx >= (uint32_t)d) status = CSK_ERR_DEVICE;  // never dereference a bad row
            if (status >= 0) {
                if (tid == 0) {
                    C.res[j].iters = k;
                    C.res[j].status = status;
                    C.res[j].fp64_fallback = 0;
                    C.res[j].final_measure = meas;
                    C.res[j].refreshes = nref;
                    s_done[t] = 1;
                    __hip_atomic_fetch_sub(C.active, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                __syncthreads();
                continue;
            }
            const double alpha = tot.r;
            const double* arow = C.A64 + (int64_t)tot.idx * C.lda64;
            // At a refresh Delta restarts at alpha * a; scale it by 2^e with
            // ||alpha a|| * 2^e in [16, 32) so the 16-bit operand keeps its
            // precision (FP16's exponent range is narrow) as x converges.
            if (refresh) {
                const double v = sqrt(tot.score);  // |alpha| ||At64^(i)|| = |r| / ||At64^(i)||
                int e = 0;
                if (v > 0.0 && isfinite(v)) e = 4 - ilogb(v);
                e = e < -960 ? -960 : (e > 960 ? 960 : e);
                if (tid == 0) coh_store(&C.dinv[j], ldexp(1.0, -e));
                s_scale[t] = ldexp(1.0, e);
            }
            __syncthreads();
            const double dscale = s_scale[t];
            double* xr = C.XrT + (int64_t)j * C.npad;
            uint16_t* dj = C.DT + (int64_t)j * C.npad;
            // four columns per thread: Delta leaves in one coherent 8-byte
            // store (columns n .. npad stay zero)
            for (int q0 = tid * 4; q0 < C.npad; q0 += kNT * 4) {
                uint64_t packed = 0;
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4) {
                    const int q = q0 + e4;
                    if (q < n) {
                        const double x = coh_load(&xj[q]);
                        double base;
                        if (refresh) {
                            xr[q] = x;
                            base = x;
                        } else {
                            base = xr[q];
                        }
                        const double xn = x + alpha * arow[q];
                        coh_store(&xj[q], xn);
                        packed |= static_cast<uint64_t>(Mfma<Tag>::round((xn - base) * dscale)) << (16 * e4);
                    }
                }
                coh_store(reinterpret_cast<uint64_t*>(dj + q0), packed);
            }
        }
        ++epoch;
        ok = grid_barrier_flags(C.flags, blockIdx.x, G, epoch, &s_ok) && ok;
        const uint32_t left = __hip_atomic_load(C.active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (left == 0u || !ok) break;
    }
}

// ---- the form with Delta held in registers (npad <= 32 * KS) --------------
//
// Per iteration there is no grid barrier; two tagged hand-offs replace them
// (words as in exchange(): 32 bits of payload, the iteration tag k + 1 in
// the upper half, two slots alternating by parity):
//   1. every workgroup (row block rb, column block cb) forms its residual
//      block and publishes, per live column, its best row (a record of
//      eight tagged words, stored word-major: word f of the records of
//      column j from row blocks 0..RB-1 is one contiguous run);
//   2. the owner of column j (workgroup (j mod RB, cb) of its column block)
//      polls one word of each of the RB records of j (a wave's polls cover
//      consecutive row blocks, so a few cache lines) and reads a record
//      once that word is fresh, reduces them in fixed order, applies the
//      stop test and publishes (i_j, alpha_j) (four tagged words; a final
//      status carries the tag kFinal in both slots), then projects its own
//      FP64 copy of X[:, j] with the FP64 row;
//   3. every workgroup polls one word of the results of its 128 columns,
//      reads the four once it is fresh, and adds
//      alpha_j At_lp^(i_j) to its copy of Delta[:, j] = X - X_ref, which each
//      lane keeps in registers, in the 16-bit type, for the k positions it
//      feeds to the matrix cores (each update summed in FP32 and rounded
//      back).  The rows of At_lp are read-only, so they come through L2 (one
//      fetch per XCD) instead of a device-coherent copy of Delta per
//      workgroup.
// Delta therefore accumulates the low-precision rows, rounded at each step,
// where the owner's X accumulates the FP64 ones; every refresh restarts both
// from the exact FP64 residual of the published X.  Owners publish X (and a flag per
// column) at the end of the iteration before each refresh.
// Polling one word instead of the whole record, and the word-major candidate
// layout, cut the device-coherent requests that every poll round puts on the
// fabric (with about 250 workgroups polling at once) by 8x and then by the
// record count per cache line; at 256 right-hand sides over d = 10000 an
// iteration went from 25.5 to 20.7 us.
constexpr uint32_t kFinalTag = 0xFFFFFFFFu;
constexpr int kRdMaxNpad = 512;  // Delta in registers: 32 * KS k positions, KS <= 16

__host__ __device__ constexpr size_t up16(size_t v) { return (v + 15) / 16 * 16; }

struct RdCtl {
    const uint16_t* Alp;       // rows_pad x npad, zero padded
    const double* A64;         // d x n, lda64
    const double* Bt;          // d x R, ldbt
    const double* nu2;         // d
    double* XT;                // Rpad x npad: X published at refreshes (X0 at launch)
    const double* XuT;         // Rpad x npad: reference solution, or null
    uint64_t* cand;            // [2][8][Rpad][RB] tagged words (word-major), zero at launch
    uint64_t* resw;            // [2][Rpad][4] tagged words, zero at launch
    uint32_t* xflag;           // Rpad: last refresh iteration whose X is published, zero at launch
    const double* colref2;     // Rpad: ||Xref[:, j]||^2
    const double* colbt2;      // Rpad: ||Bt[:, j]||^2
    csk_solve_result* res;     // R
    const volatile int32_t* cancel;
    double tol2;
    int64_t maxit;
    int64_t lda64, ldbt;
    int32_t d, n, npad, R, Rpad, RB, CB, refresh_every, check_every, stop_mode;
    int32_t a_stride;          // LDS row stride of the workgroup's rows of Alp
    int32_t nown;              // columns owned per workgroup (at most kNT / 64)
};

__device__ __forceinline__ uint64_t tagw(uint32_t payload, uint64_t tag) { return (tag << 32) | payload; }

// One 16-byte vector of eight 16-bit values of Delta (scaled by s for FP16)
// plus alpha times the matching eight values of a row, rounded back (RNE).
template <class Tag> struct Acc16;
template <> struct Acc16<tag_bf16> {
    __device__ static uint4 axpy(const uint4& dv, float alpha, const uint4& av, float s)
    {
        (void)s;
        const bf16x8 d = __builtin_bit_cast(bf16x8, dv);
        const bf16x8 a = __builtin_bit_cast(bf16x8, av);
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = static_cast<__bf16>(static_cast<float>(d[e]) + alpha * static_cast<float>(a[e]));
        return __builtin_bit_cast(uint4, o);
    }
};
template <> struct Acc16<tag_f16> {
    __device__ static uint4 axpy(const uint4& dv, float alpha, const uint4& av, float s)
    {
        const f16x8 d = __builtin_bit_cast(f16x8, dv);
        const f16x8 a = __builtin_bit_cast(f16x8, av);
        const float as = alpha * s;
        f16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = static_cast<_Float16>(static_cast<float>(d[e]) + as * static_cast<float>(a[e]));
        return __builtin_bit_cast(uint4, o);
    }
};

// The exact FP64 residual R_ref = Bt - At64 X of a lane's rows (one column)
// on the FP64 matrix cores, every refresh.
template <int RT, int NP>
__device__ __forceinline__ void refresh_product(const RdCtl& C, int row0, int mycol, int lg, int arow_perm, bool live,
                                             double (&rr)[RT][4])
{
    const int n = C.n, d = C.d;
    f64x4 acc64[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) acc64[rt] = f64x4{0.0, 0.0, 0.0, 0.0};
    // X (device-coherent) kXB k-steps per round trip; At64 (read-only,
    // cached) fragments two k-steps ahead of their products.
    constexpr int kXB = 8;
    const int nks = (n + 3) / 4;  // k-steps of four columns
    auto load_a = [&](int ks, double (&dst)[RT]) {
        const int kq = 4 * ks + lg;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int row = row0 + rt * 16 + arow_perm;
            dst[rt] = (row < d && kq < n) ? C.A64[(int64_t)row * C.lda64 + kq] : 0.0;
        }
    };
    double a0[RT], a1[RT];
    load_a(0, a0);
    load_a(1, a1);
    for (int kb = 0; kb < nks; kb += kXB) {
        double bq[kXB];
#pragma unroll
        for (int t = 0; t < kXB; ++t) {
            const int kq = 4 * (kb + t) + lg;
            bq[t] = (kq < NP) ? coh_load(&C.XT[(int64_t)mycol * NP + kq]) : 0.0;
        }
#pragma unroll
        for (int t = 0; t < kXB; ++t) {
            double acur[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                acur[rt] = a0[rt];
                a0[rt] = a1[rt];
            }
            load_a(kb + t + 2, a1);  // past the last k-step: zeros
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
                acc64[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(acur[rt], bq[t], acc64[rt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = row0 + rt * 16 + 4 * lg + q;
            rr[rt][q] = (row < d && live) ? C.Bt[(int64_t)row * C.ldbt + mycol] - acc64[rt][q] : 0.0;
        }
}

template <class Tag, int RT, int KS>
__global__ __launch_bounds__(kNT) void k_mrhs_rd(RdCtl C)
{
    constexpr int NP = 32 * KS;  // padded row length (C.npad == NP)
    __shared__ double s_nu2[RT * 16];
    __shared__ double s_inu2[RT * 16];  // 1 / nu2 (0 for empty rows)
    __shared__ double s_e2[kNT / kWave];
    __shared__ int32_t s_odone[kNT / kWave];
    extern __shared__ __align__(16) char smem[];
    uint16_t* sA = reinterpret_cast<uint16_t*>(smem);
    double* sX = reinterpret_cast<double*>(smem + up16((size_t)RT * 16 * (NP + 8) * 2));
    double* sXu = sX + (size_t)C.nown * NP;   // the owned columns' reference solution (REL_ERR)
    // owners' records, two sets alternating by iteration parity
    GridRed* red0 = reinterpret_cast<GridRed*>(reinterpret_cast<char*>(sXu) + (size_t)C.nown * NP * 8);

    const int tid = threadIdx.x;
    const int rb = blockIdx.x / C.CB;
    const int cb = blockIdx.x % C.CB;
    const int w = tid / kWave;
    const int lane = tid & (kWave - 1);
    const int lc = lane & 15;
    const int lg = lane >> 4;
    const int row0 = rb * RT * 16;
    const int mycol = cb * kCols + w * 16 + lc;
    const bool live = mycol < C.R;
    const int arow_perm = 4 * (lc & 3) + (lc >> 2);  // see k_mrhs
    const int n = C.n, d = C.d, RB = C.RB;
    const bool rel_err = C.stop_mode == CSK_STOP_REL_ERR;
    // owned column c of this workgroup: local index rb + c * RB of the block
    const int ocol = cb * kCols + rb + w * RB;  // the column wave w owns (w < nown)
    const bool owner_wave = w < C.nown && rb + w * RB < kCols && ocol < C.R;
    const double oref2 = owner_wave ? C.colref2[ocol] : 0.0;  // ||Xref[:, j]||^2
    const double obt2 = owner_wave ? C.colbt2[ocol] : 0.0;    // ||Bt[:, j]||^2

    // this workgroup's rows of Alp stay in LDS (read-only, padded before the launch)
    {
        const int chunks = NP / 8;
        for (int e = tid; e < RT * 16 * chunks; e += kNT) {
            const int r = e / chunks, c8 = (e - r * chunks) * 8;
            *reinterpret_cast<uint4*>(sA + r * (NP + 8) + c8) =
                *reinterpret_cast<const uint4*>(C.Alp + (int64_t)(row0 + r) * NP + c8);
        }
    }
    for (int i = tid; i < RT * 16; i += kNT) {
        const double nn = (row0 + i < d) ? C.nu2[row0 + i] : 0.0;
        s_nu2[i] = nn;
        s_inu2[i] = nn > 0.0 ? 1.0 / nn : 0.0;
    }
    // the owned columns' X (FP64, from X0) and their ||X - Xref||^2
    if (owner_wave) {
        double e2 = 0.0;
        for (int q = lane; q < NP; q += kWave) {
            const double x = C.XT[(int64_t)ocol * NP + q];
            const double u = C.XuT ? C.XuT[(int64_t)ocol * NP + q] : 0.0;
            sX[w * NP + q] = x;
            sXu[w * NP + q] = u;
            if (C.XuT && q < n) {
                const double e = x - u;
                e2 += e * e;
            }
        }
        e2 = wave_sum(e2);
        if (lane == 0) {
            s_e2[w] = e2;
            s_odone[w] = 0;
        }
    } else if (lane == 0) {
        s_odone[w] = 1;
    }
    __syncthreads();

    uint4 dm[KS];  // this lane's k positions of Delta[:, mycol] (16-bit, FP16 scaled)
#pragma unroll
    for (int t = 0; t < KS; ++t) dm[t] = make_uint4(0u, 0u, 0u, 0u);
    float dsc = 1.f;    // FP16 operand scale 2^e of this column's window
    double dinv = 1.0;  // and 2^-e
    bool done = !live;
    bool fail = false;
    // R_ref of this lane's rows, kept in FP32 for the inner iterations (their
    // 16-bit products carry far larger errors); a refresh iteration scores
    // the exact FP64 residual itself
    float rref[RT][4];
    int64_t k_ref = 0, nref = 0;
    constexpr int kQ = NP / kWave;  // columns of a row per lane
    for (int64_t k = 0;; ++k) {
        const bool refresh = (k == 0) || (k - k_ref >= C.refresh_every);
        const uint64_t tag = static_cast<uint32_t>(k + 1);
        const int slot = (int)(k & 1);
        double rr[RT][4];  // this iteration's residual of the lane's rows
        if (refresh) {
            // Delta restarts at zero (X_ref = X): its registers are free for
            // the FP64 product
#pragma unroll
            for (int t = 0; t < KS; ++t) dm[t] = make_uint4(0u, 0u, 0u, 0u);
            // X of this refresh is published by the owners (X0 at k = 0)
            if (!done && k > 0) {
                uint32_t spins = 0;
                while (static_cast<int32_t>(coh_load(&C.xflag[mycol]) - static_cast<uint32_t>(k)) < 0) {
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > kSpinLimit) { fail = true; done = true; break; }
                }
            }
            refresh_product<RT, NP>(C, row0, mycol, lg, arow_perm, live, rr);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int q = 0; q < 4; ++q) rref[rt][q] = static_cast<float>(rr[rt][q]);
            k_ref = k;
            ++nref;
        } else {
            f32x4 acc[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) acc[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
            // R = R_ref - At_lp Delta: A from LDS, B from this lane's Delta
#pragma unroll
            for (int t = 0; t < KS; ++t) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
                    acc[rt] = Mfma<Tag>::run(sA + (rt * 16 + lc) * (NP + 8) + lg * 8 + 32 * t, dm[t], acc[rt]);
            }
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    rr[rt][q] = static_cast<double>(rref[rt][q]) - static_cast<double>(acc[rt][q]) * dinv;
        }

        // 1. best row of this block for column mycol, published as a tagged record
        // (score r^2 / ||At^(i)||^2 by the stored reciprocal; the step length
        // r / ||At^(i)||^2 by one division, for the lane's best row only).
        // Branch-free: this lane's rows come in ascending order, so a row
        // replaces the best one only with a strictly larger score (ties keep
        // the lower index), or when there is none yet.
        GridRed cv = red_identity();
        {
            double rbest = 0.0, nbest = 1.0;
            uint32_t flags = 0u;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int lr = rt * 16 + 4 * lg + q;
                    const uint32_t row = static_cast<uint32_t>(row0 + lr);
                    const bool in = !done && row < static_cast<uint32_t>(d);
                    const double r = in ? rr[rt][q] : 0.0;
                    cv.r2 += r * r;
                    const double nn = s_nu2[lr];
                    const double score = (r * r) * s_inu2[lr];
                    const bool usable = in && nn > 0.0;
                    const bool finite = isfinite(score);
                    flags |= ((usable && !finite) || (in && isnan(nn))) ? kFlagNonfinite : 0u;
                    const bool better = usable && finite && (score > cv.score || cv.idx == kNoRow);
                    cv.score = better ? score : cv.score;
                    cv.idx = better ? row : cv.idx;
                    rbest = better ? r : rbest;
                    nbest = better ? nn : nbest;
                }
            cv.flags = flags;
            cv.r = cv.idx != kNoRow ? rbest / nbest : 0.0;
        }
#pragma unroll
        for (int off = 16; off < 64; off <<= 1) {
            GridRed o;
            o.score = __shfl_xor(cv.score, off, kWave);
            o.r = __shfl_xor(cv.r, off, kWave);
            o.r2 = __shfl_xor(cv.r2, off, kWave);
            o.e2 = 0.0;
            o.idx = __shfl_xor(cv.idx, off, kWave);
            o.flags = __shfl_xor(cv.flags, off, kWave);
            cv = red_combine(cv, o);
        }
        if (!done && lg == 0) {
            const size_t fs = (size_t)C.Rpad * RB;  // stride between the words of a record
            uint64_t* rec = C.cand + ((size_t)slot * 8 * C.Rpad + mycol) * RB + rb;
            const uint64_t sb = static_cast<uint64_t>(__double_as_longlong(cv.score));
            const uint64_t ab = static_cast<uint64_t>(__double_as_longlong(cv.r));
            const uint64_t rb2 = static_cast<uint64_t>(__double_as_longlong(cv.r2));
            coh_store(&rec[0 * fs], tagw(static_cast<uint32_t>(sb), tag));
            coh_store(&rec[1 * fs], tagw(static_cast<uint32_t>(sb >> 32), tag));
            coh_store(&rec[2 * fs], tagw(static_cast<uint32_t>(ab), tag));
            coh_store(&rec[3 * fs], tagw(static_cast<uint32_t>(ab >> 32), tag));
            coh_store(&rec[4 * fs], tagw(static_cast<uint32_t>(rb2), tag));
            coh_store(&rec[5 * fs], tagw(static_cast<uint32_t>(rb2 >> 32), tag));
            coh_store(&rec[6 * fs], tagw(cv.idx, tag));
            coh_store(&rec[7 * fs], tagw(cv.flags, tag));
        }

        // 2. owners: poll the row blocks' records of their columns (thread t:
        // owned column t / RB, row block t % RB), reduce each column in one
        // wave in fixed order, test, publish (i, alpha), project X.
        GridRed* red = red0 + (size_t)slot * C.nown * RB;
        {
            GridRed o = red_identity();
            const int c = tid / RB, b = tid - (tid / RB) * RB;
            const int jl = rb + c * RB;
            if (c < C.nown && jl < kCols && cb * kCols + jl < C.R &&
                !__hip_atomic_load(&s_odone[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
                const int j = cb * kCols + jl;
                const size_t fs = (size_t)C.Rpad * RB;
                const uint64_t* rec = C.cand + ((size_t)slot * 8 * C.Rpad + j) * RB + b;
                uint64_t v[8] = {};
                uint32_t spins = 0;
                for (;;) {
                    // one word per poll, the whole record once that word is fresh
                    bool fresh = (coh_load(&rec[7 * fs]) >> 32) == tag;
                    if (fresh) {
#pragma unroll
                        for (int f = 0; f < 8; ++f) v[f] = coh_load(&rec[f * fs]);
#pragma unroll
                        for (int f = 0; f < 8; ++f) fresh = fresh && ((v[f] >> 32) == tag);
                    }
                    if (fresh) break;
                    // the owner wave may finish the column (the previous
                    // iteration's test) while this thread already polls
                    if (__hip_atomic_load(&s_odone[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) { spins = 0; break; }
                    __builtin_amdgcn_s_sleep(2);
                    if (++spins > kSpinLimit) break;
                }
                if (spins > kSpinLimit) {
                    o.flags = kFlagTimeout;
                } else {
                    o.score = join_f64(v[0], v[1]);
                    o.r = join_f64(v[2], v[3]);
                    o.r2 = join_f64(v[4], v[5]);
                    o.idx = static_cast<uint32_t>(v[6]);
                    o.flags = static_cast<uint32_t>(v[7]);
                }
            }
            if (tid < C.nown * RB) red[tid] = o;
        }
        // The owners' barrier, which also takes the exit vote: every column
        // of the block final here (as of the previous iteration's results)
        // and this workgroup's own columns reported.  There is no barrier at
        // the end of an iteration: waves run on into the next product while
        // the owner waves project.
        {
            const bool owner_pending =
                owner_wave && !__hip_atomic_load(&s_odone[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (__syncthreads_and(((done || fail) && !owner_pending) ? 1 : 0)) break;
        }
        if (owner_wave && !__hip_atomic_load(&s_odone[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
            GridRed t = red_identity();
            for (int b = lane; b < RB; b += kWave) t = red_combine(t, red[w * RB + b]);
            const GridRed tot = wave_red_dpp(t);
            int32_t status = -1;
            double meas;
            bool conv;
            if (rel_err) {
                const double ref2 = oref2;
                const double e2 = s_e2[w];
                meas = ref2 > 0.0 ? e2 / ref2 : e2;
                conv = ref2 > 0.0 ? (e2 / ref2 <= C.tol2) : (e2 <= C.tol2);
            } else {
                const double bt2 = obt2;
                meas = bt2 > 0.0 ? tot.r2 / bt2 : tot.r2;
                conv = refresh && tot.r2 <= C.tol2 * bt2;
            }
            const bool cancelled = C.cancel && (k % C.check_every) == 0 && *C.cancel != 0;
            if (conv) status = CSK_OK;
            else if (k == C.maxit) status = CSK_NOT_CONVERGED;
            else if (tot.flags & kFlagTimeout) status = CSK_ERR_DEVICE;
            else if (cancelled) status = CSK_CANCELLED;
            else if (tot.flags & kFlagNonfinite) status = CSK_ERR_NONFINITE;
            else if (tot.idx == kNoRow) status = CSK_ERR_DEGENERATE;
            else if (tot.idx >= (uint32_t)d) status = CSK_ERR_DEVICE;  // never dereference a bad row
            uint64_t* rw = C.resw;
            if (status >= 0) {
                // the column's solution leaves through XT (copied out after the launch)
                for (int q = lane; q < n; q += kWave) coh_store(&C.XT[(int64_t)ocol * NP + q], sX[w * NP + q]);
                if (lane == 0) {
                    C.res[ocol].iters = k;
                    C.res[ocol].status = status;
                    C.res[ocol].fp64_fallback = 0;
                    C.res[ocol].final_measure = meas;
                    C.res[ocol].refreshes = nref;
                    __hip_atomic_store(&s_odone[w], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                if (lane < 8) {
                    // the final word set, in both slots
                    const int sl = lane >> 2, f = lane & 3;
                    coh_store(&rw[((size_t)sl * C.Rpad + ocol) * 4 + f],
                              tagw(f == 3 ? static_cast<uint32_t>(status) : 0u, kFinalTag));
                }
            } else {
                const double alpha = tot.r;
                int e = 0;
                if (refresh) {
                    // FP16 operand scale of the new window: ||alpha a|| * 2^e in [16, 32)
                    const double v = sqrt(tot.score);
                    if (v > 0.0 && isfinite(v)) e = 4 - ilogb(v);
                    e = e < -100 ? -100 : (e > 100 ? 100 : e);
                }
                const uint64_t ab = static_cast<uint64_t>(__double_as_longlong(alpha));
                if (lane < 4) {
                    const uint32_t p = lane == 0 ? tot.idx
                                       : lane == 1 ? static_cast<uint32_t>(ab)
                                       : lane == 2 ? static_cast<uint32_t>(ab >> 32)
                                                   : static_cast<uint32_t>(e);
                    coh_store(&rw[((size_t)slot * C.Rpad + ocol) * 4 + lane], tagw(p, tag));
                }
                // the owner's projection X[:, j] += alpha At64^(i)^T (the lane's
                // columns of the row in one round trip) and the next stop
                // measure; before a refresh X is also published
                const double* arow = C.A64 + (int64_t)tot.idx * C.lda64;
                const bool pub = (k + 1 - k_ref) >= C.refresh_every;  // the next iteration refreshes
                double av[kQ];
#pragma unroll
                for (int u = 0; u < kQ; ++u) {
                    const int q = lane + u * kWave;
                    av[u] = q < n ? arow[q] : 0.0;
                }
                if (pub) {
                    double e2 = 0.0;
#pragma unroll
                    for (int u = 0; u < kQ; ++u) {
                        const int q = lane + u * kWave;
                        if (q < n) {
                            const double x = sX[w * NP + q] + alpha * av[u];
                            sX[w * NP + q] = x;
                            const double ee = x - sXu[w * NP + q];
                            e2 += ee * ee;
                            coh_store(&C.XT[(int64_t)ocol * NP + q], x);
                        }
                    }
                    e2 = wave_sum(e2);
                    if (lane == 0) s_e2[w] = C.XuT ? e2 : 0.0;
                    // the X words are acknowledged before the flag announces them
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    __builtin_amdgcn_s_waitcnt(0);
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    if (lane == 0) coh_store(&C.xflag[ocol], static_cast<uint32_t>(k + 1));
                } else {
                    double e2 = 0.0;
#pragma unroll
                    for (int u = 0; u < kQ; ++u) {
                        const int q = lane + u * kWave;
                        if (q < n) {
                            const double x = sX[w * NP + q] + alpha * av[u];
                            sX[w * NP + q] = x;
                            const double ee = x - sXu[w * NP + q];
                            e2 += ee * ee;
                        }
                    }
                    e2 = wave_sum(e2);
                    if (lane == 0) s_e2[w] = C.XuT ? e2 : 0.0;
                }
            }
        }

        // 3. every lane: this iteration's (i, alpha) of its column; Delta += alpha At_lp^(i)
        if (!done) {
            const uint64_t* rw = C.resw + ((size_t)slot * C.Rpad + mycol) * 4;
            uint64_t v[4];
            uint32_t spins = 0;
            bool fin = false;
            for (;;) {
                // one word per poll, all four once it carries this
                // iteration's tag or the final one
                const uint64_t t3 = coh_load(&rw[3]) >> 32;
                if (t3 == tag || t3 == kFinalTag) {
#pragma unroll
                    for (int f = 0; f < 4; ++f) v[f] = coh_load(&rw[f]);
                    bool fresh = true, final_all = true;
#pragma unroll
                    for (int f = 0; f < 4; ++f) {
                        fresh = fresh && ((v[f] >> 32) == tag);
                        final_all = final_all && ((v[f] >> 32) == kFinalTag);
                    }
                    if (final_all) { fin = true; break; }
                    if (fresh) break;
                }
                __builtin_amdgcn_s_sleep(2);
                if (++spins > kSpinLimit) { fail = true; break; }
            }
            if (fin || fail) {
                done = true;
            } else {
                const uint32_t i = static_cast<uint32_t>(v[0]);
                const float alpha = static_cast<float>(join_f64(v[1], v[2]));
                if (refresh) {
                    if (std::is_same<Tag, tag_f16>::value) {
                        const int e = static_cast<int32_t>(static_cast<uint32_t>(v[3]));
                        dsc = ldexpf(1.f, e);
                        dinv = ldexp(1.0, -e);
                    }
                }
                if (i < (uint32_t)d) {
                    const uint16_t* arow = C.Alp + (int64_t)i * NP + lg * 8;
#pragma unroll
                    for (int t = 0; t < KS; ++t) {
                        dm[t] = Acc16<Tag>::axpy(dm[t], alpha, *reinterpret_cast<const uint4*>(arow + 32 * t), dsc);
                    }
                }
            }
        }
    }
}

// ---- set-up and tear-down kernels ------------------------------------------

__global__ void k_pad_lp(const uint16_t* __restrict__ src, int64_t lds, int d, int n, uint16_t* __restrict__ dst,
                         int rows_pad, int npad)
{
    const int64_t total = (int64_t)rows_pad * npad;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / npad;
        const int c = (int)(e - r * npad);
        dst[e] = (r < d && c < n) ? src[r * lds + c] : uint16_t(0);
    }
}

__global__ void k_init_cols(const double* __restrict__ X0, int64_t ldx, const double* __restrict__ Xref,
                            int64_t ldxref, int n, int R, int Rpad, int npad, double* XT, double* XrT, double* XuT,
                            uint16_t* DT)
{
    const int64_t total = (int64_t)Rpad * npad;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / npad);
        const int q = (int)(e - (int64_t)j * npad);
        const bool in = j < R && q < n;
        const double x = (in && X0) ? X0[(int64_t)q * ldx + j] : 0.0;
        XT[e] = x;
        XrT[e] = x;
        DT[e] = 0;
        if (XuT) XuT[e] = (in && Xref) ? Xref[(int64_t)q * ldxref + j] : 0.0;
    }
}

// One workgroup per column: ||Xref[:, j]||^2 and ||Bt[:, j]||^2.
__global__ __launch_bounds__(256) void k_col_norms(const double* __restrict__ XuT, int npad, int n,
                                                   const double* __restrict__ Bt, int64_t ldbt, int d,
                                                   double* colref2, double* colbt2)
{
    __shared__ double red[2][4];
    const int j = blockIdx.x;
    double a = 0.0, b = 0.0;
    if (XuT)
        for (int q = threadIdx.x; q < n; q += 256) a += XuT[(int64_t)j * npad + q] * XuT[(int64_t)j * npad + q];
    for (int i = threadIdx.x; i < d; i += 256) b += Bt[(int64_t)i * ldbt + j] * Bt[(int64_t)i * ldbt + j];
    a = wave_sum(a);
    b = wave_sum(b);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x / 64] = a;
        red[1][threadIdx.x / 64] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        colref2[j] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        colbt2[j] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

__global__ void k_init_counters(uint32_t* flags, uint32_t* active, int32_t* cancel_seen, int R,
                                CandRec* cand, int64_t ncand, double* dinv, int Rpad)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < Rpad; e += (int64_t)gridDim.x * blockDim.x)
        dinv[e] = 1.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < kMaxGrid; e += (int64_t)gridDim.x * blockDim.x)
        flags[e] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *active = (uint32_t)R;
        *cancel_seen = 0;
    }
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ncand; e += (int64_t)gridDim.x * blockDim.x) {
        CandRec c;
        c.score = 0.0;
        c.alpha = 0.0;
        c.r2 = 0.0;
        c.idx = kNoRow;
        c.flags = 0u;
        cand[e] = c;
    }
}

__global__ void k_store_x(const double* __restrict__ XT, int npad, int n, int R, double* X, int64_t ldx)
{
    const int64_t total = (int64_t)n * R;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int q = (int)(e / R);
        const int j = (int)(e - (int64_t)q * R);
        X[(int64_t)q * ldx + j] = XT[(int64_t)j * npad + q];
    }
}

struct Geom {
    int CB, RB, RT, rows_pad, npad, Rpad;
};

// Geometry of a multi-RHS launch: 128 columns per workgroup and RT 16-row
// tiles (rt = 0: the fewest that keep one workgroup per CU, the default).
Geom geom(int64_t d, int64_t n, int64_t R, int rt = 0)
{
    Geom g;
    const int cus = std::max(1, device_cu_count());
    g.CB = (int)((R + kCols - 1) / kCols);
    const int rb_max = std::max(1, cus / g.CB);
    const int64_t rows_per = (d + rb_max - 1) / rb_max;
    g.RT = rt > 0 ? rt : (int)((rows_per + 15) / 16);
    g.RB = (int)((d + 16 * g.RT - 1) / (16 * g.RT));
    g.rows_pad = g.RB * 16 * g.RT;
    // rows up to 512 columns are padded to 32 * KS, KS in {2, 4, 8, 16} (the
    // register-Delta form's compile-time width); longer rows to 32
    const int64_t ks = (n + 31) / 32;
    g.npad = ks <= 2 ? 64 : ks <= 4 ? 128 : ks <= 8 ? 256 : ks <= 16 ? 512 : (int)(ks * 32);
    g.Rpad = g.CB * kCols;
    return g;
}

int grid_for(int64_t items, int cap)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((items + 255) / 256, cap));
}

template <class Tag, int RT>
csk_status launch_mrhs(const MCtl& C_in, int G, hipStream_t st)
{
    auto kern = k_mrhs<Tag, RT>;
    MCtl arg = C_in;
    // stage the workgroup's rows of Alp in LDS when they fit beside the
    // kernel's static LDS (about 2 KB)
    arg.a_stride = arg.npad + 8;
    size_t shm = (size_t)RT * 16 * arg.a_stride * sizeof(uint16_t);
    arg.a_lds = shm + 4096 <= (size_t)device_max_lds() ? 1 : 0;
    if (!arg.a_lds) shm = 0;
    CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm));
    int per_cu = 0;
    CSK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), kNT, shm));
    if (G > per_cu * device_cu_count()) {
        set_error("multi-RHS grid of %d workgroups exceeds the %d co-resident ones", G, per_cu * device_cu_count());
        return CSK_ERR_UNSUPPORTED;
    }
    void* args[] = {&arg};
    CSK_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(G), dim3(kNT), args,
                                       (unsigned)shm, st));
    return CSK_OK;
}

template <class Tag>
csk_status dispatch(const MCtl& C, int RT, int G, hipStream_t st)
{
    switch (RT) {
    case 1: return launch_mrhs<Tag, 1>(C, G, st);
    case 2: return launch_mrhs<Tag, 2>(C, G, st);
    case 3: return launch_mrhs<Tag, 3>(C, G, st);
    case 4: return launch_mrhs<Tag, 4>(C, G, st);
    case 5: return launch_mrhs<Tag, 5>(C, G, st);
    case 6: return launch_mrhs<Tag, 6>(C, G, st);
    case 7: return launch_mrhs<Tag, 7>(C, G, st);
    case 8: return launch_mrhs<Tag, 8>(C, G, st);
    default: set_error("multi-RHS: %d row tiles per workgroup unsupported", RT); return CSK_ERR_UNSUPPORTED;
    }
}

__global__ void k_zero_u64(uint64_t* p, int64_t words)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < words; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0ull;
}

// LDS of the register-Delta form: the rows of Alp, the owned columns' X and
// the owners' records.
size_t rd_lds_bytes(const Geom& g, int nown)
{
    return up16((size_t)g.RT * 16 * (g.npad + 8) * 2) + 2 * (size_t)nown * g.npad * 8 +
           2 * (size_t)nown * g.RB * sizeof(GridRed);
}

int rd_nown(const Geom& g, int64_t nrhs)
{
    const int64_t cols = std::min<int64_t>(kCols, nrhs);
    return (int)((cols + g.RB - 1) / g.RB);
}

// Whether the register-Delta form runs this shape (else the two-barrier form).
bool rd_fits(const Geom& g, int64_t nrhs)
{
    const int nown = rd_nown(g, nrhs);
    // static LDS of k_mrhs_rd: s_nu2 and s_inu2 (RT <= kMaxRT), s_e2, s_odone, and slack
    constexpr size_t kStatic = 2 * kMaxRT * 16 * 8 + (kNT / kWave) * (8 + 4) + 256;
    return g.npad <= kRdMaxNpad && nown <= kNT / kWave && nown * g.RB <= kNT &&
           rd_lds_bytes(g, nown) + kStatic <= (size_t)device_max_lds();
}

template <class Tag, int RT, int KS>
csk_status launch_rd(const RdCtl& C_in, int G, hipStream_t st, size_t shm)
{
    auto kern = k_mrhs_rd<Tag, RT, KS>;
    RdCtl arg = C_in;
    CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm));
    int per_cu = 0;
    CSK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), kNT, shm));
    if (G > per_cu * device_cu_count()) {
        set_error("multi-RHS grid of %d workgroups exceeds the %d co-resident ones", G, per_cu * device_cu_count());
        return CSK_ERR_UNSUPPORTED;
    }
    void* args[] = {&arg};
    CSK_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(G), dim3(kNT), args,
                                       (unsigned)shm, st));
    return CSK_OK;
}

template <class Tag, int KS>
csk_status dispatch_rd_rt(const RdCtl& C, int RT, int G, hipStream_t st, size_t shm)
{
    switch (RT) {
    case 1: return launch_rd<Tag, 1, KS>(C, G, st, shm);
    case 2: return launch_rd<Tag, 2, KS>(C, G, st, shm);
    case 3: return launch_rd<Tag, 3, KS>(C, G, st, shm);
    case 4: return launch_rd<Tag, 4, KS>(C, G, st, shm);
    case 5: return launch_rd<Tag, 5, KS>(C, G, st, shm);
    case 6: return launch_rd<Tag, 6, KS>(C, G, st, shm);
    case 7: return launch_rd<Tag, 7, KS>(C, G, st, shm);
    case 8: return launch_rd<Tag, 8, KS>(C, G, st, shm);
    default: set_error("multi-RHS: %d row tiles per workgroup unsupported", RT); return CSK_ERR_UNSUPPORTED;
    }
}

template <class Tag>
csk_status dispatch_rd(const RdCtl& C, int RT, int G, hipStream_t st, size_t shm)
{
    switch (C.npad) {
    case 64: return dispatch_rd_rt<Tag, 2>(C, RT, G, st, shm);
    case 128: return dispatch_rd_rt<Tag, 4>(C, RT, G, st, shm);
    case 256: return dispatch_rd_rt<Tag, 8>(C, RT, G, st, shm);
    case 512: return dispatch_rd_rt<Tag, 16>(C, RT, G, st, shm);
    default: set_error("multi-RHS: padded row length %d unsupported", C.npad); return CSK_ERR_UNSUPPORTED;
    }
}

}  // namespace

namespace {
size_t ws_bytes_of(const Geom& g)
{
    Carve c(nullptr);
    c.take<uint16_t>((size_t)g.rows_pad * g.npad);
    c.take<double>((size_t)g.Rpad * g.npad);
    c.take<double>((size_t)g.Rpad * g.npad);
    c.take<double>((size_t)g.Rpad * g.npad);
    c.take<uint16_t>((size_t)g.Rpad * g.npad);
    c.take<CandRec>((size_t)g.RB * g.Rpad);
    c.take<double>(g.Rpad);
    c.take<double>(g.Rpad);
    c.take<double>(g.Rpad);
    c.take<uint32_t>(64);
    c.take<uint32_t>(kMaxGrid);
    c.take<uint64_t>((size_t)2 * g.RB * g.Rpad * 8);  // register-Delta form: candidate records
    c.take<uint64_t>((size_t)2 * g.Rpad * 4);         // ... result records
    c.take<uint32_t>(g.Rpad);                          // ... X publication flags
    return c.bytes();
}

std::string mrhs_tune_key(int64_t d, int64_t n, int64_t nrhs, csk_dtype lp)
{
    return tune_key("mrhs|d=%lld|n=%lld|nrhs=%lld|dtype=%d", (long long)d, (long long)n, (long long)nrhs, (int)lp);
}
}  // namespace

// The row-tile counts a launch may use: from the default (fewest) up to
// kMaxRT.  The workspace covers all of them (more row tiles can pad more rows).
int mrhs_rt_min(int64_t d, int64_t n, int64_t nrhs) { return geom(d, n, nrhs).RT; }

size_t mrhs_ws_bytes(int64_t d, int64_t n, int64_t nrhs)
{
    size_t b = 0;
    for (int rt = std::max(1, mrhs_rt_min(d, n, nrhs)); rt <= kMaxRT; ++rt) b = std::max(b, ws_bytes_of(geom(d, n, nrhs, rt)));
    return std::max(b, ws_bytes_of(geom(d, n, nrhs)));
}

csk_status mrhs_run(const void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp, const double* At64, int64_t ldat64,
                    int64_t d, int64_t n, const double* Bt, int64_t nrhs, int64_t ldbt, const double* nu2,
                    const double* X0, double* X, int64_t ldx, const double* Xref, int64_t ldxref,
                    const csk_solve_opts* o, csk_solve_result* res, void* ws, size_t ws_bytes, hipStream_t st,
                    int rt_force)
{
    // row tiles: forced (tuning), else tuned for this shape, else the default
    int rt = rt_force;
    if (rt <= 0) {
        TuneRec tr{};
        if (tune_get(mrhs_tune_key(d, n, nrhs, lp_dtype), &tr) && tr.a >= mrhs_rt_min(d, n, nrhs) && tr.a <= kMaxRT)
            rt = tr.a;
    }
    const Geom g = geom(d, n, nrhs, rt);
    if ((nrhs + (int64_t)g.RB * g.CB - 1) / ((int64_t)g.RB * g.CB) > kMaxOwned) {
        set_error("multi-RHS: %lld right-hand sides on %d workgroups exceed %d per workgroup", (long long)nrhs,
                  g.RB * g.CB, kMaxOwned);
        return CSK_ERR_UNSUPPORTED;
    }
    if (g.RT > kMaxRT) {
        set_error("multi-RHS: d=%lld needs %d row tiles per workgroup (max %d)", (long long)d, g.RT, kMaxRT);
        return CSK_ERR_UNSUPPORTED;
    }
    if (g.RB * g.CB > kMaxGrid) {
        set_error("multi-RHS: %d workgroups exceed the %d barrier flags", g.RB * g.CB, kMaxGrid);
        return CSK_ERR_UNSUPPORTED;
    }
    Carve c(ws);
    MCtl C{};
    uint16_t* alp = c.take<uint16_t>((size_t)g.rows_pad * g.npad);
    C.XT = c.take<double>((size_t)g.Rpad * g.npad);
    C.XrT = c.take<double>((size_t)g.Rpad * g.npad);
    double* xut = c.take<double>((size_t)g.Rpad * g.npad);
    C.DT = c.take<uint16_t>((size_t)g.Rpad * g.npad);
    C.cand = c.take<CandRec>((size_t)g.RB * g.Rpad);
    double* colref2 = c.take<double>(g.Rpad);
    double* colbt2 = c.take<double>(g.Rpad);
    C.dinv = c.take<double>(g.Rpad);
    uint32_t* ctr = c.take<uint32_t>(64);
    uint32_t* flags = c.take<uint32_t>(kMaxGrid);
    uint64_t* rd_cand = c.take<uint64_t>((size_t)2 * g.RB * g.Rpad * 8);
    uint64_t* rd_res = c.take<uint64_t>((size_t)2 * g.Rpad * 4);
    uint32_t* rd_xflag = c.take<uint32_t>(g.Rpad);
    if (c.bytes() > ws_bytes) {
        set_error("multi-RHS workspace too small: need %zu bytes, got %zu", c.bytes(), ws_bytes);
        return CSK_ERR_WORKSPACE;
    }
    C.Alp = alp;
    C.A64 = At64;
    C.lda64 = ldat64;
    C.Bt = Bt;
    C.ldbt = ldbt;
    C.nu2 = nu2;
    C.XuT = (o->stop_mode == CSK_STOP_REL_ERR) ? xut : nullptr;
    C.colref2 = colref2;
    C.colbt2 = colbt2;
    C.res = res;
    C.flags = flags;
    C.active = ctr + 1;
    C.cancel_seen = reinterpret_cast<int32_t*>(ctr + 2);
    C.cancel = o->cancel;
    C.tol2 = o->tol * o->tol;
    C.maxit = o->maxit;
    C.d = (int32_t)d;
    C.n = (int32_t)n;
    C.npad = g.npad;
    C.R = (int32_t)nrhs;
    C.Rpad = g.Rpad;
    C.RB = g.RB;
    C.CB = g.CB;
    C.refresh_every = o->refresh_every > 0 ? o->refresh_every : 64;
    C.check_every = o->check_every > 0 ? o->check_every : 256;
    C.stop_mode = o->stop_mode;

    k_pad_lp<<<grid_for((int64_t)g.rows_pad * g.npad, 8192), 256, 0, st>>>(
        static_cast<const uint16_t*>(At_lp), ldat_lp, (int)d, (int)n, alp, g.rows_pad, g.npad);
    CSK_LAUNCH_CHECK("k_pad_lp");
    k_init_cols<<<grid_for((int64_t)g.Rpad * g.npad, 8192), 256, 0, st>>>(
        X0, ldx, Xref, ldxref, (int)n, (int)nrhs, g.Rpad, g.npad, C.XT, C.XrT, C.XuT ? xut : nullptr, C.DT);
    CSK_LAUNCH_CHECK("k_init_cols");
    k_col_norms<<<(int)nrhs, 256, 0, st>>>(C.XuT, g.npad, (int)n, Bt, ldbt, (int)d, colref2, colbt2);
    CSK_LAUNCH_CHECK("k_col_norms");
    k_init_counters<<<grid_for((int64_t)g.RB * g.Rpad, 1024), 256, 0, st>>>(C.flags, C.active, C.cancel_seen,
                                                                              (int)nrhs, C.cand,
                                                                              (int64_t)g.RB * g.Rpad, C.dinv,
                                                                              g.Rpad);
    CSK_LAUNCH_CHECK("k_init_counters");
    const int G = g.RB * g.CB;
    csk_status r;
    if (rd_fits(g, nrhs)) {
        RdCtl D{};
        D.Alp = alp;
        D.A64 = At64;
        D.lda64 = ldat64;
        D.Bt = Bt;
        D.ldbt = ldbt;
        D.nu2 = nu2;
        D.XT = C.XT;
        D.XuT = C.XuT;
        D.cand = rd_cand;
        D.resw = rd_res;
        D.xflag = rd_xflag;
        D.colref2 = colref2;
        D.colbt2 = colbt2;
        D.res = res;
        D.cancel = o->cancel;
        D.tol2 = C.tol2;
        D.maxit = C.maxit;
        D.d = C.d;
        D.n = C.n;
        D.npad = C.npad;
        D.R = C.R;
        D.Rpad = C.Rpad;
        D.RB = C.RB;
        D.CB = C.CB;
        D.refresh_every = C.refresh_every;
        D.check_every = C.check_every;
        D.stop_mode = C.stop_mode;
        D.a_stride = g.npad + 8;
        D.nown = rd_nown(g, nrhs);
        const int64_t words = (int64_t)2 * g.RB * g.Rpad * 8 + (int64_t)2 * g.Rpad * 4 + (g.Rpad + 1) / 2;
        k_zero_u64<<<grid_for(words, 1024), 256, 0, st>>>(rd_cand, words);
        CSK_LAUNCH_CHECK("k_zero_u64");
        const size_t shm = rd_lds_bytes(g, D.nown);
        r = (lp_dtype == CSK_BF16) ? dispatch_rd<tag_bf16>(D, g.RT, G, st, shm) : dispatch_rd<tag_f16>(D, g.RT, G, st, shm);
    } else {
        r = (lp_dtype == CSK_BF16) ? dispatch<tag_bf16>(C, g.RT, G, st) : dispatch<tag_f16>(C, g.RT, G, st);
    }
    if (r != CSK_OK) return r;
    k_store_x<<<grid_for(n * nrhs, 8192), 256, 0, st>>>(C.XT, g.npad, (int)n, (int)nrhs, X, ldx);
    CSK_LAUNCH_CHECK("k_store_x");
    return CSK_OK;
}

// Times `trial_iters` iterations (no convergence: tol 0, residual mode) of
// every row-tile count from the default up to kMaxRT, and stores the fastest.
csk_status mrhs_tune(const void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp, const double* At64, int64_t ldat64,
                     int64_t d, int64_t n, const double* Bt, int64_t nrhs, int64_t ldbt, const double* nu2,
                     int32_t trial_iters, csk_tune_report* rep, void* ws, size_t ws_bytes, hipStream_t st)
{
    Carve c(ws);
    void* sws = c.take<char>(mrhs_ws_bytes(d, n, nrhs));
    double* X = c.take<double>((size_t)n * nrhs);
    csk_solve_result* res = c.take<csk_solve_result>(nrhs);
    if (c.bytes() > ws_bytes) {
        set_error("tuning workspace: need %zu bytes, got %zu", c.bytes(), ws_bytes);
        return CSK_ERR_WORKSPACE;
    }
    csk_solve_opts o{};
    o.tol = 0.0;
    o.maxit = trial_iters;
    o.stop_mode = CSK_STOP_REL_RESID;
    o.refresh_every = 64;
    o.check_every = 256;
    hipEvent_t e0, e1;
    CSK_HIP(hipEventCreate(&e0));
    CSK_HIP(hipEventCreate(&e1));
    const int rt0 = mrhs_rt_min(d, n, nrhs);
    csk_tune_report R{0, rt0, 0.0, 0.0, 0};
    csk_status r = CSK_OK;
    for (int rt = rt0; rt <= kMaxRT && r == CSK_OK; ++rt) {
        if (rt > rt0 && geom(d, n, nrhs, rt).RB == geom(d, n, nrhs, rt - 1).RB) continue;  // same launch
        r = mrhs_run(At_lp, lp_dtype, ldat_lp, At64, ldat64, d, n, Bt, nrhs, ldbt, nu2, nullptr, X, n, nullptr, 0,
                     &o, res, sws, mrhs_ws_bytes(d, n, nrhs), st, rt);
        if (r == CSK_ERR_UNSUPPORTED) { r = CSK_OK; continue; }  // this shape does not launch here
        if (r != CSK_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) { set_error("hipEventRecord failed"); r = CSK_ERR_DEVICE; break; }
        r = mrhs_run(At_lp, lp_dtype, ldat_lp, At64, ldat64, d, n, Bt, nrhs, ldbt, nu2, nullptr, X, n, nullptr, 0,
                     &o, res, sws, mrhs_ws_bytes(d, n, nrhs), st, rt);
        if (r != CSK_OK) break;
        if (hipEventRecord(e1, st) != hipSuccess) { set_error("hipEventRecord failed"); r = CSK_ERR_DEVICE; break; }
        if (hipEventSynchronize(e1) != hipSuccess) { set_error("tuning run failed"); r = CSK_ERR_DEVICE; break; }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { set_error("hipEventElapsedTime failed"); r = CSK_ERR_DEVICE; break; }
        const double us = ms * 1e3 / trial_iters;
        ++R.candidates;
        if (rt == rt0) R.default_us = us;
        if (R.choice == 0 || us < R.us) {
            R.choice = rt;
            R.us = us;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != CSK_OK) return r;
    if (R.choice == 0) { set_error("no multi-RHS launch shape fits this system"); return CSK_ERR_UNSUPPORTED; }
    tune_put(mrhs_tune_key(d, n, nrhs, lp_dtype), TuneRec{R.choice, 0, R.us});
    if (rep) *rep = R;
    return CSK_OK;
}

size_t mrhs_tune_ws_bytes(int64_t d, int64_t n, int64_t nrhs)
{
    Carve c(nullptr);
    c.take<char>(mrhs_ws_bytes(d, n, nrhs));
    c.take<double>((size_t)n * nrhs);
    c.take<csk_solve_result>(nrhs);
    return c.bytes();
}

}  // namespace csk
