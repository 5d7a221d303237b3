// csk_grid.h -- reduction record and grid-wide barrier shared by the
// persistent kernels (cooperative launch, all workgroups co-resident).
#pragma once

#include "csk_internal.h"

namespace csk {

constexpr uint32_t kSpinLimit = 5u * 1000u * 1000u;  // bounded wait: several seconds
enum : uint32_t { kFlagNonfinite = 1u, kFlagCancel = 2u, kFlagTimeout = 4u };

// A workgroup's contribution to an iteration: best candidate row (score,
// residual, index), partial ||r||^2, partial ||x - x_ref||^2 and flags.
struct GridRed {
    double score, r, r2, e2;
    uint32_t idx, flags;
};

__device__ __forceinline__ GridRed red_identity()
{
    GridRed v;
    v.score = 0.0;
    v.r = 0.0;
    v.r2 = 0.0;
    v.e2 = 0.0;
    v.idx = kNoRow;
    v.flags = 0u;
    return v;
}

// Larger score wins, then the lower row index; sums add in the order of the
// fixed reduction tree, so every workgroup computing the same reduction
// gets bitwise the same result.
__device__ __forceinline__ GridRed red_combine(GridRed a, const GridRed& b)
{
    if (cand_better(b.score, b.idx, a.score, a.idx)) {
        a.score = b.score;
        a.r = b.r;
        a.idx = b.idx;
    }
    a.r2 = a.r2 + b.r2;
    a.e2 = a.e2 + b.e2;
    a.flags |= b.flags;
    return a;
}

template <int WIDTH = kWave>
__device__ __forceinline__ GridRed wave_red(GridRed v)
{
#pragma unroll
    for (int off = WIDTH / 2; off > 0; off >>= 1) {
        GridRed o;
        o.score = __shfl_xor(v.score, off, kWave);
        o.r = __shfl_xor(v.r, off, kWave);
        o.r2 = __shfl_xor(v.r2, off, kWave);
        o.e2 = __shfl_xor(v.e2, off, kWave);
        o.idx = __shfl_xor(v.idx, off, kWave);
        o.flags = __shfl_xor(v.flags, off, kWave);
        v = red_combine(v, o);
    }
    return v;
}

// The same reduction with DPP lane moves inside each row of 16 lanes
// (quad permutations, then the half-row and row mirrors: each step pairs
// lanes whose partial results cover disjoint lane sets, so after four steps
// every lane holds its row's reduction) and the four rows combined in a
// fixed order from lanes 0, 16, 32, 48.  The result is uniform.
template <int CTRL> __device__ __forceinline__ uint32_t dpp_u32(uint32_t v)
{
    return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(v));
    const uint64_t lo = dpp_u32<CTRL>(static_cast<uint32_t>(b));
    const uint64_t hi = dpp_u32<CTRL>(static_cast<uint32_t>(b >> 32));
    return __longlong_as_double(static_cast<long long>((hi << 32) | lo));
}
template <int CTRL> __device__ __forceinline__ GridRed dpp_step(const GridRed& v)
{
    GridRed o;
    o.score = dpp_f64<CTRL>(v.score);
    o.r = dpp_f64<CTRL>(v.r);
    o.r2 = dpp_f64<CTRL>(v.r2);
    o.e2 = dpp_f64<CTRL>(v.e2);
    o.idx = dpp_u32<CTRL>(v.idx);
    o.flags = dpp_u32<CTRL>(v.flags);
    return red_combine(v, o);
}
__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(v));
    const uint64_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(b), lane));
    const uint64_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane));
    return __longlong_as_double(static_cast<long long>((hi << 32) | lo));
}
__device__ __forceinline__ GridRed readlane_red(const GridRed& v, int lane)
{
    GridRed o;
    o.score = readlane_f64(v.score, lane);
    o.r = readlane_f64(v.r, lane);
    o.r2 = readlane_f64(v.r2, lane);
    o.e2 = readlane_f64(v.e2, lane);
    o.idx = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v.idx), lane));
    o.flags = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v.flags), lane));
    return o;
}
__device__ __forceinline__ GridRed wave_red_dpp(GridRed v)
{
    v = dpp_step<0xB1>(v);   // quad_perm [1,0,3,2]
    v = dpp_step<0x4E>(v);   // quad_perm [2,3,0,1]
    v = dpp_step<0x141>(v);  // row_half_mirror
    v = dpp_step<0x140>(v);  // row_mirror
    GridRed t = readlane_red(v, 0);
    t = red_combine(t, readlane_red(v, 16));
    t = red_combine(t, readlane_red(v, 32));
    return red_combine(t, readlane_red(v, 48));
}

// Workgroup reduction with one barrier: every thread gets the result.  The
// caller alternates slot arrays so that a later reduction never overwrites
// slots another wave may still be reading (a barrier always separates two
// uses of the same array).
template <int NT>
__device__ __forceinline__ GridRed block_red1(GridRed v, GridRed* slots)
{
    v = wave_red_dpp(v);
    if ((threadIdx.x & (kWave - 1)) == 0) slots[threadIdx.x / kWave] = v;
    __syncthreads();
    GridRed t = slots[0];
#pragma unroll
    for (int w = 1; w < NT / kWave; ++w) t = red_combine(t, slots[w]);
    return t;
}

// Fixed-shape reduction over a workgroup of NT threads; every thread gets the
// result.  slots: NT/64 records in LDS.
template <int NT>
__device__ __forceinline__ GridRed block_red(GridRed v, GridRed* slots)
{
    v = wave_red_dpp(v);
    if ((threadIdx.x & (kWave - 1)) == 0) slots[threadIdx.x / kWave] = v;
    __syncthreads();
    GridRed t = slots[0];
#pragma unroll
    for (int w = 1; w < NT / kWave; ++w) t = red_combine(t, slots[w]);
    __syncthreads();
    return t;
}

// Device-coherent accesses ("sc1": coherent across the chip's L2 slices,
// without writing back or invalidating them).  Data that one workgroup
// writes and another reads while the kernel runs moves only through these.
template <class T> __device__ __forceinline__ void coh_store(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T> __device__ __forceinline__ T coh_load(const T* p)
{
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier for kernels whose cross-workgroup data moves only through
// coh_store / coh_load.  Every wavefront waits for its own stores to be
// acknowledged; then workgroup wg stores the epoch in its own flag and all
// workgroups poll all G flags in parallel (one request per flag and round).
// There is no shared atomic counter, whose G serialized updates would
// dominate, and no fence: the L2 slices keep their (read-only) lines, where
// a release/acquire pair would write them back and invalidate them.  Flags
// start at zero and epochs count up from 1; the spin is bounded (false:
// timed out).
// Ordering: the data stores before the barrier are device-coherent relaxed
// stores, and the flag store is issued only after s_waitcnt 0 has seen each
// of them acknowledged by the coherent level.  The wait builtin alone is not
// a compiler barrier, so signal fences on both sides keep the compiler from
// moving any memory access across it; the workgroup barrier then orders the
// other waves' acknowledged stores before thread 0's flag store.
__device__ __forceinline__ bool grid_barrier_flags(uint32_t* flags, int wg, int G, uint32_t epoch, uint32_t* s_ok)
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (threadIdx.x == 0) *s_ok = 1u;
    __syncthreads();
    if (threadIdx.x == 0) coh_store(&flags[wg], epoch);
    for (int w = threadIdx.x; w < G; w += blockDim.x) {
        uint32_t spins = 0;
        while (static_cast<int32_t>(coh_load(&flags[w]) - epoch) < 0) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > kSpinLimit) {
                *s_ok = 0u;
                break;
            }
        }
    }
    __syncthreads();
    return *s_ok != 0u;
}

// Sum over an aligned group of W lanes (4, 16 or 64), every lane of the
// group getting the same bits: DPP moves inside quads and 16-lane rows (each
// step adds two partial sums over disjoint lane sets, a + b on one side and
// b + a on the other), and for W = 64 the four row sums read from lanes 0,
// 16, 32, 48 and added in that order.
template <int CTRL> __device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_move(double v)
{
    return dpp_f64<CTRL>(v);
}
__device__ __forceinline__ float lane_value(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double lane_value(double v, int lane) { return readlane_f64(v, lane); }

template <class T, int W>
__device__ __forceinline__ T group_sum_t(T v)
{
    static_assert(W == 4 || W == 16 || W == 64, "lane group");
    v = v + dpp_move<0xB1>(v);  // quad_perm [1,0,3,2]
    v = v + dpp_move<0x4E>(v);  // quad_perm [2,3,0,1]
    if constexpr (W >= 16) {
        v = v + dpp_move<0x141>(v);  // row_half_mirror
        v = v + dpp_move<0x140>(v);  // row_mirror
    }
    if constexpr (W == 64) v = ((lane_value(v, 0) + lane_value(v, 16)) + lane_value(v, 32)) + lane_value(v, 48);
    return v;
}

// Storage of one workgroup's published contribution to an iteration (eight
// tagged words; exchange() interleaves the words of four records).
struct alignas(64) XRec {
    uint64_t w[8];
};

// Publish this workgroup's record for iteration k and reduce all G records
// (grid loops).  A record is eight 64-bit words, each
// carrying 32 bits of payload and, in its upper half, the iteration tag
// k + 1 (tags start at zero; two slots alternate by parity, so a stale word
// is never mistaken for a fresh one).  Words are written and read with
// device-coherent 64-bit accesses, so a reader accepts the record once all
// eight tags match: no acknowledgement wait on the writer, no second read,
// and no cache write-back or invalidation (the workgroup's rows of At stay
// in L2).  Payload: score, alpha, the stop measure (||x - x_ref||^2 part or
// ||r||^2 part), row index, flags; with `both`, ||r||^2 and ||x - x_ref||^2
// in place of alpha and the stop measure (alpha then reads zero).
// Layout: records in groups of four consecutive workgroups, word-major inside
// a group (word f of the group's records in one 32-byte run; a short last
// group takes the same form with fewer records), so the polled first words
// of 64 records lie in 16 cache lines of 128 bytes, each written by four
// workgroups.  Against one record per 64 bytes (32 lines per poll, two
// writers per line) this took the FP64 solve of a 200000 x 1000 system
// sketched to d = 20000 (256 workgroups) from 126.0 to 124.8 ms, and the
// BF16 iteration at d = 10000, n = 1000 from 9.19 to 9.02 us; groups of
// eight (eight lines, eight writers), whole word-major rows (four lines,
// sixteen writers) and one record per 128-byte line (64 lines, one writer)
// were each 1 to 10% slower.
__host__ __device__ constexpr size_t xrec_word(int f, int w, int G)
{
    return (size_t)(w & ~3) * 8 + (size_t)f * (G - (w & ~3) < 4 ? G - (w & ~3) : 4) + (w & 3);
}
__device__ __forceinline__ double join_f64(uint64_t lo, uint64_t hi)
{
    return __longlong_as_double((long long)((hi << 32) | (lo & 0xFFFFFFFFull)));
}

template <int NT>
__device__ __forceinline__ GridRed exchange(const GridRed& mine, XRec* exch, int wg, int G, int64_t k, GridRed* slots,
                                            bool rel_err, bool both = false)  // slots: reduced with block_red1
{
    uint64_t* slot = reinterpret_cast<uint64_t*>(exch + (size_t)(k & 1) * G);  // words xrec_word(f, w, G)
    const uint64_t tag = static_cast<uint64_t>(static_cast<uint32_t>(k + 1)) << 32;
    if (threadIdx.x < 8) {
        const int f = threadIdx.x;
        const double dv = f < 2 ? mine.score
                          : f < 4 ? (both ? mine.r2 : mine.r)
                                  : ((rel_err || both) ? mine.e2 : mine.r2);
        const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(dv));
        const uint32_t p = f < 6 ? static_cast<uint32_t>((f & 1) ? (bits >> 32) : bits)
                                 : (f == 6 ? mine.idx : mine.flags);
        coh_store(&slot[xrec_word(f, wg, G)], tag | p);
    }
    bool ok = true;
    GridRed all = red_identity();
    for (int w = threadIdx.x; w < G; w += NT) {
        GridRed o;
        if (w == wg) {
            o = mine;  // this workgroup's own record needs no round trip
            if (both) o.r = 0.0;
            else if (rel_err) o.r2 = 0.0;
            else o.e2 = 0.0;
        } else {
            // Poll one word of the record (one request per record and round:
            // the G x G polls of a grid are the exchange's main traffic), then
            // read the record; its eight words leave in one store instruction, so
            // a stale word after a fresh first one is rare and just re-read.
            // Between polls a thread sleeps about 0.3 us (12 x 64 cycles): at
            // 256 workgroups, polling every 0.05 us made the solve 0.3%
            // slower at 17 and at 9 us per iteration, and every 0.6 or 1.3 us
            // up to 4% slower at 9 us (a fresh record is seen later).
            uint64_t v[8];
            uint32_t spins = 0;
            while ((coh_load(&slot[xrec_word(0, w, G)]) & 0xFFFFFFFF00000000ull) != tag) {
                __builtin_amdgcn_s_sleep(12);
                if (++spins > kSpinLimit) {
                    ok = false;
                    break;
                }
            }
            while (ok) {
#pragma unroll
                for (int f = 0; f < 8; ++f) v[f] = coh_load(&slot[xrec_word(f, w, G)]);
                bool fresh = true;
#pragma unroll
                for (int f = 0; f < 8; ++f) fresh = fresh && ((v[f] & 0xFFFFFFFF00000000ull) == tag);
                if (fresh) break;
                __builtin_amdgcn_s_sleep(1);
                if (++spins > kSpinLimit) ok = false;
            }
            if (!ok) break;
            o.score = join_f64(v[0], v[1]);
            const double w23 = join_f64(v[2], v[3]);
            const double w45 = join_f64(v[4], v[5]);
            o.r = both ? 0.0 : w23;
            o.r2 = both ? w23 : (rel_err ? 0.0 : w45);
            o.e2 = (both || rel_err) ? w45 : 0.0;
            o.idx = static_cast<uint32_t>(v[6]);
            o.flags = static_cast<uint32_t>(v[7]);
        }
        all = red_combine(all, o);
    }
    if (!ok) all.flags |= kFlagTimeout;
    return block_red1<NT>(all, slots);
}

}  // namespace csk
