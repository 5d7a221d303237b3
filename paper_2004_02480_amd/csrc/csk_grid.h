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

// Fixed-shape reduction over a workgroup of NT threads; every thread gets the
// result.  slots: NT/64 records in LDS.
template <int NT>
__device__ __forceinline__ GridRed block_red(GridRed v, GridRed* slots)
{
    v = wave_red(v);
    if ((threadIdx.x & (kWave - 1)) == 0) slots[threadIdx.x / kWave] = v;
    __syncthreads();
    GridRed t = slots[0];
#pragma unroll
    for (int w = 1; w < NT / kWave; ++w) t = red_combine(t, slots[w]);
    __syncthreads();
    return t;
}

// Grid barrier: arrival counter (zeroed before launch) with release/acquire
// at device scope; epoch e waits for e * G arrivals.  The spin is bounded,
// so a kernel always terminates; false means the wait timed out.
// Only thread 0 performs the device-scope release, and a workgroup barrier
// by itself does not wait for other wavefronts' stores to complete.  When
// wavefronts other than the one holding thread 0 wrote data that other
// workgroups read after the barrier, ALL_WAVES makes every wavefront wait
// for its stores before the workgroup barrier, so the release covers them.
template <bool ALL_WAVES = false>
__device__ __forceinline__ bool grid_barrier(uint32_t* ctr, uint32_t target, uint32_t* s_ok)
{
    if constexpr (ALL_WAVES) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        uint32_t ok = 1u;
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        while (static_cast<int32_t>(__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kSpinLimit) {
                ok = 0u;
                break;
            }
        }
        *s_ok = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return *s_ok != 0u;
}

}  // namespace csk
