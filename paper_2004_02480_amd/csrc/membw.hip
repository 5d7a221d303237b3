// membw.hip -- read-bandwidth reference kernels for the benchmark (built
// into libcsk_membw.so, separate from libcsk.so; nothing on the solve path
// calls them).  They give the ceilings the solve and the sketch are compared
// against: a plain streaming read of a buffer far larger than the Infinity
// Cache (HBM), and repeated reads of a buffer that fits it (MALL), with the
// access pattern of the persistent solve (each workgroup walks its own
// contiguous block, 16-byte vectors per lane, many loads in flight), and a
// streaming read+write mix with the sketch's ratio of bytes read to bytes
// written (P arrays summed into one).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kThreads = 512;
constexpr int kUnroll = 8;  // 16-byte loads in flight per lane

// Each workgroup reads its contiguous block [lo, hi) of the `nvec` 16-byte
// vectors (equal blocks, the last one shorter), `reps` times, and folds what
// it read into one word (so no load can be dropped).
__global__ __launch_bounds__(kThreads) void k_read_blocks(const uint4* __restrict__ p, int64_t nvec, int reps,
                                                           uint32_t* __restrict__ sink)
{
    const int64_t G = gridDim.x;
    const int64_t round = (int64_t)kThreads * kUnroll;
    const int64_t per = (nvec + G - 1) / G;
    const int64_t lo = min(nvec, (int64_t)blockIdx.x * per);
    const int64_t hi = min(nvec, lo + per);
    uint32_t acc = 0;
    for (int r = 0; r < reps; ++r) {
        int64_t i = lo + threadIdx.x;
        for (; i + (kUnroll - 1) * kThreads < hi; i += round) {
            uint4 v[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) v[u] = p[i + u * kThreads];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
        }
        for (; i < hi; i += kThreads) {
            const uint4 v = p[i];
            acc ^= v.x ^ v.y ^ v.z ^ v.w;
        }
    }
    if (acc == 0x9E3779B9u) sink[blockIdx.x] = acc;  // practically never taken; keeps the loads live
}

// out[k] = sum over c < P of src[c * nvec + k], in 16-byte vectors of two
// doubles: P streams read and one written, all coalesced, one vector per
// thread (a grid-stride loop covers grids smaller than nvec / 256).
constexpr int kMixMax = 16;
constexpr int kMixThreads = 256;
__global__ __launch_bounds__(kMixThreads) void k_read_mix(const double2* __restrict__ src, int64_t nvec, int P,
                                                          double2* __restrict__ out)
{
    for (int64_t k = blockIdx.x * (int64_t)kMixThreads + threadIdx.x; k < nvec; k += (int64_t)gridDim.x * kMixThreads) {
        double2 v[kMixMax];
#pragma unroll
        for (int c = 0; c < kMixMax; ++c)
            if (c < P) v[c] = src[c * nvec + k];
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < kMixMax; ++c)
            if (c < P) {
                s.x += v[c].x;
                s.y += v[c].y;
            }
        out[k] = s;
    }
}

}  // namespace

extern "C" {

// Reads `bytes` (a multiple of 16, from a 16-byte aligned device pointer)
// `reps` times with `grid` workgroups of 512 threads on `stream`.  `sink`:
// device scratch of `grid` words (written at most by chance).  Returns 0, or
// the HIP error code of the launch.
int membw_read(const void* p, int64_t bytes, int reps, int grid, void* sink, void* stream)
{
    if (!p || bytes < 16 || (bytes & 15) || reps < 1 || grid < 1 || !sink) return (int)hipErrorInvalidValue;
    k_read_blocks<<<grid, kThreads, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<const uint4*>(p), bytes / 16, reps, static_cast<uint32_t*>(sink));
    return (int)hipGetLastError();
}

// Sums `P` (1..16) arrays of `nvec` 16-byte vectors, stored one after
// another from `src`, into `out` (nvec vectors) with `grid` workgroups of
// 256 threads on `stream`: P * nvec * 16 bytes read and nvec * 16 written.
// Both pointers 16-byte aligned.  Returns 0, or the HIP error code.
int membw_mix(const void* src, int64_t nvec, int P, void* out, int grid, void* stream)
{
    if (!src || !out || nvec < 1 || P < 1 || P > kMixMax || grid < 1 ||
        ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(out)) & 15))
        return (int)hipErrorInvalidValue;
    k_read_mix<<<grid, kMixThreads, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<const double2*>(src), nvec, P, static_cast<double2*>(out));
    return (int)hipGetLastError();
}

}  // extern "C"
