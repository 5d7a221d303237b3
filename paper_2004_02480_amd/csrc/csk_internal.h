// csk_internal.h -- device helpers and host plumbing shared by the libcsk
// translation units (hash of Definition 1, precision conversions, wavefront
// reductions, workspace carving, error reporting).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "csk.h"

namespace csk {

// ---------------------------------------------------------------------------
// Definition 1: the count sketch's random map h and signs D.
// One 64-bit SplitMix64 output per input row (counter form: the (i+1)-th
// output of the generator seeded with `seed`), bucket from the high word by
// a 32x32 multiply-high, sign from the low bit.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint64_t draw_word(uint64_t seed, uint64_t row)
{
    uint64_t z = seed + (row + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Uniforms of the randomized selection rules: the k-th of a stream is the
// top 52 bits of the k-th SplitMix64 output of its seed plus one half, times
// 2^-52 (every step exact; strictly inside (0, 1)).
__device__ __forceinline__ double select_uniform(uint64_t seed, uint64_t k)
{
    return (static_cast<double>(draw_word(seed, k) >> 12) + 0.5) * 0x1p-52;
}

__device__ __forceinline__ uint32_t draw_bucket(uint64_t w, uint32_t d)
{
    return __umulhi(static_cast<uint32_t>(w >> 32), d);
}

__device__ __forceinline__ double draw_sign(uint64_t w)
{
    return (w & 1ull) ? -1.0 : 1.0;
}

// ---------------------------------------------------------------------------
// Precision.  Low-precision copies of an FP64 value are rounded in two IEEE
// round-to-nearest-even steps (FP64 -> FP32 -> 16-bit); the conversions are
// the compiler's IEEE conversions for __bf16 and _Float16.
// ---------------------------------------------------------------------------
// The FP32 intermediate is pinned in a register (empty asm) so the compiler
// cannot fuse the two conversions into one direct FP64 -> 16-bit rounding,
// which differs from the two-step result when the FP64 value lies within
// one FP32 ulp of a 16-bit halfway point.
__device__ __forceinline__ float f64_to_f32_pinned(double v)
{
    float f = static_cast<float>(v);
    asm volatile("" : "+v"(f));
    return f;
}

__device__ __forceinline__ uint16_t f64_to_bf16_bits(double v)
{
    __bf16 h = static_cast<__bf16>(f64_to_f32_pinned(v));
    return __builtin_bit_cast(uint16_t, h);
}

__device__ __forceinline__ uint16_t f64_to_f16_bits(double v)
{
    _Float16 h = static_cast<_Float16>(f64_to_f32_pinned(v));
    return __builtin_bit_cast(uint16_t, h);
}

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b)
{
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

__device__ __forceinline__ float f16_bits_to_f32(uint16_t b)
{
    return static_cast<float>(__builtin_bit_cast(_Float16, b));
}

// Storage tags for the low-precision sketch.
struct tag_f32 { using storage = float; };
struct tag_f16 { using storage = uint16_t; };
struct tag_bf16 { using storage = uint16_t; };

template <class Tag> __device__ __forceinline__ typename Tag::storage round_store(double v);
template <> __device__ __forceinline__ float round_store<tag_f32>(double v) { return static_cast<float>(v); }
template <> __device__ __forceinline__ uint16_t round_store<tag_f16>(double v) { return f64_to_f16_bits(v); }
template <> __device__ __forceinline__ uint16_t round_store<tag_bf16>(double v) { return f64_to_bf16_bits(v); }

template <class Tag> __device__ __forceinline__ float widen(typename Tag::storage v);
template <> __device__ __forceinline__ float widen<tag_f32>(float v) { return v; }
template <> __device__ __forceinline__ float widen<tag_f16>(uint16_t v) { return f16_bits_to_f32(v); }
template <> __device__ __forceinline__ float widen<tag_bf16>(uint16_t v) { return bf16_bits_to_f32(v); }

// ---------------------------------------------------------------------------
// Wavefront (64-lane) reductions.  The xor-butterfly gives every lane the
// same result with a fixed association order, so repeated runs are bitwise
// identical.
// ---------------------------------------------------------------------------
constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <int WIDTH>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int off = WIDTH / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WIDTH);
    return v;
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// A selection candidate: weighted score of a row (r^2 / nu2), its residual
// and index.  Larger score wins; equal scores go to the lower index; rows
// that cannot be selected carry idx = kNoRow.
constexpr uint32_t kNoRow = 0xFFFFFFFFu;

struct Cand {
    double score;
    double r;
    uint32_t idx;
};

__device__ __forceinline__ bool cand_better(double s1, uint32_t i1, double s2, uint32_t i2)
{
    if (i1 == kNoRow) return false;
    if (i2 == kNoRow) return true;
    return (s1 > s2) || (s1 == s2 && i1 < i2);
}

__device__ __forceinline__ Cand wave_argmax(Cand c)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double os = __shfl_xor(c.score, off, kWave);
        double orr = __shfl_xor(c.r, off, kWave);
        uint32_t oi = __shfl_xor(c.idx, off, kWave);
        if (cand_better(os, oi, c.score, c.idx)) { c.score = os; c.r = orr; c.idx = oi; }
    }
    return c;
}

// ---------------------------------------------------------------------------
// Host helpers.
// ---------------------------------------------------------------------------
void set_error(const char* fmt, ...);
csk_status hip_fail(hipError_t e, const char* what);

#define CSK_HIP(call)                                           \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return ::csk::hip_fail(e_, #call); \
    } while (0)

#define CSK_LAUNCH_CHECK(what)                                  \
    do {                                                        \
        hipError_t e_ = hipGetLastError();                      \
        if (e_ != hipSuccess) return ::csk::hip_fail(e_, what); \
    } while (0)

// Bump allocator over the caller's workspace (256-byte aligned pieces).  Used
// both by the size queries (base == nullptr) and by the calls themselves, so
// the two always agree.
struct Carve {
    char* base;
    size_t used = 0;
    explicit Carve(void* b) : base(static_cast<char*>(b)) {}
    template <class T> T* take(size_t count)
    {
        size_t off = (used + 255) & ~size_t(255);
        used = off + count * sizeof(T);
        return base ? reinterpret_cast<T*>(base + off) : nullptr;
    }
    size_t bytes() const { return (used + 255) & ~size_t(255); }
};

inline size_t dtype_size(csk_dtype t)
{
    switch (t) {
    case CSK_F64: return 8;
    case CSK_F32: return 4;
    case CSK_F16: return 2;
    case CSK_BF16: return 2;
    default: return 0;
    }
}

int device_cu_count();
// Copies count host int32 values to device memory, stream-ordered, through
// kernel arguments (no staging allocation).
csk_status upload_i32(const int32_t* host, int64_t count, int32_t* dev, hipStream_t st);
// Largest LDS allocation of one workgroup on the current device, in bytes.
int device_max_lds();

}  // namespace csk
