// sketch.hip -- Algorithm 1, Initialize: At = S A and Bt = S B with the count
// sketch of Definition 1, for one system or a batch of systems.
//
// Pipeline (all on the caller's stream, no host round trip):
//   k_hash_hist      hash every row (h(i), D_ii) and count rows per bucket
//   k_scan_*         exclusive scan of the counts -> bucket offsets ptr
//   k_scatter        place each row index in its bucket's segment of perm
//   k_sort_segments  sort each segment ascending (one wavefront, in LDS)
//   k_long_segments  segments longer than the LDS sort capacity are rebuilt
//                    in ascending order by an ordered scan of the rows
//   k_segsum         one wavefront per (bucket, column chunk): stream the
//                    bucket's rows of A in ascending row order, accumulate the
//                    signed sum in FP64 registers (one lane owns each output
//                    element, so each sum is sequential and bit-exact), then
//                    store At64 / the rounded low-precision copy, the squared
//                    row norm and bt.
//   k_nu2_finalize   adds per-chunk squared norms in chunk order.
// The hot kernel is k_segsum: it reads A exactly once (m*n elements) and
// writes At once, so it is bound by HBM bandwidth.
#include "csk_sketch.h"

#include <algorithm>
#include <vector>

namespace csk {
namespace {

constexpr int kSortCap = 512;     // longest segment sorted by one wavefront in LDS
constexpr int kScanTile = 4096;   // counts per block in the scan (256 threads x 16)

struct Batch {
    const SketchSys* sys;        // nsys descriptors (device), when nsys > 1
    SketchSys one;               // the descriptor itself, when nsys == 1
    const int64_t* row_offs;     // nsys+1 prefix over rows (device)
    const int64_t* bkt_offs;     // nsys+1 prefix over buckets
    const int64_t* task_offs;    // nsys+1 prefix over segsum tasks
    uint32_t* cnt;               // D
    uint32_t* ptr;               // D+1
    uint32_t* perm;              // M (row index local to its system)
    double* nu2part;             // T
    uint32_t* scan_part;         // ceil(D / kScanTile)
    int64_t M, D, T;
    int32_t nsys;
};

__device__ __forceinline__ const SketchSys& sys_at(const Batch& b, int s)
{
    return b.nsys == 1 ? b.one : b.sys[s];
}

// Largest s with offs[s] <= g (offs[0] = 0, strictly increasing).
__device__ __forceinline__ int find_sys(const int64_t* offs, int nsys, int64_t g)
{
    int lo = 0, hi = nsys;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (offs[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_fill_u32(uint32_t* p, int64_t count, uint32_t v)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

__global__ __launch_bounds__(256) void k_hash_hist(Batch b)
{
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < b.M;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int s = b.nsys == 1 ? 0 : find_sys(b.row_offs, b.nsys, g);
        const SketchSys& S = sys_at(b, s);
        const uint64_t w = draw_word(S.seed, static_cast<uint64_t>(g - S.row_off));
        atomicAdd(&b.cnt[S.bkt_off + draw_bucket(w, static_cast<uint32_t>(S.d))], 1u);
    }
}

// Inclusive scan of one u32 per thread over a block of NT threads; returns
// the inclusive value and the block total in *total.
template <int NT>
__device__ __forceinline__ uint32_t block_incl_scan(uint32_t v, uint32_t* total)
{
    __shared__ uint32_t wsum[NT / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t t = __shfl_up(v, off, kWave);
        if (lane >= off) v += t;
    }
    if (lane == kWave - 1) wsum[wid] = v;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < NT / kWave; ++w) {
        uint32_t t = wsum[w];
        if (w < wid) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return v + before;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* __restrict__ cnt, int64_t D,
                                                    uint32_t* __restrict__ part)
{
    const int64_t base = blockIdx.x * (int64_t)kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanTile / 256; ++k) {
        const int64_t j = base + k * 256 + threadIdx.x;
        if (j < D) s += cnt[j];
    }
    uint32_t total;
    block_incl_scan<256>(s, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* __restrict__ part, int64_t nb,
                                                  uint32_t* __restrict__ ptr, int64_t D)
{
    uint32_t carry = 0;
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t j = base + threadIdx.x;
        const uint32_t v = j < nb ? part[j] : 0u;
        uint32_t total;
        const uint32_t incl = block_incl_scan<1024>(v, &total);
        if (j < nb) part[j] = carry + incl - v;
        carry += total;
    }
    if (threadIdx.x == 0) ptr[D] = carry;
}

__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* __restrict__ cnt, int64_t D,
                                                   const uint32_t* __restrict__ part,
                                                   uint32_t* __restrict__ ptr)
{
    constexpr int kPer = kScanTile / 256;
    const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * (int64_t)kPer;
    uint32_t v[kPer];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        v[k] = (base + k < D) ? cnt[base + k] : 0u;
        s += v[k];
    }
    uint32_t total;
    uint32_t run = block_incl_scan<256>(s, &total) - s + part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (base + k < D) ptr[base + k] = run;
        run += v[k];
    }
}

// The whole exclusive scan in one block when the counts are few (at most
// 1024 x kScanRegs): the counts are staged in LDS with coalesced loads, each
// thread sums and then rewrites a contiguous run of at most kScanRegs of
// them, one wave scan (plus the 16 wave totals) turns the run totals into
// run offsets, and the result leaves with coalesced stores.  (A per-wave
// scan of 64-element slices in registers cost six cross-lane shuffles per
// slice: about 13 us at 2500 to 22500 counts.)
constexpr int kScanRegs = 32;
constexpr int64_t kScanSingleMax = 16 * 64 * kScanRegs;
__global__ __launch_bounds__(1024) void k_scan_single(const uint32_t* __restrict__ cnt, int64_t D,
                                                     uint32_t* __restrict__ ptr)
{
    extern __shared__ uint32_t sc[];  // D counts, then their exclusive prefixes
    __shared__ uint32_t wtot[16];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    {
        // all of a thread's loads are issued before the first is waited for
        uint32_t v[kScanRegs];
#pragma unroll
        for (int k = 0; k < kScanRegs; ++k) {
            const int64_t j = threadIdx.x + (int64_t)k * 1024;
            v[k] = j < D ? cnt[j] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kScanRegs; ++k) {
            const int64_t j = threadIdx.x + (int64_t)k * 1024;
            if (j < D) sc[j] = v[k];
        }
    }
    __syncthreads();
    const int64_t per = (D + 1023) / 1024;
    const int64_t lo = min<int64_t>(D, threadIdx.x * per), hi = min<int64_t>(D, lo + per);
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanRegs; ++k)
        if (lo + k < hi) sum += sc[lo + k];
    uint32_t x = sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t t = __shfl_up(x, off, kWave);
        if (lane >= off) x += t;
    }
    if (lane == kWave - 1) wtot[w] = x;
    __syncthreads();
    uint32_t carry = 0, total = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t t = wtot[k];
        if (k < w) carry += t;
        total += t;
    }
    uint32_t run = carry + x - sum;
#pragma unroll
    for (int k = 0; k < kScanRegs; ++k)
        if (lo + k < hi) {
            const uint32_t v = sc[lo + k];
            sc[lo + k] = run;
            run += v;
        }
    __syncthreads();
    for (int64_t j = threadIdx.x; j < D; j += 1024) ptr[j] = sc[j];
    if (threadIdx.x == 0) ptr[D] = total;
}

__global__ __launch_bounds__(256) void k_scatter(Batch b)
{
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < b.M;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int s = b.nsys == 1 ? 0 : find_sys(b.row_offs, b.nsys, g);
        const SketchSys& S = sys_at(b, s);
        const uint64_t i = static_cast<uint64_t>(g - S.row_off);
        const int64_t gb = S.bkt_off + draw_bucket(draw_word(S.seed, i), static_cast<uint32_t>(S.d));
        // Counting down through cnt leaves it zero; the order inside the
        // segment is fixed afterwards by the sort.
        const uint32_t pos = atomicSub(&b.cnt[gb], 1u) - 1u;
        b.perm[b.ptr[gb] + pos] = static_cast<uint32_t>(i);
    }
}

// The same two steps for one system with at most kHistCap buckets, with the
// contention of the global counters taken out: each block owns a contiguous
// range of rows, counts them per bucket in LDS, and touches a global counter
// once per bucket it holds (a few dozen blocks, so a counter sees a few
// dozen updates instead of one per row).  The scatter reserves each bucket's
// slots for the block in one update and hands them out from LDS; the order
// inside a segment is fixed by the sort, as before.
constexpr int kHistCap = 32768;  // buckets counted in LDS (128 KB, dynamic)
constexpr int kHistNT = 1024;

__device__ __forceinline__ void block_hist(const SketchSys& S, int64_t r0, int64_t r1, uint32_t* h)
{
    const uint32_t d = static_cast<uint32_t>(S.d);
    for (uint32_t j = threadIdx.x; j < d; j += kHistNT) h[j] = 0u;
    __syncthreads();
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kHistNT)
        atomicAdd(&h[draw_bucket(draw_word(S.seed, static_cast<uint64_t>(i)), d)], 1u);
    __syncthreads();
}

__global__ __launch_bounds__(kHistNT) void k_hash_hist_lds(Batch b, int64_t rows_per_block)
{
    extern __shared__ uint32_t h[];  // d counters
    const SketchSys& S = b.one;
    const int64_t r0 = min(b.M, blockIdx.x * rows_per_block), r1 = min(b.M, r0 + rows_per_block);
    block_hist(S, r0, r1, h);
    for (uint32_t j = threadIdx.x; j < static_cast<uint32_t>(S.d); j += kHistNT)
        if (h[j]) atomicAdd(&b.cnt[j], h[j]);
}

__global__ __launch_bounds__(kHistNT) void k_scatter_lds(Batch b, int64_t rows_per_block)
{
    extern __shared__ uint32_t h[];  // d counters, then the block's next slot per bucket
    const SketchSys& S = b.one;
    const uint32_t d = static_cast<uint32_t>(S.d);
    const int64_t r0 = min(b.M, blockIdx.x * rows_per_block), r1 = min(b.M, r0 + rows_per_block);
    block_hist(S, r0, r1, h);
    // counting down through cnt (it ends at zero): this block's slots of
    // bucket j are ptr[j] + [old - h[j], old).  A thread's counter updates
    // and ptr loads are all issued before the first is waited for (d is at
    // most kHistCap, so a thread holds at most kPer buckets).
    constexpr int kPer = kHistCap / kHistNT;
    {
        uint32_t hv[kPer], old[kPer], base[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint32_t j = threadIdx.x + k * kHistNT;
            hv[k] = j < d ? h[j] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint32_t j = threadIdx.x + k * kHistNT;
            old[k] = hv[k] ? atomicSub(&b.cnt[j], hv[k]) : 0u;
            base[k] = hv[k] ? b.ptr[j] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint32_t j = threadIdx.x + k * kHistNT;
            if (hv[k]) h[j] = base[k] + old[k] - hv[k];
        }
    }
    __syncthreads();
    for (int64_t i = r0 + threadIdx.x; i < r1; i += kHistNT) {
        const uint32_t j = draw_bucket(draw_word(S.seed, static_cast<uint64_t>(i)), d);
        b.perm[atomicAdd(&h[j], 1u)] = static_cast<uint32_t>(i);
    }
}

// Four wavefronts per block, one bucket each per round; rank sort in LDS
// (row indices within a segment are distinct).
__global__ __launch_bounds__(256) void k_sort_segments(Batch b)
{
    __shared__ uint32_t buf[4][kSortCap];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int64_t rounds = (b.D + 4 * (int64_t)gridDim.x - 1) / (4 * (int64_t)gridDim.x);
    for (int64_t rd = 0; rd < rounds; ++rd) {
        const int64_t gb = (rd * gridDim.x + blockIdx.x) * 4 + wid;
        uint32_t beg = 0, len = 0;
        if (gb < b.D) {
            beg = b.ptr[gb];
            len = b.ptr[gb + 1] - beg;
        }
        const bool active = len > 1 && len <= (uint32_t)kSortCap;
        if (active)
            for (uint32_t e = lane; e < len; e += kWave) buf[wid][e] = b.perm[beg + e];
        __syncthreads();
        if (active) {
            for (uint32_t e = lane; e < len; e += kWave) {
                const uint32_t v = buf[wid][e];
                uint32_t rank = 0;
                for (uint32_t k = 0; k < len; ++k) rank += buf[wid][k] < v ? 1u : 0u;
                b.perm[beg + rank] = v;
            }
        }
        __syncthreads();
    }
}

// Segments longer than kSortCap: rebuild the segment in ascending row order
// by scanning the system's rows in order and compacting those that hash to
// the bucket (ballot + block prefix).
__global__ __launch_bounds__(256) void k_long_segments(Batch b)
{
    __shared__ uint32_t wcount[4];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    for (int64_t gb = blockIdx.x; gb < b.D; gb += gridDim.x) {
        const uint32_t beg = b.ptr[gb];
        const uint32_t len = b.ptr[gb + 1] - beg;
        if (len <= (uint32_t)kSortCap) continue;
        const int s = b.nsys == 1 ? 0 : find_sys(b.bkt_offs, b.nsys, gb);
        const SketchSys& S = sys_at(b, s);
        const uint32_t j = static_cast<uint32_t>(gb - S.bkt_off);
        uint32_t running = 0;
        for (int64_t base = 0; base < S.m; base += 256) {
            const int64_t i = base + threadIdx.x;
            const bool hit = i < S.m &&
                draw_bucket(draw_word(S.seed, static_cast<uint64_t>(i)), static_cast<uint32_t>(S.d)) == j;
            const unsigned long long mask = __ballot(hit);
            const uint32_t below = __popcll(mask & ((1ull << lane) - 1ull));
            if (lane == 0) wcount[wid] = __popcll(mask);
            __syncthreads();
            uint32_t before = 0, all = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                if (w < wid) before += wcount[w];
                all += wcount[w];
            }
            if (hit) b.perm[beg + running + before + below] = static_cast<uint32_t>(i);
            running += all;
            __syncthreads();
        }
    }
}

template <class T> struct VecOf;
template <> struct VecOf<double> { using type = double2; };
template <> struct VecOf<float> { using type = float4; };

// LP: 0 none, 1 f32, 2 f16, 3 bf16 (matches csk_dtype values for 1..3).
template <int LP>
__device__ __forceinline__ void store_lp(void* base, int64_t off, double v)
{
    if constexpr (LP == CSK_F32) static_cast<float*>(base)[off] = round_store<tag_f32>(v);
    if constexpr (LP == CSK_F16) static_cast<uint16_t*>(base)[off] = round_store<tag_f16>(v);
    if constexpr (LP == CSK_BF16) static_cast<uint16_t*>(base)[off] = round_store<tag_bf16>(v);
}

// Raw loads of one lane's part of a row chunk: VPL vectors of VW elements
// (16 bytes each when VW > 1).  Branch-free: a vector that starts at or past
// column n reads the row's first vector instead; a vector that starts before
// n may end past it, inside the row's 16-byte padded length (the vector
// path requires 16-byte rows).  Elements past n are never stored, so their
// bits do not matter.  Without branches the compiler never merges different
// loads, and its waits on the in-order vector-memory counter only wait for
// the row slot that is consumed.
template <class TA, int VW, int VPL>
__device__ __forceinline__ void load_row_chunk(TA (&v)[VPL][VW], const TA* __restrict__ rowp, int col0, int lane, int n)
{
#pragma unroll
    for (int q = 0; q < VPL; ++q) {
        const int col = col0 + (q * kWave + lane) * VW;
        const int cc = col < n ? col : 0;
        if constexpr (VW == 1) {
            v[q][0] = rowp[cc];
        } else {
            using V = typename VecOf<TA>::type;
            static_assert(sizeof(V) == sizeof(TA) * VW, "vector width");
            const V x = *reinterpret_cast<const V*>(rowp + cc);
            __builtin_memcpy(&v[q][0], &x, sizeof(V));
        }
    }
}

// One wavefront per (bucket, column chunk).  A chunk is VPL vectors of VW
// elements per lane, i.e. 64*VW*VPL columns.  The bucket's row indices are
// read 64 at a time (one per lane, with their signs and b values); the rows
// then stream through a ring of D row slots whose indices are broadcast from
// those lanes, so D rows are always in flight.  The ring runs whole rounds
// (slots past the bucket's last row reload that row and are not added), so
// every load is unconditional.  Every accumulation stays in ascending row
// order, sequential per output element (one lane each); a padding slot is
// excluded by a select, never by a zero factor.
template <class TA, int VW, int VPL, int D, int LP>
__global__ __launch_bounds__(256) void k_segsum(Batch b)
{
    constexpr int CW = kWave * VW * VPL;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    for (int64_t t = blockIdx.x * 4 + threadIdx.x / kWave; t < b.T; t += nwaves) {
        const int s = b.nsys == 1 ? 0 : find_sys(b.task_offs, b.nsys, t);
        const SketchSys& S = sys_at(b, s);
        const int64_t lt = t - S.task_off;
        const int64_t j = lt / S.nchunks;
        const int c = static_cast<int>(lt - j * S.nchunks);
        const int n = S.n;
        const int col0 = c * CW;
        const TA* __restrict__ A = static_cast<const TA*>(S.A);
        const int64_t lda = S.lda;
        const uint32_t beg = b.ptr[S.bkt_off + j];
        const uint32_t end = b.ptr[S.bkt_off + j + 1];
        const bool with_b = (S.B != nullptr) && c == 0;

        double acc[VPL][VW];
#pragma unroll
        for (int q = 0; q < VPL; ++q)
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[q][e] = 0.0;
        double bacc = 0.0;

        for (uint32_t base = beg; base < end; base += kWave) {
            const int cnt = static_cast<int>(min((uint32_t)kWave, end - base));
            const uint32_t my_row = lane < cnt ? b.perm[base + lane] : 0u;
            const double my_sg = draw_sign(draw_word(S.seed, my_row));
            const double my_b = (with_b && lane < cnt) ? S.B[(int64_t)my_row * S.ldb] : 0.0;
            const int nround = (cnt + D - 1) / D;
            TA val[D][VPL][VW];
#pragma unroll
            for (int u = 0; u < D; ++u) {
                const uint32_t row = __builtin_amdgcn_readlane(my_row, min(u, cnt - 1));
                load_row_chunk<TA, VW, VPL>(val[u], A + (int64_t)row * lda, col0, lane, n);
            }
            for (int rd = 0; rd < nround; ++rd) {
#pragma unroll
                for (int u = 0; u < D; ++u) {
                    const int qi = rd * D + u;
                    const bool use = qi < cnt;
                    const double sg = __shfl(my_sg, min(qi, kWave - 1), kWave);
#pragma unroll
                    for (int q = 0; q < VPL; ++q)
#pragma unroll
                        for (int e = 0; e < VW; ++e) {
                            const double nv = acc[q][e] + sg * static_cast<double>(val[u][q][e]);
                            acc[q][e] = use ? nv : acc[q][e];
                        }
                    if (with_b) {
                        const double nb = bacc + sg * __shfl(my_b, min(qi, kWave - 1), kWave);
                        bacc = use ? nb : bacc;
                    }
                    const uint32_t row = __builtin_amdgcn_readlane(my_row, min(qi + D, cnt - 1));
                    load_row_chunk<TA, VW, VPL>(val[u], A + (int64_t)row * lda, col0, lane, n);
                }
            }
        }

        double nrm = 0.0;
#pragma unroll
        for (int q = 0; q < VPL; ++q) {
            const int col = col0 + (q * kWave + lane) * VW;
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                if (col + e < n) {
                    nrm += acc[q][e] * acc[q][e];
                    if (S.At64) S.At64[j * S.ldat64 + col + e] = acc[q][e];
                    if constexpr (LP != 0) store_lp<LP>(S.Atlp, j * S.ldatlp + col + e, acc[q][e]);
                } else if (S.zpad) {
                    // the padding lies in the row's last chunk (ld < n + 32)
                    if (S.At64 && col + e < S.ldat64) S.At64[j * S.ldat64 + col + e] = 0.0;
                    if constexpr (LP != 0)
                        if (col + e < S.ldatlp) store_lp<LP>(S.Atlp, j * S.ldatlp + col + e, 0.0);
                }
            }
        }
        nrm = wave_sum(nrm);
        if (lane == 0) {
            if (S.nchunks == 1) {
                if (S.nu2) S.nu2[j] = nrm;
            } else {
                b.nu2part[t] = nrm;
            }
            if (with_b) S.Bt[j * S.ldbt] = bacc;
        }
    }
}

__global__ void k_nu2_finalize(Batch b)
{
    for (int64_t gb = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; gb < b.D;
         gb += (int64_t)gridDim.x * blockDim.x) {
        const int s = b.nsys == 1 ? 0 : find_sys(b.bkt_offs, b.nsys, gb);
        const SketchSys& S = sys_at(b, s);
        if (S.nchunks <= 1 || S.nu2 == nullptr) continue;
        const int64_t j = gb - S.bkt_off;
        double acc = 0.0;
        for (int c = 0; c < S.nchunks; ++c) acc += b.nu2part[S.task_off + j * S.nchunks + c];
        S.nu2[j] = acc;
    }
}


// ---------------------------------------------------------------------------
// CSR input.  One workgroup per bucket: the bucket's stored entries are staged
// in LDS in ascending row order (signed, widened to FP64), wavefront 0 adds
// them row by row into an FP64 accumulator row in LDS (lanes take distinct
// columns of one row, rows follow in order, so each column's sum is
// sequential in the row order), then the whole workgroup writes the dense
// row(s) and reduces the squared norm.  Entries beyond the staging capacity
// are read straight from global memory by the same ordered walk.
// Sparse output (SP): the accumulation also marks the touched columns in an
// LDS bitmap, and instead of the dense row the workgroup writes the touched
// columns, ascending, with their sums at the bucket's offset of the CSR
// result.  Adding only the stored entries to an accumulator that starts at
// +0.0 gives the same bits as the dense sum, where the absent entries add
// signed zeros, so both outputs hold the same values.
// ---------------------------------------------------------------------------
constexpr int kCsrNT = 256;
constexpr int kCsrStage = 1024;   // staged entries per bucket
constexpr int kCsrRows = 256;     // staged rows per bucket
constexpr int kCsrChunk = kCsrNT * 32;  // accumulator columns: one bitmap word per thread

// Where the sparse result goes: ofs is the exclusive scan of the distinct
// column counts of the buckets (d + 1 entries).
struct CsrOut {
    const uint32_t* ofs;
    int64_t* rp;     // d + 1
    int32_t* col;
    double* val;
};

template <int LP, bool SP>
__global__ __launch_bounds__(kCsrNT) void k_segsum_csr(Batch b, const int64_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ colidx,
                                                       const float* __restrict__ val, int chunk, CsrOut so,
                                                       const uint32_t* __restrict__ queue)
{
    extern __shared__ __align__(16) char smem[];
    double* acc = reinterpret_cast<double*>(smem);              // chunk columns
    uint32_t* bm = reinterpret_cast<uint32_t*>(smem + (size_t)chunk * 8);  // SP: touched columns of the chunk
    __shared__ double s_val[kCsrStage];
    __shared__ int32_t s_col[kCsrStage];
    __shared__ int32_t s_rowend[kCsrRows];                      // staged-entry end per row
    __shared__ double s_b[kCsrRows];
    __shared__ uint32_t s_wsum[kCsrNT / kWave];
    __shared__ double s_red[kCsrNT / kWave];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    const SketchSys S = sys_at(b, 0);
    const int n = S.n;
    // queue: null (every bucket), or a count followed by the buckets to do
    const int64_t count = queue ? (int64_t)queue[0] : (int64_t)S.d;
    for (int64_t q = blockIdx.x; q < count; q += gridDim.x) {
        const int64_t j = queue ? (int64_t)queue[1 + q] : q;
        const uint32_t beg = b.ptr[j], end = b.ptr[j + 1];
        const uint32_t len = end - beg;
        // stage: thread t takes row beg+t (first kCsrRows rows)
        const bool staged = len <= (uint32_t)kCsrRows;
        uint32_t mycnt = 0;
        int64_t rs = 0;
        double sg = 0.0;
        uint32_t myrow = 0;
        if (staged && (uint32_t)tid < len) {
            myrow = b.perm[beg + tid];
            sg = draw_sign(draw_word(S.seed, myrow));
            rs = row_ptr[myrow];
            mycnt = (uint32_t)(row_ptr[myrow + 1] - rs);
            s_b[tid] = S.B ? sg * S.B[myrow] : 0.0;
        }
        // block exclusive scan of per-row counts
        uint32_t v = mycnt;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t t = __shfl_up(v, off, kWave);
            if (lane >= off) v += t;
        }
        if (lane == kWave - 1) s_wsum[wid] = v;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kCsrNT / kWave; ++w) {
            if (w < wid) before += s_wsum[w];
            total += s_wsum[w];
        }
        const uint32_t start = before + v - mycnt;
        const bool fits = staged && total <= (uint32_t)kCsrStage;
        if (fits && (uint32_t)tid < len) {
            for (uint32_t e = 0; e < mycnt; ++e) {
                s_col[start + e] = colidx[rs + e];
                s_val[start + e] = sg * static_cast<double>(val[rs + e]);
            }
            s_rowend[tid] = (int32_t)(start + mycnt);
        }
        double nrm = 0.0;
        uint32_t out = 0;  // SP: entries of the bucket written so far
        for (int c0 = 0; c0 < n; c0 += chunk) {
            const int cw = min(chunk, n - c0);
            for (int c = tid; c < cw; c += kCsrNT) acc[c] = 0.0;
            if constexpr (SP) bm[tid] = 0u;
            __syncthreads();
            auto add = [&](int c, double v) {
                acc[c] = acc[c] + v;
                if constexpr (SP) atomicOr(&bm[c >> 5], 1u << (c & 31));
            };
            if (wid == 0) {
                if (fits) {
                    int32_t e0 = 0;
                    for (uint32_t p = 0; p < len; ++p) {
                        const int32_t e1 = s_rowend[p];
                        for (int32_t e = e0 + lane; e < e1; e += kWave) {
                            const int c = s_col[e] - c0;
                            if (c >= 0 && c < cw) add(c, s_val[e]);
                        }
                        e0 = e1;
                    }
                } else {
                    for (uint32_t p = beg; p < end; ++p) {
                        const uint32_t row = b.perm[p];
                        const double sgn = draw_sign(draw_word(S.seed, row));
                        const int64_t e1 = row_ptr[row + 1];
                        for (int64_t e = row_ptr[row] + lane; e < e1; e += kWave) {
                            const int c = colidx[e] - c0;
                            if (c >= 0 && c < cw) add(c, sgn * static_cast<double>(val[e]));
                        }
                    }
                }
            }
            __syncthreads();
            for (int c = tid; c < cw; c += kCsrNT) {
                const double a = acc[c];
                nrm += a * a;
                if constexpr (!SP) {
                    if (S.At64) S.At64[j * S.ldat64 + c0 + c] = a;
                    if constexpr (LP != 0) store_lp<LP>(S.Atlp, j * S.ldatlp + c0 + c, a);
                }
            }
            if constexpr (SP) {
                // thread t owns bitmap word t (columns 32t .. 32t + 31 of the
                // chunk): its marked columns go, ascending, after those of
                // the threads before it
                uint32_t word = bm[tid];
                const uint32_t cnt = __popc(word);
                uint32_t total;
                uint32_t pos = so.ofs[j] + out + block_incl_scan<kCsrNT>(cnt, &total) - cnt;
                while (word) {
                    const int bit = __ffs(word) - 1;
                    word &= word - 1u;
                    const int c = tid * 32 + bit;
                    so.col[pos] = c0 + c;
                    so.val[pos] = acc[c];
                    ++pos;
                }
                out += total;
            }
            __syncthreads();
        }
        if constexpr (SP) {
            if (tid == 0) {
                so.rp[j] = so.ofs[j];
                if (j == S.d - 1) so.rp[S.d] = so.ofs[S.d];
            }
        }
        nrm = wave_sum(nrm);
        if (lane == 0) s_red[wid] = nrm;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < kCsrNT / kWave; ++w) t += s_red[w];
            if (S.nu2) S.nu2[j] = t;
            if (S.Bt) {
                double bacc = 0.0;
                if (staged) {
                    for (uint32_t p = 0; p < len; ++p) bacc = bacc + s_b[p];
                } else {
                    for (uint32_t p = beg; p < end; ++p) {
                        const uint32_t row = b.perm[p];
                        bacc = bacc + draw_sign(draw_word(S.seed, row)) * S.B[row];
                    }
                }
                S.Bt[j] = bacc;
            }
        }
        __syncthreads();
    }
}

// The same sums for the common bucket, without an accumulator row: its
// stored entries (at most kCsrSortCap, from at most kCsrRows rows, with
// n <= kCsrRunsMaxN) are staged in LDS in row order and ranked by
// (column, position), so each column's entries form one run in ascending
// row order; every run is summed sequentially from +0.0 by one thread, all
// runs at once.  A bitmap of the touched columns with per-word prefix counts
// gives any column's run in O(1): the dense output and the squared norm walk
// each thread's columns (c = t, t + 256, ...: the operand order of
// k_segsum_csr, so the bits are the same), and the sparse output is the
// runs themselves.  The LDS loops issue their reads ahead (unrolled, 16-byte
// reads in the ranking), since a serial loop would wait out the LDS latency
// once per step.  About 23 KB of LDS per workgroup, so six workgroups share a
// CU.  A bucket that does not fit is appended to `queue` (count, then bucket
// indices) for k_segsum_csr.
constexpr int kCsrSortCap = 512;
constexpr int kCsrRunsMaxN = 16384;  // columns: bitmap of 512 words

template <int LP, bool SP>
__global__ __launch_bounds__(kCsrNT) void k_segsum_csr_runs(Batch b, const int64_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ colidx,
                                                            const float* __restrict__ val, CsrOut so,
                                                            uint32_t* __restrict__ queue)
{
    // staged entries in row order; after the ranking, the runs (column, sum)
    __shared__ __align__(16) int32_t s_col[kCsrSortCap];
    __shared__ double s_val[kCsrSortCap];
    __shared__ int32_t s_sc[kCsrSortCap];   // entries sorted by (column, position)
    __shared__ double s_sv[kCsrSortCap];
    __shared__ double s_b[kCsrRows];
    __shared__ int64_t s_rs[kCsrRows];      // staged row: first stored entry in the CSR arrays
    __shared__ uint32_t s_st[kCsrRows];     // staged row: first staging slot
    __shared__ double s_sg[kCsrRows];       // staged row: sign
    __shared__ uint32_t s_bm[kCsrRunsMaxN / 32];    // touched columns
    __shared__ uint32_t s_wpre[kCsrRunsMaxN / 32];  // runs before each bitmap word
    __shared__ double s_red[kCsrNT / kWave];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wid = tid / kWave;
    const SketchSys S = sys_at(b, 0);
    const int n = S.n;
    const int nwords = (n + 31) >> 5;
    for (int64_t j = blockIdx.x; j < S.d; j += gridDim.x) {
        const uint32_t beg = b.ptr[j], end = b.ptr[j + 1];
        const uint32_t len = end - beg;
        const bool rows_fit = len <= (uint32_t)kCsrRows && n <= kCsrRunsMaxN;
        uint32_t mycnt = 0;
        int64_t rs = 0;
        double sg = 0.0;
        if (rows_fit && (uint32_t)tid < len) {
            const uint32_t myrow = b.perm[beg + tid];
            sg = draw_sign(draw_word(S.seed, myrow));
            rs = row_ptr[myrow];
            mycnt = (uint32_t)(row_ptr[myrow + 1] - rs);
            s_b[tid] = S.B ? sg * S.B[myrow] : 0.0;
        }
        uint32_t T;
        const uint32_t start = block_incl_scan<kCsrNT>(mycnt, &T) - mycnt;
        if (!rows_fit || T > (uint32_t)kCsrSortCap) {
            if (tid == 0) queue[1 + atomicAdd(&queue[0], 1u)] = static_cast<uint32_t>(j);
            continue;  // uniform: every thread saw the same len and T
        }
        if ((uint32_t)tid < len) {
            s_rs[tid] = rs;
            s_st[tid] = start;
            s_sg[tid] = sg;
        }
        for (int w = tid; w < nwords; w += kCsrNT) s_bm[w] = 0u;
        const uint32_t T4 = (T + 3u) & ~3u;
        if ((uint32_t)tid < T4 - T) s_col[T + tid] = INT32_MAX;  // padding: above every column
        __syncthreads();
        // stage slot p from the row holding it (the last row whose first
        // slot is at most p: rows without entries share their successor's
        // first slot), all of a thread's loads at once
        for (uint32_t p = tid; p < T; p += kCsrNT) {
            uint32_t lo = 0, hi = len - 1;
            while (lo < hi) {
                const uint32_t mid = (lo + hi + 1) >> 1;
                if (s_st[mid] <= p) lo = mid;
                else hi = mid - 1;
            }
            const int64_t e = s_rs[lo] + (p - s_st[lo]);
            s_col[p] = colidx[e];
            s_val[p] = s_sg[lo] * static_cast<double>(val[e]);
        }
        __syncthreads();
        // rank by (column, position): distinct keys, a permutation of [0, T)
        for (uint32_t e = tid; e < T; e += kCsrNT) {
            const int32_t ce = s_col[e];
            uint32_t rank = 0;
            const int4* c4 = reinterpret_cast<const int4*>(s_col);
#pragma unroll 4
            for (uint32_t f = 0; f < T4; f += 4) {
                const int4 v = c4[f >> 2];
                rank += (v.x < ce || (v.x == ce && f < e)) ? 1u : 0u;
                rank += (v.y < ce || (v.y == ce && f + 1 < e)) ? 1u : 0u;
                rank += (v.z < ce || (v.z == ce && f + 2 < e)) ? 1u : 0u;
                rank += (v.w < ce || (v.w == ce && f + 3 < e)) ? 1u : 0u;
            }
            s_sc[rank] = ce;
            s_sv[rank] = s_val[e];
        }
        __syncthreads();
        // runs: thread t looks at sorted positions 2t and 2t + 1 (T <= 512);
        // a run's column and sum go to s_col / s_val at its index
        const uint32_t p0 = 2u * tid, p1 = p0 + 1u;
        const int32_t c0 = p0 < T ? s_sc[p0] : 0;
        const int32_t c1 = p1 < T ? s_sc[p1] : 0;
        const uint32_t f0 = (p0 < T && (p0 == 0 || s_sc[p0 - 1] != c0)) ? 1u : 0u;
        const uint32_t f1 = (p1 < T && c1 != c0) ? 1u : 0u;
        uint32_t nruns;
        const uint32_t r0 = block_incl_scan<kCsrNT>(f0 + f1, &nruns) - (f0 + f1);
        auto run_sum = [&](uint32_t p, int32_t c, uint32_t r) {
            double acc = 0.0;
            for (uint32_t q = p; q < T && s_sc[q] == c; ++q) acc = acc + s_sv[q];
            s_col[r] = c;
            s_val[r] = acc;
            atomicOr(&s_bm[c >> 5], 1u << (c & 31));
        };
        if (f0) run_sum(p0, c0, r0);
        if (f1) run_sum(p1, c1, r0 + f0);
        __syncthreads();
        // runs before each bitmap word (thread t: words 2t and 2t + 1)
        {
            const int w0 = 2 * tid, w1 = w0 + 1;
            const uint32_t n0 = w0 < nwords ? __popc(s_bm[w0]) : 0u;
            const uint32_t n1 = w1 < nwords ? __popc(s_bm[w1]) : 0u;
            uint32_t all;
            const uint32_t before = block_incl_scan<kCsrNT>(n0 + n1, &all) - (n0 + n1);
            if (w0 < nwords) s_wpre[w0] = before;
            if (w1 < nwords) s_wpre[w1] = before + n0;
        }
        __syncthreads();
        double nrm = 0.0;
        double* const At64 = S.At64 ? S.At64 + j * S.ldat64 : nullptr;
        void* const Atlp = LP != 0 ? static_cast<void*>(static_cast<char*>(S.Atlp) + j * S.ldatlp * (LP == CSK_F32 ? 4 : 2)) : nullptr;
        auto column = [&](int c) {
            const uint32_t word = s_bm[c >> 5];
            const uint32_t below = word & ((1u << (c & 31)) - 1u);
            const bool hit = (word >> (c & 31)) & 1u;
            const double a = hit ? s_val[s_wpre[c >> 5] + __popc(below)] : 0.0;
            nrm += a * a;
            if constexpr (!SP) {
                if (At64) At64[c] = a;
                if constexpr (LP != 0) store_lp<LP>(Atlp, c, a);
            }
        };
        // whole rounds of 256 columns without a bound check, then the tail
        const int full = n / kCsrNT;
#pragma unroll 4
        for (int k = 0; k < full; ++k) column(k * kCsrNT + tid);
        if (full * kCsrNT + tid < n) column(full * kCsrNT + tid);
        if constexpr (SP) {
            const uint32_t o = so.ofs[j];
            for (uint32_t r = tid; r < nruns; r += kCsrNT) {
                so.col[o + r] = s_col[r];
                so.val[o + r] = s_val[r];
            }
            if (tid == 0) {
                so.rp[j] = so.ofs[j];
                if (j == S.d - 1) so.rp[S.d] = so.ofs[S.d];
            }
        }
        nrm = wave_sum(nrm);
        if (lane == 0) s_red[wid] = nrm;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int w = 0; w < kCsrNT / kWave; ++w) t += s_red[w];
            if (S.nu2) S.nu2[j] = t;
            if (S.Bt) {
                double bacc = 0.0;
#pragma unroll 8
                for (uint32_t p = 0; p < len; ++p) bacc = bacc + s_b[p];
                S.Bt[j] = bacc;
            }
        }
        __syncthreads();
    }
}

// Distinct stored columns per bucket, the row lengths of the sparse sketch.
// One wavefront per bucket; each lane takes whole rows of the bucket and
// marks their columns in the wavefront's LDS bitmap, counting the marks that
// were new (the LDS atomic returns the old word, so a column shared by rows
// on different lanes is counted once).  The marked words are cleared by the
// same walk afterwards, ready for the next bucket.
constexpr int kDistinctWaves = 4;

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__global__ __launch_bounds__(kDistinctWaves * kWave) void k_csr_distinct(Batch b, const int64_t* __restrict__ row_ptr,
                                                                      const int32_t* __restrict__ colidx,
                                                                      int nwords, uint32_t* __restrict__ cnt)
{
    extern __shared__ uint32_t bm_all[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    uint32_t* bm = bm_all + (size_t)wid * nwords;
    for (int w = lane; w < nwords; w += kWave) bm[w] = 0u;
    for (int64_t j = (int64_t)blockIdx.x * kDistinctWaves + wid; j < b.D;
         j += (int64_t)gridDim.x * kDistinctWaves) {
        const uint32_t beg = b.ptr[j], end = b.ptr[j + 1];
        uint32_t fresh = 0;
        for (uint32_t p = beg + lane; p < end; p += kWave) {
            const uint32_t row = b.perm[p];
            const int64_t e1 = row_ptr[row + 1];
            for (int64_t e = row_ptr[row]; e < e1; ++e) {
                const uint32_t c = static_cast<uint32_t>(colidx[e]);
                const uint32_t bit = 1u << (c & 31u);
                fresh += (atomicOr(&bm[c >> 5], bit) & bit) ? 0u : 1u;
            }
        }
        fresh = wave_sum_u32(fresh);
        if (lane == 0) cnt[j] = fresh;
        for (uint32_t p = beg + lane; p < end; p += kWave) {
            const uint32_t row = b.perm[p];
            const int64_t e1 = row_ptr[row + 1];
            for (int64_t e = row_ptr[row]; e < e1; ++e) bm[static_cast<uint32_t>(colidx[e]) >> 5] = 0u;
        }
    }
}

// Descriptors travel to the device as kernel arguments, 8 at a time, so the
// call needs no host staging buffer and stays capturable.
struct DescPack {
    SketchSys s[24];
};

__global__ void k_store_descs(DescPack pack, int count, SketchSys* dst)
{
    if (threadIdx.x < count) dst[threadIdx.x] = pack.s[threadIdx.x];
}

struct OffPack {
    int64_t v[400];
};

__global__ void k_store_offs(OffPack pack, int count, int64_t* dst)
{
    for (int k = threadIdx.x; k < count; k += blockDim.x) dst[k] = pack.v[k];
}

int grid_for(int64_t items, int per_block, int cap)
{
    int64_t g = (items + per_block - 1) / per_block;
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(g, cap)));
}

// Column-chunk geometry: VW elements per vector (16 bytes), VPL vectors per
// lane.  For FP64 input a chunk covers 128*VPL columns, for FP32 256*VPL.
struct Geometry {
    int vw, vpl;
};

Geometry pick_geometry(int64_t n_max, csk_dtype a_dtype, bool vec_ok)
{
    const int vw = vec_ok ? (a_dtype == CSK_F64 ? 2 : 4) : 1;
    const int64_t per_vpl = (int64_t)kWave * vw;
    // up to 8 vectors per lane: a row of up to 1024 FP64 (2048 FP32) columns
    // is one chunk, so the squared norm needs no second pass
    int vpl = static_cast<int>(std::min<int64_t>(8, (n_max + per_vpl - 1) / per_vpl));
    if (vpl == 3) vpl = 4;
    if (vpl > 4) vpl = 8;
    return {vw, std::max(1, vpl)};
}

template <class TA, int VW, int VPL, int LP>
void launch_segsum_lp(const Batch& b, hipStream_t st)
{
    constexpr int D = VPL >= 8 ? 2 : VPL >= 4 ? 4 : 8;  // rows in flight per wavefront (16 KB of FP64)
    k_segsum<TA, VW, VPL, D, LP><<<grid_for(b.T, 4, 1 << 20), 256, 0, st>>>(b);
}

template <class TA, int VW, int VPL>
void launch_segsum_vpl(const Batch& b, csk_dtype lp, hipStream_t st)
{
    switch (lp) {
    case CSK_F32: launch_segsum_lp<TA, VW, VPL, CSK_F32>(b, st); break;
    case CSK_F16: launch_segsum_lp<TA, VW, VPL, CSK_F16>(b, st); break;
    case CSK_BF16: launch_segsum_lp<TA, VW, VPL, CSK_BF16>(b, st); break;
    default: launch_segsum_lp<TA, VW, VPL, 0>(b, st); break;
    }
}

template <class TA, int VW>
void launch_segsum_vw(const Batch& b, int vpl, csk_dtype lp, hipStream_t st)
{
    switch (vpl) {
    case 1: launch_segsum_vpl<TA, VW, 1>(b, lp, st); break;
    case 2: launch_segsum_vpl<TA, VW, 2>(b, lp, st); break;
    case 4: launch_segsum_vpl<TA, VW, 4>(b, lp, st); break;
    default: launch_segsum_vpl<TA, VW, 8>(b, lp, st); break;
    }
}

void launch_segsum(const Batch& b, csk_dtype a_dtype, Geometry g, csk_dtype lp, hipStream_t st)
{
    if (a_dtype == CSK_F64) {
        if (g.vw == 2) launch_segsum_vw<double, 2>(b, g.vpl, lp, st);
        else launch_segsum_vw<double, 1>(b, g.vpl, lp, st);
    } else {
        if (g.vw == 4) launch_segsum_vw<float, 4>(b, g.vpl, lp, st);
        else launch_segsum_vw<float, 1>(b, g.vpl, lp, st);
    }
}

// ptr[0 .. D] = exclusive scan of cnt[0 .. D) (ptr[D] = total): one block for
// few counts, else per-tile sums, a scan of those, and the tiles' scans.
csk_status exclusive_scan(const uint32_t* cnt, int64_t D, uint32_t* part, uint32_t* ptr, hipStream_t st)
{
    if (D <= kScanSingleMax) {
        const size_t shm = (size_t)D * sizeof(uint32_t);
        if (shm > (size_t)48 * 1024)
            CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_scan_single),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
        k_scan_single<<<1, 1024, shm, st>>>(cnt, D, ptr);
        CSK_LAUNCH_CHECK("k_scan_single");
        return CSK_OK;
    }
    const int nb_scan = static_cast<int>((D + kScanTile - 1) / kScanTile);
    k_scan_reduce<<<nb_scan, 256, 0, st>>>(cnt, D, part);
    CSK_LAUNCH_CHECK("k_scan_reduce");
    k_scan_top<<<1, 1024, 0, st>>>(part, nb_scan, ptr, D);
    CSK_LAUNCH_CHECK("k_scan_top");
    k_scan_apply<<<nb_scan, 256, 0, st>>>(cnt, D, part, ptr);
    CSK_LAUNCH_CHECK("k_scan_apply");
    return CSK_OK;
}

// Hash, count, scan, scatter and sort: afterwards perm[ptr[gb] .. ptr[gb+1])
// lists the rows of global bucket gb in ascending order.
csk_status group_rows(const Batch& b, hipStream_t st)
{
    const int64_t M = b.M, D = b.D;
    k_fill_u32<<<grid_for(D, 256, 4096), 256, 0, st>>>(b.cnt, D, 0u);
    CSK_LAUNCH_CHECK("k_fill_u32");
    // one system with few buckets: block-aggregated counters (at most 64
    // blocks of at least 8192 rows each)
    const bool lds = b.nsys == 1 && D <= kHistCap;
    const int64_t hblocks = std::max<int64_t>(1, std::min<int64_t>(64, (M + 8191) / 8192));
    const int64_t hrows = (M + hblocks - 1) / hblocks;
    const size_t hshm = (size_t)D * sizeof(uint32_t);
    if (lds && hshm > (size_t)48 * 1024) {
        CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_hash_hist_lds),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)hshm));
        CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_scatter_lds),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)hshm));
    }
    if (lds) k_hash_hist_lds<<<(int)hblocks, kHistNT, hshm, st>>>(b, hrows);
    else k_hash_hist<<<grid_for(M, 256, 16384), 256, 0, st>>>(b);
    CSK_LAUNCH_CHECK("k_hash_hist");
    csk_status r = exclusive_scan(b.cnt, D, b.scan_part, b.ptr, st);
    if (r != CSK_OK) return r;
    if (lds) k_scatter_lds<<<(int)hblocks, kHistNT, hshm, st>>>(b, hrows);
    else k_scatter<<<grid_for(M, 256, 16384), 256, 0, st>>>(b);
    CSK_LAUNCH_CHECK("k_scatter");
    k_sort_segments<<<grid_for(D, 4, 8192), 256, 0, st>>>(b);
    CSK_LAUNCH_CHECK("k_sort_segments");
    k_long_segments<<<grid_for(D, 1, 1024), 256, 0, st>>>(b);
    CSK_LAUNCH_CHECK("k_long_segments");
    return CSK_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

int64_t sketch_chunks(int64_t n, csk_dtype a_dtype)
{
    (void)a_dtype;
    // Upper bound used for workspace sizing: the smallest chunk is 64 columns.
    return (n + kWave - 1) / kWave;
}

size_t sketch_ws_bytes(int64_t M, int64_t D, int64_t T, int32_t nsys)
{
    Carve c(nullptr);
    c.take<SketchSys>(nsys);
    c.take<SketchSys>(nsys);
    c.take<int64_t>(nsys + 1);
    c.take<int64_t>(nsys + 1);
    c.take<int64_t>(nsys + 1);
    c.take<int64_t>(nsys + 1);
    c.take<uint32_t>(D);
    c.take<uint32_t>(D + 1);
    c.take<uint32_t>(M);
    c.take<double>(T);
    c.take<uint32_t>(D / kScanTile + 2);
    return c.bytes();
}

static csk_status upload_descs(const std::vector<SketchSys>& h, SketchSys* d, hipStream_t st)
{
    for (size_t k = 0; k < h.size(); k += 24) {
        DescPack pack;
        const int cnt = static_cast<int>(std::min<size_t>(24, h.size() - k));
        for (int q = 0; q < cnt; ++q) pack.s[q] = h[k + q];
        k_store_descs<<<1, 64, 0, st>>>(pack, cnt, d + k);
        CSK_LAUNCH_CHECK("k_store_descs");
    }
    return CSK_OK;
}

static csk_status upload_offs(const std::vector<int64_t>& h, int64_t* d, hipStream_t st)
{
    for (size_t k = 0; k < h.size(); k += 400) {
        OffPack pack;
        const int cnt = static_cast<int>(std::min<size_t>(400, h.size() - k));
        for (int q = 0; q < cnt; ++q) pack.v[q] = h[k + q];
        k_store_offs<<<1, 64, 0, st>>>(pack, cnt, d + k);
        CSK_LAUNCH_CHECK("k_store_offs");
    }
    return CSK_OK;
}

csk_status sketch_run(const SketchJob* jobs, int32_t nsys, csk_dtype a_dtype, csk_dtype lp_dtype,
                      uint32_t* perm_out, uint32_t* ptr_out, void* ws, size_t ws_bytes, hipStream_t st)
{
    // Geometry shared by the batch: vector loads only when every system's
    // rows are 16-byte aligned.
    int64_t n_max = 0, nrhs_max = 0;
    bool vec_ok = true, vec_ok_b = true;
    const size_t esz = dtype_size(a_dtype);
    for (int s = 0; s < nsys; ++s) {
        const SketchJob& J = jobs[s];
        n_max = std::max(n_max, J.n);
        const int vw = (a_dtype == CSK_F64) ? 2 : 4;
        (void)vw;
        if (!aligned16(J.A) || (J.lda * esz) % 16 != 0) vec_ok = false;
        if (J.B && J.nrhs > 1) {
            nrhs_max = std::max(nrhs_max, J.nrhs);
            if (!aligned16(J.B) || (J.ldb * 8) % 16 != 0) vec_ok_b = false;
        }
    }
    const Geometry g = pick_geometry(n_max, a_dtype, vec_ok);
    const int64_t cw = (int64_t)kWave * g.vw * g.vpl;

    std::vector<SketchSys> hs(nsys);
    std::vector<int64_t> row_offs(nsys + 1), bkt_offs(nsys + 1), task_offs(nsys + 1);
    int64_t M = 0, D = 0, T = 0;
    for (int s = 0; s < nsys; ++s) {
        const SketchJob& J = jobs[s];
        SketchSys& S = hs[s];
        S.A = J.A;
        S.B = (J.B && J.nrhs == 1) ? J.B : nullptr;
        S.At64 = J.At64;
        S.Atlp = J.Atlp;
        S.Bt = J.Bt;
        S.nu2 = J.nu2;
        S.lda = J.lda;
        S.ldb = J.ldb;
        S.ldat64 = J.ldat64;
        S.ldatlp = J.ldatlp;
        S.ldbt = J.ldbt;
        S.m = J.m;
        S.seed = J.seed;
        S.n = static_cast<int32_t>(J.n);
        S.d = static_cast<int32_t>(J.d);
        S.nrhs = static_cast<int32_t>(J.nrhs);
        S.nchunks = static_cast<int32_t>((J.n + cw - 1) / cw);
        S.zpad = J.zpad;
        S.row_off = M;
        S.bkt_off = D;
        S.task_off = T;
        row_offs[s] = M;
        bkt_offs[s] = D;
        task_offs[s] = T;
        M += J.m;
        D += J.d;
        T += J.d * S.nchunks;
    }
    row_offs[nsys] = M;
    bkt_offs[nsys] = D;
    task_offs[nsys] = T;
    if (M >= (int64_t)UINT32_MAX) {
        set_error("total rows %lld exceed the 32-bit row index", (long long)M);
        return CSK_ERR_UNSUPPORTED;
    }

    Carve c(ws);
    Batch b{};
    SketchSys* d_sys = c.take<SketchSys>(nsys);
    SketchSys* d_sys_b = c.take<SketchSys>(nsys);
    int64_t* d_row = c.take<int64_t>(nsys + 1);
    int64_t* d_bkt = c.take<int64_t>(nsys + 1);
    int64_t* d_task = c.take<int64_t>(nsys + 1);
    int64_t* d_task_b = c.take<int64_t>(nsys + 1);
    b.cnt = c.take<uint32_t>(D);
    b.ptr = c.take<uint32_t>(D + 1);
    b.perm = c.take<uint32_t>(M);
    b.nu2part = c.take<double>(T);
    b.scan_part = c.take<uint32_t>(D / kScanTile + 2);
    if (c.bytes() > ws_bytes) {
        set_error("sketch workspace too small: need %zu bytes, got %zu", c.bytes(), ws_bytes);
        return CSK_ERR_WORKSPACE;
    }
    b.sys = d_sys;
    b.row_offs = d_row;
    b.bkt_offs = d_bkt;
    b.task_offs = d_task;
    b.M = M;
    b.D = D;
    b.T = T;
    b.nsys = nsys;

    csk_status r;
    if (nsys == 1) b.one = hs[0];
    else if ((r = upload_descs(hs, d_sys, st)) != CSK_OK) return r;
    if (nsys > 1) {
        if ((r = upload_offs(row_offs, d_row, st)) != CSK_OK) return r;
        if ((r = upload_offs(bkt_offs, d_bkt, st)) != CSK_OK) return r;
        if ((r = upload_offs(task_offs, d_task, st)) != CSK_OK) return r;
    }

    if ((r = group_rows(b, st)) != CSK_OK) return r;
    launch_segsum(b, a_dtype, g, lp_dtype, st);
    CSK_LAUNCH_CHECK("k_segsum");
    if (T > D) {
        k_nu2_finalize<<<grid_for(D, 256, 4096), 256, 0, st>>>(b);
        CSK_LAUNCH_CHECK("k_nu2_finalize");
    }

    // Multi-column right-hand sides: the same segmented sum over B.
    if (nrhs_max > 1) {
        const Geometry gb = pick_geometry(nrhs_max, CSK_F64, vec_ok_b);
        const int64_t cwb = (int64_t)kWave * gb.vw * gb.vpl;
        std::vector<SketchSys> hb(nsys);
        std::vector<int64_t> toffs(nsys + 1);
        int64_t TB = 0;
        for (int s = 0; s < nsys; ++s) {
            const SketchJob& J = jobs[s];
            SketchSys S = hs[s];
            S.A = J.B;
            S.lda = J.ldb;
            S.n = static_cast<int32_t>(J.B && J.nrhs > 1 ? J.nrhs : 0);
            S.B = nullptr;
            S.At64 = (J.B && J.nrhs > 1) ? J.Bt : nullptr;
            S.ldat64 = J.ldbt;
            S.Atlp = nullptr;
            S.nu2 = nullptr;
            S.nchunks = static_cast<int32_t>(std::max<int64_t>(1, (S.n + cwb - 1) / cwb));
            S.task_off = TB;
            toffs[s] = TB;
            TB += J.d * S.nchunks;
            hb[s] = S;
        }
        toffs[nsys] = TB;
        if (TB > T) {
            set_error("internal: right-hand-side task space exceeds workspace");
            return CSK_ERR_UNSUPPORTED;
        }
        Batch bb = b;
        if (nsys == 1) bb.one = hb[0];
        else if ((r = upload_descs(hb, d_sys_b, st)) != CSK_OK) return r;
        if (nsys > 1 && (r = upload_offs(toffs, d_task_b, st)) != CSK_OK) return r;
        bb.sys = d_sys_b;
        bb.task_offs = d_task_b;
        bb.T = TB;
        launch_segsum(bb, CSK_F64, gb, (csk_dtype)0, st);
        CSK_LAUNCH_CHECK("k_segsum(B)");
    }

    if (perm_out) CSK_HIP(hipMemcpyAsync(perm_out, b.perm, sizeof(uint32_t) * M, hipMemcpyDeviceToDevice, st));
    if (ptr_out) CSK_HIP(hipMemcpyAsync(ptr_out, b.ptr, sizeof(uint32_t) * (D + 1), hipMemcpyDeviceToDevice, st));
    return CSK_OK;
}

namespace {

// Bucket grouping of a CSR sketch; scratch carved from ws (the layout that
// sketch_csr_ws_bytes sizes).  ofs (d + 1) only for the sparse output.
csk_status csr_setup(const double* b, double* bt, double* nu2, int64_t m, int64_t n, int64_t d, uint64_t seed,
                     double* At64, int64_t ldat64, void* At_lp, int64_t ldat_lp, void* ws, size_t ws_bytes,
                     bool sparse, Batch& bt_, uint32_t** queue, uint32_t** ofs, hipStream_t st)
{
    std::vector<SketchSys> hs(1);
    SketchSys& S = hs[0];
    S = SketchSys{};
    S.B = b;
    S.At64 = At64;
    S.Atlp = At_lp;
    S.Bt = bt;
    S.nu2 = nu2;
    S.ldat64 = ldat64;
    S.ldatlp = ldat_lp;
    S.m = m;
    S.seed = seed;
    S.n = static_cast<int32_t>(n);
    S.d = static_cast<int32_t>(d);
    S.nrhs = 1;
    S.nchunks = 1;
    Carve c(ws);
    bt_ = Batch{};
    SketchSys* d_sys = c.take<SketchSys>(1);
    c.take<SketchSys>(1);
    c.take<int64_t>(2);
    c.take<int64_t>(2);
    c.take<int64_t>(2);
    c.take<int64_t>(2);
    bt_.cnt = c.take<uint32_t>(d);
    bt_.ptr = c.take<uint32_t>(d + 1);
    bt_.perm = c.take<uint32_t>(m);
    bt_.nu2part = c.take<double>(d);
    bt_.scan_part = c.take<uint32_t>(d / kScanTile + 2);
    *queue = c.take<uint32_t>(d + 1);
    if (sparse) *ofs = c.take<uint32_t>(d + 1);
    if (c.bytes() > ws_bytes) {
        set_error("sketch workspace too small: need %zu bytes, got %zu", c.bytes(), ws_bytes);
        return CSK_ERR_WORKSPACE;
    }
    bt_.sys = d_sys;
    bt_.M = m;
    bt_.D = d;
    bt_.T = d;
    bt_.nsys = 1;
    bt_.one = hs[0];
    return group_rows(bt_, st);
}

// Every bucket goes to k_segsum_csr_runs; the few that do not fit its
// staging (queue: count, then bucket indices; d + 1 words) follow through
// k_segsum_csr, whose grid loops over the queue's count.
template <int LP, bool SP>
csk_status launch_segsum_csr(const Batch& b, const int64_t* row_ptr, const int32_t* col, const float* val, int64_t n,
                             int64_t d, const CsrOut& so, uint32_t* queue, hipStream_t st)
{
    k_fill_u32<<<1, 64, 0, st>>>(queue, 1, 0u);
    CSK_LAUNCH_CHECK("k_fill_u32");
    k_segsum_csr_runs<LP, SP><<<grid_for(d, 1, 1 << 20), kCsrNT, 0, st>>>(b, row_ptr, col, val, so, queue);
    CSK_LAUNCH_CHECK("k_segsum_csr_runs");
    // accumulator chunk: up to 8192 columns (64 KB of LDS), plus its bitmap
    const int chunk = static_cast<int>(std::min<int64_t>(n, kCsrChunk));
    const size_t shm = (size_t)chunk * 8 + (SP ? kCsrNT * 4 : 0);
    const int grid = grid_for(d, 1, 1024);
    CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_segsum_csr<LP, SP>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    k_segsum_csr<LP, SP><<<grid, kCsrNT, shm, st>>>(b, row_ptr, col, val, chunk, so, queue);
    CSK_LAUNCH_CHECK("k_segsum_csr");
    return CSK_OK;
}

}  // namespace

size_t group_ws_bytes(int64_t m, int64_t d) { return sketch_csr_ws_bytes(m, d, false); }

csk_status group_only(int64_t m, int64_t d, uint64_t seed, void* ws, size_t ws_bytes, const uint32_t** perm,
                      const uint32_t** ptr, hipStream_t st)
{
    Batch bt_;
    uint32_t* queue = nullptr;
    const csk_status r = csr_setup(nullptr, nullptr, nullptr, m, 1, d, seed, nullptr, 0, nullptr, 0, ws, ws_bytes,
                                   false, bt_, &queue, nullptr, st);
    if (r != CSK_OK) return r;
    *perm = bt_.perm;
    *ptr = bt_.ptr;
    return CSK_OK;
}

size_t sketch_csr_ws_bytes(int64_t m, int64_t d, bool sparse)
{
    return sketch_ws_bytes(m, d, d, 1) + (size_t)(d + 1) * 4 + 256 + (sparse ? (size_t)(d + 1) * 4 + 256 : 0);
}

csk_status sketch_csr_run(const int64_t* row_ptr, const int32_t* col, const float* val, int64_t m, int64_t n,
                          int64_t nnz, const double* b, int64_t d, uint64_t seed, double* At64, int64_t ldat64,
                          void* At_lp, csk_dtype lp_dtype, int64_t ldat_lp, double* bt, double* nu2,
                          void* ws, size_t ws_bytes, hipStream_t st)
{
    (void)nnz;
    Batch bt_;
    uint32_t* queue = nullptr;
    csk_status r = csr_setup(b, bt, nu2, m, n, d, seed, At64, ldat64, At_lp, ldat_lp, ws, ws_bytes, false, bt_,
                             &queue, nullptr, st);
    if (r != CSK_OK) return r;
    const CsrOut none{};
    switch (lp_dtype) {
    case CSK_F32: return launch_segsum_csr<CSK_F32, false>(bt_, row_ptr, col, val, n, d, none, queue, st);
    case CSK_F16: return launch_segsum_csr<CSK_F16, false>(bt_, row_ptr, col, val, n, d, none, queue, st);
    case CSK_BF16: return launch_segsum_csr<CSK_BF16, false>(bt_, row_ptr, col, val, n, d, none, queue, st);
    default: return launch_segsum_csr<0, false>(bt_, row_ptr, col, val, n, d, none, queue, st);
    }
}

csk_status sketch_csr_sparse_run(const int64_t* row_ptr, const int32_t* col, const float* val, int64_t m,
                                 int64_t n, const double* b, int64_t d, uint64_t seed, int64_t* at_rp,
                                 int32_t* at_col, double* at_val, double* bt, double* nu2, void* ws, size_t ws_bytes,
                                 hipStream_t st)
{
    Batch bt_;
    uint32_t* ofs = nullptr;
    uint32_t* queue = nullptr;
    csk_status r = csr_setup(b, bt, nu2, m, n, d, seed, nullptr, 0, nullptr, 0, ws, ws_bytes, true, bt_, &queue, &ofs,
                             st);
    if (r != CSK_OK) return r;
    // distinct columns per bucket (into cnt, which the grouping left zero),
    // then their exclusive scan: each bucket's offset in the result
    const int nwords = static_cast<int>((n + 31) / 32);
    const size_t shm = (size_t)kDistinctWaves * nwords * 4;
    CSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_csr_distinct),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    k_csr_distinct<<<grid_for(d, kDistinctWaves, 1 << 16), kDistinctWaves * kWave, shm, st>>>(bt_, row_ptr, col,
                                                                                             nwords, bt_.cnt);
    CSK_LAUNCH_CHECK("k_csr_distinct");
    if ((r = exclusive_scan(bt_.cnt, d, bt_.scan_part, ofs, st)) != CSK_OK) return r;
    const CsrOut so{ofs, at_rp, at_col, at_val};
    return launch_segsum_csr<0, true>(bt_, row_ptr, col, val, n, d, so, queue, st);
}

}  // namespace csk
