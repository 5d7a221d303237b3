// solve_rk.hip -- randomized Kaczmarz (Strohmer & Vershynin), the simplest
// member of the row-selection family that the introduction places
// Algorithm 1's loop in: each iteration draws row i with probability
// ||At^(i)||^2 / ||At||_F^2, independently of x, and projects onto it.  Only
// the drawn row's residual is formed, so an iteration reads one row.
//
// One workgroup runs the whole loop (one row per iteration leaves nothing to
// spread over the chip; the cost is latency), a single wavefront for rows of
// up to 1024 columns, so an iteration needs no barrier between waves:
//   * setup (kernels of their own): the cumulative squared norms C_i into
//     the workspace, by block sums, their prefix and block-local scans (the
//     rounding differs from one running sum in index order only by where
//     the partial sums meet);
//   * the draws do not depend on x, so the rows of 512 iterations are found
//     at once, one binary search per thread for the smallest i with
//     C_i > u_k C_{d-1} (u_k the k-th uniform of the selection stream), and
//     kept in LDS a batch ahead;
//   * each thread owns columns tid + NT j of x, x_ref and the rows
//     (registers), so an iteration is one workgroup reduction (the row's dot
//     product with x_k and ||x_k - x_ref||^2), the stop test on x_k, and the
//     update of the thread's own columns.  Rows are loaded up to four
//     iterations ahead (a ring of registers), which hides the latency of a
//     row read from HBM behind the iterations before it.
#include "csk_grid.h"
#include "csk_solve.h"

#include <algorithm>
#include <cmath>

namespace csk {
namespace {

constexpr int kRkNT = 512;          // threads of the setup, and of the loop for wide rows
constexpr int kRkBatch = 512;       // iterations whose rows are drawn together
// Iterations between a row's load and its use: 4, fewer where the ring
// would not fit the registers (columns per thread J of 8 and 16).
template <int J> constexpr int rk_ahead() { return J >= 16 ? 1 : J >= 8 ? 2 : 4; }

struct RkArgs {
    const double* At;
    const double* bt;
    const double* nu2;
    const double* x0;
    const double* xref;
    double* x;
    double* cum;  // d, workspace
    csk_solve_result* res;
    const volatile int32_t* cancel;
    int64_t ldat;
    int64_t maxit;
    uint64_t seed;
    double tol2;
    int64_t* trace;  // nullable: row projected at each iteration
    int32_t d, n;
    int32_t check_every;
};

// Smallest i with cum[i] > t (cum[d-1] > t when the distribution is valid;
// otherwise the result is d - 1, never used), for K draws at once: the
// searches run in lockstep with unconditional loads (mid = lo once a search
// has ended), so their loads overlap.  Where two segments of the prefix sum
// meet, cum may step back by a few units in the last place; a draw landing
// in such a sliver could reach a row of zero norm, which is then replaced by
// the nearest row of nonzero norm before it (or after it).
template <int K>
__device__ __forceinline__ void rk_search(const double* __restrict__ cum, const double* __restrict__ nu2, int d,
                                          const double (&t)[K], int (&out)[K])
{
    int lo[K], hi[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        lo[k] = 0;
        hi[k] = d - 1;
    }
    // each round halves every open interval: bit length of d rounds suffice
    for (int span = d; span > 0; span >>= 1) {
        double c[K];
        int mid[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            mid[k] = lo[k] + ((hi[k] - lo[k]) >> 1);
            c[k] = cum[mid[k]];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (lo[k] < hi[k]) {
                if (c[k] > t[k]) hi[k] = mid[k];
                else lo[k] = mid[k] + 1;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int i = lo[k];
        if (!(nu2[i] > 0.0)) {
            while (i > 0 && !(nu2[i] > 0.0)) --i;
            if (!(nu2[i] > 0.0))
                for (i = lo[k]; i + 1 < d && !(nu2[i] > 0.0);) ++i;
        }
        out[k] = i;
    }
}

// C_i for i < d into P.cum, over kRkScanBlocks blocks of 256 threads: the
// blocks' sums (coalesced), their exclusive prefix (one thread, in order),
// then each block scans its range 256 elements at a time (wave scans, then
// the four wave totals) from its offset.
constexpr int kRkScanBlocks = 256;
constexpr int kRkScanNT = 256;

__device__ __forceinline__ double rk_block_sum(double v, double* wred)
{
    v = group_sum_t<double, kWave>(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) wred[w] = v;
    __syncthreads();
    const double t = ((wred[0] + wred[1]) + wred[2]) + wred[3];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(kRkScanNT) void k_rk_blocksum(RkArgs P, double* bsum)
{
    __shared__ double wred[kRkScanNT / kWave];
    const int64_t span = (P.d + kRkScanBlocks - 1) / kRkScanBlocks;
    const int64_t lo = min<int64_t>(P.d, blockIdx.x * span), hi = min<int64_t>(P.d, lo + span);
    double v = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kRkScanNT) v += P.nu2[i];
    const double t = rk_block_sum(v, wred);
    if (threadIdx.x == 0) bsum[blockIdx.x] = t;
}

__global__ void k_rk_blockoff(double* bsum)
{
    if (threadIdx.x == 0) {
        double run = 0.0;
        for (int b = 0; b < kRkScanBlocks; ++b) {
            const double v = bsum[b];
            bsum[b] = run;
            run += v;
        }
    }
}

__global__ __launch_bounds__(kRkScanNT) void k_rk_prefix(RkArgs P, const double* boff)
{
    __shared__ double wtot[kRkScanNT / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int64_t span = (P.d + kRkScanBlocks - 1) / kRkScanBlocks;
    const int64_t lo = min<int64_t>(P.d, blockIdx.x * span), hi = min<int64_t>(P.d, lo + span);
    double carry = boff[blockIdx.x];
    for (int64_t base = lo; base < hi; base += kRkScanNT) {
        const int64_t i = base + threadIdx.x;
        const double v = i < hi ? P.nu2[i] : 0.0;
        double x = v;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const double t = __shfl_up(x, off, kWave);
            if (lane >= off) x += t;
        }
        if (lane == kWave - 1) wtot[w] = x;
        __syncthreads();
        double before = carry;
        for (int k = 0; k < w; ++k) before += wtot[k];
        if (i < hi) P.cum[i] = before + x;
        // the same additions as the chunk's last element, so the next chunk
        // starts exactly where this one ended
        carry = (((carry + wtot[0]) + wtot[1]) + wtot[2]) + wtot[3];
        __syncthreads();
    }
}

// NT threads (64: one wavefront; or 512), J columns per thread.
template <int NT, int J>
__global__ __launch_bounds__(NT) void k_solve_rk(RkArgs P)
{
    constexpr int NW = NT / kWave;
    __shared__ int32_t pick[2][kRkBatch];
    __shared__ double red[2][NW][2];
    __shared__ int32_t s_cancel[2];
    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int lane = tid & (kWave - 1);
    const int d = P.d, n = P.n;

    const double total = P.cum[d - 1];  // the last running sum, as the search sees it
    const bool valid = isfinite(total) && total > 0.0;

    // this thread's draws of a batch: iterations b * kRkBatch + tid + NT q
    constexpr int KD = kRkBatch / NT;
    auto draw_batch = [&](int64_t b) {
        double t[KD];
        int r[KD];
#pragma unroll
        for (int q = 0; q < KD; ++q)
            t[q] = select_uniform(P.seed, static_cast<uint64_t>(b * kRkBatch + tid + NT * q)) * total;
        if (valid) rk_search<KD>(P.cum, P.nu2, d, t, r);
#pragma unroll
        for (int q = 0; q < KD; ++q) pick[b & 1][tid + NT * q] = valid ? r[q] : 0;
    };
    draw_batch(0);
    draw_batch(1);

    double x[J], xr[J];
    for (int j = 0; j < J; ++j) {
        const int c = tid + j * NT;
        x[j] = (c < n && P.x0) ? P.x0[c] : 0.0;
        xr[j] = c < n ? P.xref[c] : 0.0;
    }
    double q = 0.0;
    for (int j = 0; j < J; ++j) q += xr[j] * xr[j];
    q = group_sum_t<double, kWave>(q);
    if (lane == 0) red[1][wave][0] = q;
    __syncthreads();
    double xref2 = 0.0;
    for (int w = 0; w < NW; ++w) xref2 += red[1][w][0];

    auto load_row = [&](int i, double (&v)[J], double& bi, double& ni, int& ii) {
        ii = i;
        const double* __restrict__ row = P.At + (int64_t)i * P.ldat;
        for (int j = 0; j < J; ++j) {
            const int c = tid + j * NT;
            v[j] = c < n ? row[c] : 0.0;
        }
        bi = P.bt[i];
        ni = P.nu2[i];
    };
    // ring slot u holds the row of every iteration k with k % AH == u
    constexpr int AH = rk_ahead<J>();
    double ring[AH][J], rb[AH], rn[AH];
    int ri[AH];  // the row index of each slot
#pragma unroll
    for (int u = 0; u < AH; ++u) {
        if (u <= P.maxit) load_row(pick[0][u], ring[u], rb[u], rn[u], ri[u]);
        else {
            for (int j = 0; j < J; ++j) ring[u][j] = 0.0;
            rb[u] = rn[u] = 0.0;
            ri[u] = 0;
        }
    }

    int32_t status = CSK_NOT_CONVERGED;
    double meas = NAN;
    int64_t k = 0;
    bool done = false;
    while (!done) {
#pragma unroll
        for (int u = 0; u < AH; ++u) {
            const int par = static_cast<int>(k & 1);
            // draw the batch after next once this batch starts
            if (k >= kRkBatch && (k % kRkBatch) == 0) draw_batch(k / kRkBatch + 1);
            double a[J];
            for (int j = 0; j < J; ++j) a[j] = ring[u][j];
            const double bi = rb[u], ni = rn[u];
            const int row = ri[u];
            // the row of iteration k + AH into the freed slot
            const int64_t kn = k + AH;
            if (kn <= P.maxit) load_row(pick[(kn / kRkBatch) & 1][kn % kRkBatch], ring[u], rb[u], rn[u], ri[u]);
            double pd = 0.0, pe = 0.0;
            for (int j = 0; j < J; ++j) {
                pd += a[j] * x[j];
                const double e = x[j] - xr[j];
                pe += e * e;
            }
            pd = group_sum_t<double, kWave>(pd);
            pe = group_sum_t<double, kWave>(pe);
            if (lane == 0) {
                red[par][wave][0] = pd;
                red[par][wave][1] = pe;
            }
            if (tid == 0) s_cancel[par] = (P.cancel && (k % P.check_every) == 0 && *P.cancel != 0) ? 1 : 0;
            __syncthreads();
            double dot = 0.0, e2 = 0.0;
            for (int w = 0; w < NW; ++w) {
                dot += red[par][w][0];
                e2 += red[par][w][1];
            }
            // stop test on x_k
            meas = xref2 > 0.0 ? e2 / xref2 : e2;
            if (xref2 > 0.0 ? (e2 / xref2 <= P.tol2) : (e2 <= P.tol2)) { status = CSK_OK; done = true; break; }
            if (k == P.maxit) { status = CSK_NOT_CONVERGED; done = true; break; }
            if (s_cancel[par]) { status = CSK_CANCELLED; done = true; break; }
            if (!isfinite(total)) { status = CSK_ERR_NONFINITE; done = true; break; }
            if (!(total > 0.0)) { status = CSK_ERR_DEGENERATE; done = true; break; }
            const double r = bi - dot;
            if (!isfinite(r)) { status = CSK_ERR_NONFINITE; done = true; break; }
            const double alpha = r / ni;
            if (P.trace && tid == 0) P.trace[k] = row;
            for (int j = 0; j < J; ++j) x[j] = x[j] + alpha * a[j];
            ++k;
        }
    }
    for (int j = 0; j < J; ++j) {
        const int c = tid + j * NT;
        if (c < n) P.x[c] = x[j];
    }
    if (tid == 0 && P.res) {
        P.res->iters = k;
        P.res->status = status;
        P.res->fp64_fallback = 0;
        P.res->final_measure = meas;
        P.res->refreshes = 0;
    }
}

}  // namespace

size_t solve_rk_ws_bytes(int64_t d)
{
    Carve c(nullptr);
    c.take<double>(d);  // cumulative squared norms
    c.take<double>(d);  // nu2 when not supplied
    c.take<double>(kRkScanBlocks);  // block sums of the prefix
    return c.bytes();
}

csk_status solve_rk_run(const double* At, int64_t ldat, int64_t d, int64_t n, const double* bt, const double* nu2,
                        const double* x0, double* x, const csk_solve_opts* o, uint64_t sel_seed,
                        csk_solve_result* res, void* ws, size_t ws_bytes, hipStream_t st)
{
    Carve c(ws);
    RkArgs P{};
    P.cum = c.take<double>(d);
    double* nu2_ws = c.take<double>(d);
    double* bsum = c.take<double>(kRkScanBlocks);
    if (c.bytes() > ws_bytes) {
        set_error("solve workspace too small: need %zu bytes, got %zu", c.bytes(), ws_bytes);
        return CSK_ERR_WORKSPACE;
    }
    if (nu2 == nullptr) {
        const csk_status e = launch_row_norms2(At, ldat, d, n, nu2_ws, st);
        if (e != CSK_OK) return e;
        nu2 = nu2_ws;
    }
    P.At = At;
    P.bt = bt;
    P.nu2 = nu2;
    P.x0 = x0;
    P.xref = o->x_ref;
    P.x = x;
    P.res = res;
    P.cancel = o->cancel;
    P.ldat = ldat;
    P.maxit = o->maxit;
    P.seed = sel_seed;
    P.tol2 = o->tol * o->tol;
    P.trace = o->trace_idx;
    P.d = (int32_t)d;
    P.n = (int32_t)n;
    P.check_every = o->check_every > 0 ? o->check_every : 256;
    k_rk_blocksum<<<kRkScanBlocks, kRkScanNT, 0, st>>>(P, bsum);
    CSK_LAUNCH_CHECK("k_rk_blocksum");
    k_rk_blockoff<<<1, kWave, 0, st>>>(bsum);
    CSK_LAUNCH_CHECK("k_rk_blockoff");
    k_rk_prefix<<<kRkScanBlocks, kRkScanNT, 0, st>>>(P, bsum);
    CSK_LAUNCH_CHECK("k_rk_prefix");
    // one wavefront up to 16 columns per lane (1024), else 512 threads
    if (n <= 16 * kWave) {
        const int64_t per = (n + kWave - 1) / kWave;
        if (per <= 1) k_solve_rk<kWave, 1><<<1, kWave, 0, st>>>(P);
        else if (per <= 2) k_solve_rk<kWave, 2><<<1, kWave, 0, st>>>(P);
        else if (per <= 4) k_solve_rk<kWave, 4><<<1, kWave, 0, st>>>(P);
        else if (per <= 8) k_solve_rk<kWave, 8><<<1, kWave, 0, st>>>(P);
        else k_solve_rk<kWave, 16><<<1, kWave, 0, st>>>(P);
    } else {
        const int64_t per = (n + kRkNT - 1) / kRkNT;
        if (per <= 4) k_solve_rk<kRkNT, 4><<<1, kRkNT, 0, st>>>(P);
        else if (per <= 8) k_solve_rk<kRkNT, 8><<<1, kRkNT, 0, st>>>(P);
        else if (per <= 16) k_solve_rk<kRkNT, 16><<<1, kRkNT, 0, st>>>(P);
        else {
            set_error("n=%lld exceeds %d", (long long)n, 16 * kRkNT);
            return CSK_ERR_UNSUPPORTED;
        }
    }
    CSK_LAUNCH_CHECK("k_solve_rk");
    return CSK_OK;
}

}  // namespace csk
