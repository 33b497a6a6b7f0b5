// DAMAS sweeps (section "DAMAS"): projected Gauss-Seidel on A~ x~ = b~,
//   r_i = sum_j A_ij x_j - b~_i   (x_j already updated for j < i)
//   x_i = max(x_i - r_i / A_ii, 0),  i = 0 .. S~-1, for every sweep,
// followed by the scatter of x~ back onto the full grid (zero elsewhere).
//
// One workgroup (4 waves) owns one bin for all its sweeps; x~ lives in LDS
// in double, whatever A's storage type: the sweep state, b~ and every sum
// are double, and float storage of A only rounds its entries once.
// Rows go in tiles of 64.  For a tile starting at t0:
//   phase A (all waves): r_l = sum_j A_lj x_j - b~_l for the 64 rows, with
//     the current x: rows before the tile already carry this sweep's values,
//     the tile and the rows after it the previous sweep's.  A rows stream
//     from memory as 16-byte vectors; each wave owns 16 rows and reduces
//     them across its lanes with a transpose-reduction;
//   phase B (wave 0): the 64 rows are updated in order, lane l holding r_l;
//     after row i moves by delta, every lane adds A_li * delta, so row l
//     sees the new value of every earlier row of the tile.  A is symmetric,
//     so A_li is read as A_il: row i of the tile block, coalesced.
// This is the same iteration as the row-by-row scheme; only the order in
// which each r_i's terms are summed differs.
#include "common.h"

namespace damas {

constexpr int kGsThreads = 256;
constexpr int kGsTile = 64;

// 16 bytes of one A row per lane: 4 floats or 2 doubles; x~ is double.
template <typename TA> struct Row16;
template <> struct Row16<float> {
    static constexpr int n = 4;
    __device__ static double dot(const float *a, const double *x)
    {
        const float4 v = *reinterpret_cast<const float4 *>(a);
        const double2 x0 = *reinterpret_cast<const double2 *>(x);
        const double2 x1 = *reinterpret_cast<const double2 *>(x + 2);
        return ((double)v.x * x0.x + (double)v.y * x0.y) +
               ((double)v.z * x1.x + (double)v.w * x1.y);
    }
};
template <> struct Row16<double> {
    static constexpr int n = 2;
    __device__ static double dot(const double *a, const double *x)
    {
        const double2 v = *reinterpret_cast<const double2 *>(a);
        const double2 x0 = *reinterpret_cast<const double2 *>(x);
        return v.x * x0.x + v.y * x0.y;
    }
};

// Sum 16 per-lane partial sums across the 64 lanes of a wave.  Lane l ends
// with the full sum of row (l >> 2) (every lane of a quad agrees).
__device__ inline double transpose_reduce16(double v[16], int lane)
{
#pragma unroll
    for (int h = 8, mask = 32; h >= 1; h >>= 1, mask >>= 1) {
        const bool upper = (lane & mask) != 0;
#pragma unroll
        for (int r = 0; r < h; ++r) {
            double send = upper ? v[r] : v[r + h];
            double keep = upper ? v[r + h] : v[r];
            v[r] = keep + __shfl_xor(send, mask);
        }
    }
    double s = v[0];
    s += __shfl_xor(s, 2);
    s += __shfl_xor(s, 1);
    return s;
}

template <typename TA, typename TX>
__global__ __launch_bounds__(kGsThreads) void gs_kernel(
    int N, const int32_t *__restrict__ s_tilde, int max_kept,
    const int32_t *__restrict__ idx, const int64_t *__restrict__ off,
    const TA *__restrict__ A_all, const double *__restrict__ b, int iters,
    const TX *__restrict__ x_init, TX *__restrict__ x_map, int *fault)
{
    constexpr int V = Row16<TA>::n;
    extern __shared__ double xs[]; // [ld_cap] x~, then [64] residuals
    const int64_t ld_cap = ld_of(max_kept);
    double *rs = xs + ld_cap;

    const int f = blockIdx.x;
    const int S = N * N;
    int St = s_tilde[f];
    if (St > max_kept) {
        if (threadIdx.x == 0)
            atomicOr(fault, 4);
        St = 0;
    }
    const int64_t ld = ld_of(St);
    const TA *A = A_all + (St > 0 ? off[f] : 0);
    const int32_t *id = idx + (int64_t)f * S;
    const double *bf = b + (int64_t)f * S;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);

    for (int64_t i = tid; i < ld; i += kGsThreads)
        xs[i] = (i < St && x_init) ? (double)x_init[(int64_t)f * S + id[i]] : 0.0;
    __syncthreads();

    for (int it = 0; it < iters; ++it) {
        for (int t0 = 0; t0 < St; t0 += kGsTile) {
            const int rows = min(kGsTile, St - t0);
            // ---- phase A: residuals of the tile's rows -------------------
            const int rbase = t0 + w * 16;
            const int nrw = max(0, min(16, St - rbase));
            const int myrow = rbase + (lane >> 2);
            double bt = 0.0;
            if ((lane & 3) == 0 && myrow < St)
                bt = bf[id[myrow]];
            double acc[16];
#pragma unroll
            for (int r = 0; r < 16; ++r)
                acc[r] = 0.0;
            for (int64_t j = (int64_t)lane * V; j < ld; j += 64 * V) {
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    if (r < nrw)
                        acc[r] += Row16<TA>::dot(&A[(int64_t)(rbase + r) * ld + j], &xs[j]);
            }
            const double sum = transpose_reduce16(acc, lane);
            if ((lane & 3) == 0 && myrow < St)
                rs[myrow - t0] = sum - bt;
            __syncthreads();
            // ---- phase B: the tile's rows in order -----------------------
            if (w == 0) {
                const bool mine = lane < rows;
                double a[kGsTile];
#pragma unroll
                for (int i = 0; i < kGsTile; ++i)
                    a[i] = (i < rows && mine) ? (double)A[(int64_t)(t0 + i) * ld + t0 + lane] : 0.0;
                double rl = mine ? rs[lane] : 0.0;
                const double xo = mine ? xs[t0 + lane] : 0.0;
                const double iv =
                    mine ? 1.0 / (double)A[(int64_t)(t0 + lane) * ld + t0 + lane] : 0.0;
                double xmine = xo;
#pragma unroll
                for (int i = 0; i < kGsTile; ++i) {
                    if (i < rows) {
                        const double ri = lane_bcast(rl, i);
                        const double xi = lane_bcast(xo, i);
                        const double ivi = lane_bcast(iv, i);
                        double xn = xi - ri * ivi;
                        xn = xn > 0.0 ? xn : 0.0;
                        const double dlt = xn - xi;
                        rl += a[i] * dlt;
                        xmine = lane == i ? xn : xmine;
                    }
                }
                if (mine)
                    xs[t0 + lane] = xmine;
            }
            __syncthreads();
        }
    }

    // Scatter: x_map[n] = x~_i at n = idx[i], 0 in the gaps between kept
    // points, so every grid point is written exactly once.
    TX *xo = x_map + (int64_t)f * S;
    if (St == 0) {
        for (int n = tid; n < S; n += kGsThreads)
            xo[n] = (TX)0;
        return;
    }
    for (int i = tid; i < St; i += kGsThreads) {
        const int n = id[i];
        const int prev = i == 0 ? -1 : id[i - 1];
        for (int q = prev + 1; q < n; ++q)
            xo[q] = (TX)0;
        xo[n] = (TX)xs[i];
        if (i == St - 1)
            for (int q = n + 1; q < S; ++q)
                xo[q] = (TX)0;
    }
}

int gs_max_kept(int precision)
{
    // x~ (ld doubles) plus 64 residuals in 160 KB of LDS, less a margin.
    (void)precision;
    const size_t lds = 160 * 1024 - 1024;
    return (int)((lds / sizeof(double) - kGsTile) & ~(size_t)7);
}

hipError_t launch_gs(int N, int n_bins, const int32_t *s_tilde, int max_kept,
                     const int32_t *idx, const int64_t *off, int precision,
                     const void *A, const double *b, int iterations,
                     const void *x_init, void *x_map, int *fault,
                     hipStream_t s)
{
    if (n_bins == 0)
        return hipSuccess;
    const size_t lds = sizeof(double) * ((size_t)ld_of(max_kept) + kGsTile);
    static const hipError_t attr =
        allow_big_lds((const void *)gs_kernel<double, double>) == hipSuccess
            ? allow_big_lds((const void *)gs_kernel<float, float>)
            : hipErrorInvalidValue;
    if (attr != hipSuccess)
        return attr;
    if (precision == DAMAS_PREC_FP64)
        hipLaunchKernelGGL((gs_kernel<double, double>), dim3(n_bins), dim3(kGsThreads), lds,
                           s, N, s_tilde, max_kept, idx, off, (const double *)A, b,
                           iterations, (const double *)x_init, (double *)x_map, fault);
    else
        hipLaunchKernelGGL((gs_kernel<float, float>), dim3(n_bins), dim3(kGsThreads), lds,
                           s, N, s_tilde, max_kept, idx, off, (const float *)A, b,
                           iterations, (const float *)x_init, (float *)x_map, fault);
    return hipGetLastError();
}

} // namespace damas
