// Delay-and-sum beamforming map (section "Beamforming", Eq. dirty_map_1):
// b_n = Re(v_n^H C v_n) / M^2 at every grid point of every bin, in double,
// with v the unit-magnitude steering vector e_n or (the paper's beamformer
// vector) v_nm = (|r_n - r_m| / |r_n|) e_nm; with the CSM diagonal removed
// (the paper notes it is usually applied) the m = m' terms are dropped and
// the map is normalised by M^2 - M instead.
//
// One workgroup = one bin x 64 grid points; lane = grid point.  The 64
// steering vectors of the tile are built once into LDS (M x 64 complex
// doubles, mic-major so a wave reads 64 consecutive points).  Wave w of the
// workgroup takes the CSM rows m = w (mod waves); a CSM row is wave-uniform,
// so its entries come through the scalar cache while LDS feeds the per-lane
// steering values.  The tile's steering takes most of a CU's LDS, so one
// workgroup runs per CU and its waves hide each other's scalar-load
// latency.
#include "common.h"

namespace damas {

constexpr int kDasPts = 64;
constexpr int kDasThreads = 1024;
constexpr int kDasWaves = kDasThreads / 64;
constexpr int kDasRows = 4; // CSM rows per pass of a wave

template <bool PAPER, bool DIAG>
__global__ __launch_bounds__(kDasThreads) void das_kernel(
    Geom g, int S, const double *__restrict__ freq,
    const double *__restrict__ csm, double *__restrict__ b)
{
    extern __shared__ double2 sh_e[]; // [M][64]: a (cos, -sin) of k d, a = 1 or d / |r|
    __shared__ double part[kDasThreads / 64][kDasPts];

    const int f = blockIdx.y;
    const int p0 = blockIdx.x * kDasPts;
    const int M = g.M;
    const double k = kTwoPi * freq[f] / g.c;

    for (int t = threadIdx.x; t < M * kDasPts; t += kDasThreads) {
        int m = t / kDasPts, p = t % kDasPts;
        int n = p0 + p;
        double2 e = make_double2(0.0, 0.0);
        if (n < S) {
            double s, c;
            const double d = point_mic_dist(g, n, m);
            sincos(k * d, &s, &c);
            const double a = PAPER ? d / point_origin_dist(g, n) : 1.0;
            e = make_double2(a * c, -a * s);
        }
        sh_e[m * kDasPts + p] = e;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const double *C = csm + (size_t)f * M * M * 2;
    double acc = 0.0;
    // Wave w takes CSM rows m = w (mod kDasWaves), kDasRows of them per
    // pass, so each steering value read from LDS feeds 4 kDasRows
    // multiply-adds; the rows' terms are added to the point's sum in row
    // order whatever kDasRows is.
    for (int m = w; m < M; m += kDasWaves * kDasRows) {
        const double *cr[kDasRows];
#pragma unroll
        for (int q = 0; q < kDasRows; ++q)
            cr[q] = C + (size_t)(m + kDasWaves * q < M ? m + kDasWaves * q : m) * M * 2;
        double yr[kDasRows], yi[kDasRows];
#pragma unroll
        for (int q = 0; q < kDasRows; ++q)
            yr[q] = yi[q] = 0.0;
        for (int mp = 0; mp < M; ++mp) {
            const double2 e = sh_e[mp * kDasPts + lane];
#pragma unroll
            for (int q = 0; q < kDasRows; ++q) {
                const double ar = cr[q][2 * mp], ai = cr[q][2 * mp + 1];
                yr[q] += ar * e.x - ai * e.y;
                yi[q] += ar * e.y + ai * e.x;
            }
        }
        // Re(conj(e_m) y_m) = er*yr + ei*yi
#pragma unroll
        for (int q = 0; q < kDasRows; ++q)
            if (m + kDasWaves * q < M) {
                const double2 e0 = sh_e[(m + kDasWaves * q) * kDasPts + lane];
                acc += e0.x * yr[q] + e0.y * yi[q];
            }
    }
    if (DIAG) {
        // The m = m' terms, |v_m|^2 C_mm (C_mm real), of this wave's rows.
        double dsum = 0.0;
        for (int m = w; m < M; m += kDasWaves) {
            const double2 e = sh_e[m * kDasPts + lane];
            dsum += (e.x * e.x + e.y * e.y) * C[((size_t)m * M + m) * 2];
        }
        acc -= dsum;
    }
    part[w][lane] = acc;
    __syncthreads();
    if (threadIdx.x < kDasPts) {
        int n = p0 + lane;
        if (n < S) {
            double s = 0.0;
#pragma unroll
            for (int v = 0; v < kDasWaves; ++v)
                s += part[v][lane];
            b[(size_t)f * S + n] = s / ((double)M * (double)M - (DIAG ? (double)M : 0.0));
        }
    }
}

template <bool PAPER, bool DIAG>
static hipError_t launch_das_t(const Geom &g, int n_bins, const double *freq,
                               const double *csm, double *b, hipStream_t s)
{
    const int S = g.N * g.N;
    dim3 grid((S + kDasPts - 1) / kDasPts, n_bins);
    size_t lds = sizeof(double2) * (size_t)g.M * kDasPts;
    static const hipError_t attr = allow_big_lds((const void *)das_kernel<PAPER, DIAG>);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL((das_kernel<PAPER, DIAG>), grid, dim3(kDasThreads), lds, s, g, S, freq,
                       csm, b);
    return hipGetLastError();
}

hipError_t launch_das(const Geom &g, int n_bins, const double *freq,
                      const double *csm, double *b, hipStream_t s, int steering, int diag)
{
    if (n_bins == 0 || g.N == 0)
        return hipSuccess;
    if (steering == DAMAS_STEER_PAPER)
        return diag ? launch_das_t<true, true>(g, n_bins, freq, csm, b, s)
                    : launch_das_t<true, false>(g, n_bins, freq, csm, b, s);
    return diag ? launch_das_t<false, true>(g, n_bins, freq, csm, b, s)
                : launch_das_t<false, false>(g, n_bins, freq, csm, b, s);
}

} // namespace damas
