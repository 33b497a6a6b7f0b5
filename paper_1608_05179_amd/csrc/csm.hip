// Cross-spectral matrix from snapshots (Eq. (1)): C = (1/K) sum_k p_k p_k^H,
// C[m][q] = (1/K) sum_k p_k[m] conj(p_k[q]), per frequency bin.
//
// With p_k[m] = a + ib and p_k[q] = c + id the entry splits into real
// products over the snapshots, Re = sum (a c + b d) and Im = sum (b c - a d),
// i.e. two real GEMMs of the M x K matrices of real and imaginary parts,
// which run on the FP64 matrix cores (v_mfma_f64_16x16x4f64).  A wave owns a
// 16 x 16 block (one MFMA tile) of the upper block triangle of one bin
// and writes each entry and its conjugate mirror, so C is exactly
// Hermitian with a real diagonal.
#include "common.h"

namespace damas {

typedef double dacc4c __attribute__((ext_vector_type(4)));

constexpr int kCsmTiles = 1;   // MFMA tiles of 16 per block side
constexpr int kCsmBlock = 16 * kCsmTiles; // output block per wave
constexpr int kCsmWaves = 4;   // waves per workgroup, each on its own block
constexpr int kCsmDepth = 8;   // snapshot steps of 4 loaded ahead

__device__ inline dacc4c mma_csm(double a, double b, dacc4c c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Operand layout of v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][k] and
// B[k][l % 16] with k = l / 16; accumulator element v of lane l holds
// D[l / 16 + 4 v][l % 16].  Both operands here are mic vectors of the same
// snapshots: lane l reads p_{k0 + l/16}[r + l % 16] (16 bytes, 16 lanes on
// consecutive microphones).
__global__ __launch_bounds__(64 * kCsmWaves) void csm_kernel(
    int M, int K, int n_bins, int n_upper, const double2 *__restrict__ snap,
    double2 *__restrict__ csm)
{
    const int lane = threadIdx.x & 63;
    const int64_t job = (int64_t)blockIdx.x * kCsmWaves + (threadIdx.x >> 6);
    if (job >= (int64_t)n_bins * n_upper)
        return; // whole wave (no barrier in this kernel)
    const int f = (int)(job / n_upper);
    const int t = (int)(job % n_upper);
    // Upper block (I <= J), J-major numbering t = J (J + 1) / 2 + I.
    int J = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (J * (J + 1) / 2 > t)
        --J;
    while ((J + 1) * (J + 2) / 2 <= t)
        ++J;
    const int I = t - J * (J + 1) / 2;
    const int m0 = I * kCsmBlock, q0 = J * kCsmBlock;

    const double2 *P = snap + (int64_t)f * K * M;
    const int lr = lane & 15, lk = lane >> 4;
    int rows[kCsmTiles], cols[kCsmTiles];
    bool rok[kCsmTiles], cok[kCsmTiles];
    for (int a = 0; a < kCsmTiles; ++a) {
        rows[a] = m0 + a * 16 + lr;
        cols[a] = q0 + a * 16 + lr;
        rok[a] = rows[a] < M;
        cok[a] = cols[a] < M;
    }

    dacc4c re[kCsmTiles][kCsmTiles], im[kCsmTiles][kCsmTiles];
    for (int a = 0; a < kCsmTiles; ++a)
        for (int c = 0; c < kCsmTiles; ++c) {
            re[a][c] = dacc4c{0, 0, 0, 0};
            im[a][c] = dacc4c{0, 0, 0, 0};
        }

    const double2 zero2 = make_double2(0.0, 0.0);
    auto fetch = [&](int k, double2 (&x)[kCsmTiles], double2 (&y)[kCsmTiles]) {
        const bool kok = k < K;
        const double2 *row = P + (int64_t)(kok ? k : 0) * M;
        for (int a = 0; a < kCsmTiles; ++a) {
            x[a] = kok && rok[a] ? row[rows[a]] : zero2;
            y[a] = kok && cok[a] ? row[cols[a]] : zero2;
        }
    };
    // kCsmDepth snapshot steps in flight: a ring of register sets, slot d
    // holding step k0 + 4 d, refilled with step k0 + 4 d + 4 kCsmDepth once
    // its MFMAs have read it.  A bin's blocks first touch each snapshot row
    // together, from HBM, so one step ahead would not hide the latency.
    // Steps past K load zeros and add nothing.
    double2 x[kCsmDepth][kCsmTiles], y[kCsmDepth][kCsmTiles];
#pragma unroll
    for (int d = 0; d < kCsmDepth; ++d)
        fetch(4 * d + lk, x[d], y[d]);
    for (int k0 = 0; k0 < K; k0 += 4 * kCsmDepth) {
#pragma unroll
        for (int d = 0; d < kCsmDepth; ++d) {
            // p[m] = x = a + ib (rows), p[q] = y = c + id (columns)
            for (int a = 0; a < kCsmTiles; ++a)
                for (int c = 0; c < kCsmTiles; ++c) {
                    re[a][c] = mma_csm(x[d][a].x, y[d][c].x, re[a][c]);
                    im[a][c] = mma_csm(x[d][a].y, y[d][c].x, im[a][c]);
                }
            for (int a = 0; a < kCsmTiles; ++a)
                for (int c = 0; c < kCsmTiles; ++c) {
                    re[a][c] = mma_csm(x[d][a].y, y[d][c].y, re[a][c]);
                    im[a][c] = mma_csm(-x[d][a].x, y[d][c].y, im[a][c]);
                }
            fetch(k0 + 4 * (d + kCsmDepth) + lk, x[d], y[d]);
        }
    }

    // Entry (m, q) with m <= q and its mirror (q, m) = conj; the diagonal's
    // imaginary part is 0 exactly.
    double2 *C = csm + (int64_t)f * M * M;
    const double inv = 1.0 / (double)K;
    for (int a = 0; a < kCsmTiles; ++a)
        for (int c = 0; c < kCsmTiles; ++c)
            for (int v = 0; v < 4; ++v) {
                const int m = m0 + a * 16 + lk + 4 * v;
                const int q = q0 + c * 16 + lr;
                if (m >= M || q >= M || m > q)
                    continue;
                const double xr = re[a][c][v] * inv, xi = im[a][c][v] * inv;
                if (m == q) {
                    C[(int64_t)m * M + m] = make_double2(xr, 0.0);
                } else {
                    C[(int64_t)m * M + q] = make_double2(xr, xi);
                    C[(int64_t)q * M + m] = make_double2(xr, -xi);
                }
            }
}

int csm_upper_blocks(int M)
{
    const int nb = (M + kCsmBlock - 1) / kCsmBlock;
    return nb * (nb + 1) / 2;
}

hipError_t launch_csm(int M, int K, int n_bins, const double *snap, double *csm,
                      hipStream_t s)
{
    if (n_bins == 0)
        return hipSuccess;
    const int nu = csm_upper_blocks(M);
    const int64_t jobs = (int64_t)n_bins * nu;
    dim3 grid((unsigned)((jobs + kCsmWaves - 1) / kCsmWaves));
    hipLaunchKernelGGL(csm_kernel, grid, dim3(64 * kCsmWaves), 0, s, M, K, n_bins, nu,
                       (const double2 *)snap, (double2 *)csm);
    return hipGetLastError();
}

} // namespace damas
