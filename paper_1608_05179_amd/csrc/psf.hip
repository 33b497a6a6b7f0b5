// Steering rows of the kept points and the point-spread matrix over them
// (section "DAMAS": PSF(r|r_s) = |v(r)^H g_{r_s}|^2 / M^2 arranged as A of
// Eq. Axb, restricted to the compressed grid as in Eq. Axb_CG).
//
// With unit-magnitude steering e_m = er_m + i ei_m the complex Gram entry
// G_ij = sum_m conj(e_im) e_jm splits into two real products over the mics:
//   Re G = Er_I Er_J^T + Ei_I Ei_J^T,   Im G = Er_I Ei_J^T - Ei_I Er_J^T,
// and A_ij = ((Re G)^2 + (Im G)^2) / M^2.  Both products run on the matrix
// cores (16x16x4 f64 MFMA); A is formed in double and rounded once to its
// storage type.  A is symmetric, so only tiles I <= J are computed and each
// value is written to (i,j) and (j,i).
//
// With the paper's pair (beamformer v, propagation g of different
// magnitudes) A is not symmetric: every tile is computed, and the arena
// holds A transposed, row r = source point, column c = beam point,
// arena[r][c] = A[c][r] = |g_r^H v_c|^2 / M^2, so that a 64-column strip of
// the arena holds the coefficients of 64 rows of A x, as the sweeps read it.
// With the CSM diagonal removed, A = (|G|^2 - sum_m |v_m|^2 |g_m|^2) /
// (M^2 - M): the sum is M for unit steering and one more real product (of
// squared magnitudes) on the matrix cores for the paper's pair.
#include "common.h"

namespace damas {

// ---------------------------------------------------------------------------
// Steering rows (double): E[f][i] = [cos(k d_0..M-1), -sin(k d_0..M-1)] for
// the kept points i < s_tilde, zero for the padding rows up to ld.

// With the paper's pair (PAPER) two row sets per bin: rows [0, ld) hold the
// beamformer vectors v = (d / |r|) e, rows [ld, 2 ld) the propagation
// vectors g = (|r| / d) e.
template <bool PAPER>
__global__ __launch_bounds__(256) void steer_kernel(
    Geom g, const double *__restrict__ freq, const int32_t *__restrict__ idx,
    const int32_t *__restrict__ s_tilde, int max_kept, double *__restrict__ E,
    int64_t e_stride, int *fault)
{
    const int f = blockIdx.y;
    int St = s_tilde[f];
    if (St > max_kept) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            atomicOr(fault, 1);
        St = 0;
    }
    const int64_t ld = ld_of(St);
    const int M = g.M;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / M;
    const int m = (int)(t % M);
    if (i >= ld)
        return;
    double *row = E + (int64_t)f * e_stride + i * 2 * M;
    double *row_g = row + ld * 2 * M; // PAPER: the propagation vectors
    if (i < St) {
        const int S = g.N * g.N;
        const int n = idx[(int64_t)f * S + i];
        const double k = kTwoPi * freq[f] / g.c;
        double s, c;
        const double d = point_mic_dist(g, n, m);
        sincos(k * d, &s, &c);
        if (PAPER) {
            const double rn = point_origin_dist(g, n);
            const double av = d / rn, ag = rn / d;
            row[m] = av * c;
            row[M + m] = -av * s;
            row_g[m] = ag * c;
            row_g[M + m] = -ag * s;
        } else {
            row[m] = c;
            row[M + m] = -s;
        }
    } else {
        row[m] = 0.0;
        row[M + m] = 0.0;
        if (PAPER) {
            row_g[m] = 0.0;
            row_g[M + m] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// MFMA tile of A: f64 16x16x4 products (steering in double), stored as TS.
//
// Operand layout of v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][k] and
// B[k][l % 16] with k = l / 16; accumulator element v of lane l holds
// D[l / 16 + 4 v][l % 16].  The k index may be any permutation of the mics
// as long as both operands use the same one: each lane reads two
// consecutive mics (16 bytes) and feeds them to two successive MFMAs.

typedef double dacc4 __attribute__((ext_vector_type(4)));

constexpr int kPsfTile = 64;
constexpr int kPsfThreads = 256;
constexpr int kPsfChunk = 32;                // mics staged in LDS at a time
constexpr int kPsfPitch = kPsfChunk + 2;     // doubles per LDS row

__device__ inline dacc4 mma64(double a, double b, dacc4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline uint16_t bf16_rne_f(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7fffu + ((u >> 16) & 1u); // round to nearest even (finite inputs)
    return (uint16_t)(u >> 16);
}

// Optional outputs of the float PSF for the per-bin storage classes:
//   lo    bf16 residuals lo = bf16(A - float(A)) at the arena's offsets,
//   tsum  per bin and tile, the sum of the tile's entries of A over kept
//         rows and columns, each off-diagonal value counted for (i,j) and
//         (j,i) (tile index t of the launch grid, stride tstride per bin).
struct PsfExtra {
    uint16_t *lo;
    double *tsum;
    int64_t tstride;
};

template <typename TS, bool PAIR, bool DIAG>
__global__ __launch_bounds__(kPsfThreads) void psf_kernel(
    int M, const int32_t *__restrict__ s_tilde, int max_kept,
    const double *__restrict__ E, int64_t e_stride,
    const int64_t *__restrict__ off, TS *__restrict__ A, int *fault, PsfExtra ex)
{
    __shared__ double erI[kPsfTile * kPsfPitch];
    __shared__ double eiI[kPsfTile * kPsfPitch];
    __shared__ double erJ[kPsfTile * kPsfPitch];
    __shared__ double eiJ[kPsfTile * kPsfPitch];
    __shared__ double red[kPsfThreads / 64];

    const int f = blockIdx.y;
    const int St = s_tilde[f];
    if (St > max_kept) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            atomicOr(fault, 2);
        return;
    }
    const int64_t ld = ld_of(St);
    const int nt = (int)((ld + kPsfTile - 1) / kPsfTile);
    const int t = blockIdx.x;
    int I, J;
    if (PAIR) {
        // Every tile, I (arena rows, sources) fastest.
        if (t >= nt * nt)
            return;
        I = t % nt;
        J = t / nt;
    } else {
        if (t >= nt * (nt + 1) / 2)
            return;
        // Upper-triangle tile (I <= J), J-major numbering t = J(J+1)/2 + I.
        J = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while (J * (J + 1) / 2 > t)
            --J;
        while ((J + 1) * (J + 2) / 2 <= t)
            ++J;
        I = t - J * (J + 1) / 2;
    }
    const int64_t I0 = (int64_t)I * kPsfTile, J0 = (int64_t)J * kPsfTile;

    const double *Ef = E + (int64_t)f * e_stride;
    // Row operands: tile I from the propagation rows (the pair) or the
    // steering rows, tile J from the (beamformer) steering rows.
    const double *EfI = PAIR ? Ef + ld * 2 * M : Ef;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int wr = w >> 1, wc = w & 1; // 32 x 32 quadrant of the tile
    const int lr = lane & 15, lg = lane >> 4;

    dacc4 re[2][2], im[2][2], dd[PAIR && DIAG ? 2 : 1][PAIR && DIAG ? 2 : 1];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) {
            re[a][c] = dacc4{0, 0, 0, 0};
            im[a][c] = dacc4{0, 0, 0, 0};
            if constexpr (PAIR && DIAG)
                dd[a][c] = dacc4{0, 0, 0, 0};
        }

    for (int mc = 0; mc < M; mc += kPsfChunk) {
        __syncthreads();
        for (int e = threadIdx.x; e < kPsfTile * kPsfChunk; e += kPsfThreads) {
            const int r = e / kPsfChunk, mm = e % kPsfChunk, m = mc + mm;
            double vrI = 0, viI = 0, vrJ = 0, viJ = 0;
            if (m < M) {
                if (I0 + r < ld) {
                    const double *row = EfI + (I0 + r) * 2 * M;
                    vrI = row[m];
                    viI = row[M + m];
                }
                if (J0 + r < ld) {
                    const double *row = Ef + (J0 + r) * 2 * M;
                    vrJ = row[m];
                    viJ = row[M + m];
                }
            }
            erI[r * kPsfPitch + mm] = vrI;
            eiI[r * kPsfPitch + mm] = viI;
            erJ[r * kPsfPitch + mm] = vrJ;
            eiJ[r * kPsfPitch + mm] = viJ;
        }
        __syncthreads();
        const int mlen = min(kPsfChunk, M - mc);
        // Groups of 8 mics: lane group lg reads mics [m8 + 2 lg, m8 + 2 lg + 2).
        for (int m8 = 0; m8 < mlen; m8 += 8) {
            double2 ar[2], ai[2], br[2], bi[2];
            const int col = m8 + 2 * lg;
            for (int a = 0; a < 2; ++a) {
                const int r = wr * 32 + a * 16 + lr;
                ar[a] = *reinterpret_cast<const double2 *>(&erI[r * kPsfPitch + col]);
                ai[a] = *reinterpret_cast<const double2 *>(&eiI[r * kPsfPitch + col]);
            }
            for (int c = 0; c < 2; ++c) {
                const int r = wc * 32 + c * 16 + lr;
                br[c] = *reinterpret_cast<const double2 *>(&erJ[r * kPsfPitch + col]);
                bi[c] = *reinterpret_cast<const double2 *>(&eiJ[r * kPsfPitch + col]);
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) {
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const double xr = s ? ar[a].y : ar[a].x;
                    const double xi = s ? ai[a].y : ai[a].x;
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const double yr = s ? br[c].y : br[c].x;
                        const double yi = s ? bi[c].y : bi[c].x;
                        re[a][c] = mma64(xr, yr, re[a][c]);
                        re[a][c] = mma64(xi, yi, re[a][c]);
                        im[a][c] = mma64(xr, yi, im[a][c]);
                        im[a][c] = mma64(-xi, yr, im[a][c]);
                        if constexpr (PAIR && DIAG)
                            dd[a][c] = mma64(xr * xr + xi * xi, yr * yr + yi * yi, dd[a][c]);
                    }
                }
            }
        }
    }

    // Epilogue: A = (Re^2 + Im^2) / M^2 in double, rounded once to TS,
    // mirrored; unit diagonal.
    TS *Af = A + off[f];
    uint16_t *Lf = ex.lo ? ex.lo + off[f] : nullptr;
    const double inv = 1.0 / ((double)M * (double)M - (DIAG ? (double)M : 0.0));
    double tacc = 0.0; // this thread's share of the tile's sum
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c)
            for (int v = 0; v < 4; ++v) {
                const int64_t row = I0 + wr * 32 + a * 16 + lg + 4 * v;
                const int64_t colj = J0 + wc * 32 + c * 16 + lr;
                if (row >= ld || colj >= ld)
                    continue;
                const double x = re[a][c][v], y = im[a][c][v];
                // The m = m' terms removed with the diagonal (M for unit
                // steering, on kept rows and columns only: padding stays 0).
                double dterm = 0.0;
                if constexpr (DIAG)
                    dterm = PAIR ? dd[PAIR && DIAG ? a : 0][PAIR && DIAG ? c : 0][v]
                                 : (row < St && colj < St ? (double)M : 0.0);
                const double vd = (x * x + y * y - dterm) * inv;
                const TS val = (TS)vd;
                if constexpr (PAIR) {
                    // Every entry on its own (arena[row][colj] = A[colj][row]);
                    // the same point's entry is A_ii = 1.
                    const bool same = colj == row;
                    const TS sv = same ? (row < St ? (TS)1 : (TS)0) : val;
                    Af[row * ld + colj] = sv;
                    if (Lf)
                        Lf[row * ld + colj] =
                            same ? (uint16_t)0 : bf16_rne_f((float)(vd - (double)val));
                    if (row < St && colj < St)
                        tacc += same ? 1.0 : vd;
                    continue;
                }
                // Tiles with I < J have every column beyond every row; on
                // diagonal tiles the lower half is the mirror of the upper.
                if (colj > row) {
                    Af[row * ld + colj] = val;
                    Af[colj * ld + row] = val;
                    if (Lf) {
                        const uint16_t l = bf16_rne_f((float)(vd - (double)val));
                        Lf[row * ld + colj] = l;
                        Lf[colj * ld + row] = l;
                    }
                    if (colj < St)
                        tacc += 2.0 * vd;
                } else if (colj == row) {
                    Af[row * ld + row] = row < St ? (TS)1 : (TS)0;
                    if (Lf)
                        Lf[row * ld + row] = 0;
                    if (row < St)
                        tacc += 1.0;
                }
            }
    if (ex.tsum) {
        // Fixed-order reduction (lanes, then waves), so the sum and the
        // classes chosen from it are the same in every run.
        for (int o = 32; o >= 1; o >>= 1)
            tacc += __shfl_xor(tacc, o, 64);
        if (lane == 0)
            red[w] = tacc;
        __syncthreads();
        if (threadIdx.x == 0)
            ex.tsum[(int64_t)f * ex.tstride + t] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// Storage class of each bin from the mean row sum of its A over the kept
// points, rho = (1/S~) sum_ij A_ij: about the number of kept points inside
// one main lobe, a measure of how strongly the unknowns overlap (the bins
// whose iterates move most with A's rounding have the largest).  A bin
// above rho_wide (and within the wide sweeps' capacity) is wide; in a bf16
// solve a bin above rho_f32 runs every sweep on the float system.  One
// wave per bin; the tile sums are added in a fixed order.
__global__ __launch_bounds__(64) void class_kernel(const int32_t *__restrict__ s_tilde,
                                                   int max_kept, const double *__restrict__ tsum,
                                                   int64_t tstride, double rho_wide,
                                                   double rho_f32, int wide_cap, int pair,
                                                   uint8_t *__restrict__ cls)
{
    const int f = blockIdx.x;
    const int St = s_tilde[f];
    const int lane = threadIdx.x;
    const int64_t nt = (ld_of(St) + kPsfTile - 1) / kPsfTile;
    const int64_t ntiles =
        St > 0 && St <= max_kept ? (pair ? nt * nt : nt * (nt + 1) / 2) : 0;
    double acc = 0.0;
    for (int64_t t = lane; t < ntiles; t += 64)
        acc += tsum[(int64_t)f * tstride + t];
    for (int o = 32; o >= 1; o >>= 1)
        acc += __shfl_xor(acc, o, 64);
    if (lane == 0) {
        const double rho = St > 0 ? acc / (double)St : 0.0;
        uint8_t c = 0;
        if (rho > rho_wide && St <= wide_cap && ntiles > 0)
            c = kClsWide;
        else if (rho > rho_f32 && ntiles > 0)
            c = kClsF32;
        cls[f] = c;
    }
}

// ---------------------------------------------------------------------------
// BF16 path: steering rows in bf16 and the PSF on the bf16 matrix cores.
//
// Row i of E16 (per bin, stride e16_stride elements) is
//   [er_0 .. er_{MP-1} | ei_0 .. ei_{MP-1}],  er = cos(k d), ei = -sin(k d),
// MP = M rounded up to 16 (padding zero), K = 2 MP a multiple of 32.  With
// P_i = row i and Q_j = [ei_j | -er_j]:
//   Re G_ij = P_i . P_j,   Im G_ij = P_i . Q_j,
// so both are real products over K on v_mfma_f32_16x16x32_bf16 (FP32
// accumulation).  Q_j is P_j read half a row further on, the sign flipped on
// its second half.

__device__ inline uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7fffu + ((u >> 16) & 1u); // round to nearest even (finite inputs)
    return (uint16_t)(u >> 16);
}

int mp_of(int M) { return (M + 15) & ~15; }

__global__ __launch_bounds__(256) void steer16_kernel(
    Geom g, const double *__restrict__ freq, const int32_t *__restrict__ idx,
    const int32_t *__restrict__ s_tilde, int max_kept, uint16_t *__restrict__ E,
    int64_t e_stride, int *fault)
{
    const int f = blockIdx.y;
    int St = s_tilde[f];
    if (St > max_kept) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            atomicOr(fault, 1);
        St = 0;
    }
    const int64_t ld = ld_of(St);
    const int M = g.M, MP = (M + 15) & ~15;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / MP;
    const int m = (int)(t % MP);
    if (i >= ld)
        return;
    uint16_t *row = E + (int64_t)f * e_stride + i * 2 * MP;
    uint16_t c16 = 0, s16 = 0;
    if (i < St && m < M) {
        const int S = g.N * g.N;
        const int n = idx[(int64_t)f * S + i];
        const double k = kTwoPi * freq[f] / g.c;
        double s, c;
        sincos(k * point_mic_dist(g, n, m), &s, &c);
        c16 = f32_to_bf16_rne((float)c);
        s16 = f32_to_bf16_rne((float)(-s));
    }
    row[m] = c16;
    row[MP + m] = s16;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kPsf16Pitch = kPsfTile + 8; // bf16 per LDS row of the staged tile

// One 64 x 64 tile (I <= J) of the bf16 A per 256-thread workgroup; wave w
// computes the 32 x 32 quadrant (w >> 1, w & 1) as 2 x 2 blocks of 16 x 16.
// MFMA operand layout: lane l holds row l % 16 of its block, k = 8 (l / 16)
// .. +7 of the current 32-wide k step (16 contiguous bytes of a row); the
// accumulator element v of lane l is D[4 (l / 16) + v][l % 16].
template <bool DIAG>
__global__ __launch_bounds__(kPsfThreads) void psf16_kernel(
    int M, const int32_t *__restrict__ s_tilde, int max_kept,
    const uint16_t *__restrict__ E, int64_t e_stride, const int64_t *__restrict__ off,
    uint16_t *__restrict__ A, int *fault)
{
    __shared__ uint16_t T[kPsfTile * kPsf16Pitch];

    const int f = blockIdx.y;
    const int St = s_tilde[f];
    if (St > max_kept) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            atomicOr(fault, 2);
        return;
    }
    const int64_t ld = ld_of(St);
    const int nt = (int)((ld + kPsfTile - 1) / kPsfTile);
    const int t = blockIdx.x;
    if (t >= nt * (nt + 1) / 2)
        return;
    int J = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (J * (J + 1) / 2 > t)
        --J;
    while ((J + 1) * (J + 2) / 2 <= t)
        ++J;
    const int I = t - J * (J + 1) / 2;
    const int64_t I0 = (int64_t)I * kPsfTile, J0 = (int64_t)J * kPsfTile;

    const int MP = (M + 15) & ~15, K = 2 * MP;
    const uint16_t *Ef = E + (int64_t)f * e_stride;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int wr = w >> 1, wc = w & 1;
    const int lr = lane & 15, lg = lane >> 4;

    // Rows past ld read row 0 (their results are never stored).
    const uint16_t *pa[2], *pb[2];
    for (int a = 0; a < 2; ++a) {
        const int64_t r = I0 + wr * 32 + a * 16 + lr;
        pa[a] = Ef + (r < ld ? r : 0) * K;
    }
    for (int c = 0; c < 2; ++c) {
        const int64_t r = J0 + wc * 32 + c * 16 + lr;
        pb[c] = Ef + (r < ld ? r : 0) * K;
    }

    f32x4 re[2][2], im[2][2];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) {
            re[a][c] = f32x4{0.f, 0.f, 0.f, 0.f};
            im[a][c] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    for (int kk = 0; kk < K; kk += 32) {
        const int k0 = kk + 8 * lg;                 // this lane's 8 k values
        const int kq = k0 < MP ? k0 + MP : k0 - MP; // Q_j = P_j shifted by MP
        const uint32_t qsign = k0 < MP ? 0u : 0x80008000u;
        bf16x8 xa[2], xb[2], xq[2];
        for (int a = 0; a < 2; ++a)
            xa[a] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(pa[a] + k0));
        for (int c = 0; c < 2; ++c) {
            xb[c] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(pb[c] + k0));
            uint4 q = *reinterpret_cast<const uint4 *>(pb[c] + kq);
            q.x ^= qsign;
            q.y ^= qsign;
            q.z ^= qsign;
            q.w ^= qsign;
            xq[c] = __builtin_bit_cast(bf16x8, q);
        }
        for (int a = 0; a < 2; ++a)
            for (int c = 0; c < 2; ++c) {
                re[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[a], xb[c], re[a][c], 0, 0, 0);
                im[a][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[a], xq[c], im[a][c], 0, 0, 0);
            }
    }

    // A = (Re^2 + Im^2) / M^2 in FP32 (with the diagonal removed:
    // (Re^2 + Im^2 - M) / (M^2 - M) on kept entries), rounded once to bf16,
    // staged in LDS.
    const float inv = 1.0f / ((float)M * (float)M - (DIAG ? (float)M : 0.0f));
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c)
            for (int v = 0; v < 4; ++v) {
                const int r = wr * 32 + a * 16 + 4 * lg + v, col = wc * 32 + c * 16 + lr;
                const float x = re[a][c][v], y = im[a][c][v];
                const float dterm =
                    DIAG && I0 + r < St && J0 + col < St ? (float)M : 0.0f;
                T[r * kPsf16Pitch + col] = f32_to_bf16_rne((x * x + y * y - dterm) * inv);
            }
    __syncthreads();

    // Coalesced stores of 8 bf16 per thread: the tile at (I, J) and, for
    // I < J, its transpose at (J, I).  A diagonal tile mirrors its upper
    // half, so A is bitwise symmetric; A_ii = 1 on kept rows, 0 on padding.
    uint16_t *Af = A + off[f];
    const bool diag = I == J;
    for (int e = threadIdx.x; e < kPsfTile * kPsfTile / 8; e += kPsfThreads) {
        const int r = e / (kPsfTile / 8), c0 = (e % (kPsfTile / 8)) * 8;
        uint16_t v8[8];
        uint16_t w8[8];
        for (int s = 0; s < 8; ++s) {
            const int c = c0 + s;
            uint16_t v;
            if (!diag || c > r)
                v = T[r * kPsf16Pitch + c];
            else if (c < r)
                v = T[c * kPsf16Pitch + r];
            else
                v = I0 + r < St ? (uint16_t)0x3f80 : (uint16_t)0; // 1.0 or 0
            v8[s] = v;
            w8[s] = T[c * kPsf16Pitch + r]; // transpose: row c0.. of (J, I)
        }
        // e indexes (row r, cols c0..c0+7) of the tile; the transposed store
        // writes row c of (J, I) -- here the roles of r and c swap, so the
        // transpose is written as (row r of (J,I)) = column r of T.
        if (I0 + r < ld && J0 + c0 < ld)
            *reinterpret_cast<uint4 *>(&Af[(I0 + r) * ld + J0 + c0]) =
                make_uint4(v8[0] | ((uint32_t)v8[1] << 16), v8[2] | ((uint32_t)v8[3] << 16),
                           v8[4] | ((uint32_t)v8[5] << 16), v8[6] | ((uint32_t)v8[7] << 16));
        if (!diag && J0 + r < ld && I0 + c0 < ld)
            *reinterpret_cast<uint4 *>(&Af[(J0 + r) * ld + I0 + c0]) =
                make_uint4(w8[0] | ((uint32_t)w8[1] << 16), w8[2] | ((uint32_t)w8[3] << 16),
                           w8[4] | ((uint32_t)w8[5] << 16), w8[6] | ((uint32_t)w8[7] << 16));
    }
}

hipError_t launch_steer16(const Geom &g, int n_bins, const double *freq, const int32_t *idx,
                          const int32_t *s_tilde, int max_kept, uint16_t *E, int64_t e_stride,
                          int *fault, hipStream_t s)
{
    if (n_bins == 0 || max_kept == 0)
        return hipSuccess;
    const int64_t work = ld_of(max_kept) * mp_of(g.M);
    dim3 grid((unsigned)((work + 255) / 256), n_bins);
    hipLaunchKernelGGL(steer16_kernel, grid, dim3(256), 0, s, g, freq, idx, s_tilde, max_kept,
                       E, e_stride, fault);
    return hipGetLastError();
}

hipError_t launch_psf16(int M, int n_bins, const int32_t *s_tilde, int max_kept,
                        const uint16_t *E, int64_t e_stride, const int64_t *off, uint16_t *A,
                        int *fault, hipStream_t s, int diag)
{
    if (n_bins == 0 || max_kept == 0)
        return hipSuccess;
    const int64_t nt = (ld_of(max_kept) + kPsfTile - 1) / kPsfTile;
    dim3 grid((unsigned)(nt * (nt + 1) / 2), n_bins);
    if (diag)
        hipLaunchKernelGGL(psf16_kernel<true>, grid, dim3(kPsfThreads), 0, s, M, s_tilde,
                           max_kept, E, e_stride, off, A, fault);
    else
        hipLaunchKernelGGL(psf16_kernel<false>, grid, dim3(kPsfThreads), 0, s, M, s_tilde,
                           max_kept, E, e_stride, off, A, fault);
    return hipGetLastError();
}

hipError_t launch_steer(const Geom &g, int n_bins, const double *freq,
                        const int32_t *idx, const int32_t *s_tilde,
                        int max_kept, double *E, int64_t e_stride, int *fault,
                        hipStream_t s, int steering)
{
    if (n_bins == 0 || max_kept == 0)
        return hipSuccess;
    const int64_t work = ld_of(max_kept) * g.M;
    dim3 grid((unsigned)((work + 255) / 256), n_bins);
    if (steering == DAMAS_STEER_PAPER)
        hipLaunchKernelGGL(steer_kernel<true>, grid, dim3(256), 0, s, g, freq, idx, s_tilde,
                           max_kept, E, e_stride, fault);
    else
        hipLaunchKernelGGL(steer_kernel<false>, grid, dim3(256), 0, s, g, freq, idx, s_tilde,
                           max_kept, E, e_stride, fault);
    return hipGetLastError();
}

int64_t psf_tiles(int max_kept, int steering)
{
    const int64_t nt = (ld_of(max_kept) + kPsfTile - 1) / kPsfTile;
    return steering == DAMAS_STEER_PAPER ? nt * nt : nt * (nt + 1) / 2;
}

template <typename TS>
static hipError_t launch_psf_t(dim3 grid, hipStream_t s, int steering, int diag, int M,
                               const int32_t *s_tilde, int max_kept, const double *E,
                               int64_t e_stride, const int64_t *off, TS *A, int *fault,
                               PsfExtra ex)
{
#define DAMAS_PSF_LAUNCH(P, D)                                                                 \
    hipLaunchKernelGGL((psf_kernel<TS, P, D>), grid, dim3(kPsfThreads), 0, s, M, s_tilde,      \
                       max_kept, E, e_stride, off, A, fault, ex)
    if (steering == DAMAS_STEER_PAPER) {
        if (diag)
            DAMAS_PSF_LAUNCH(true, true);
        else
            DAMAS_PSF_LAUNCH(true, false);
    } else {
        if (diag)
            DAMAS_PSF_LAUNCH(false, true);
        else
            DAMAS_PSF_LAUNCH(false, false);
    }
#undef DAMAS_PSF_LAUNCH
    return hipGetLastError();
}

hipError_t launch_psf(int M, int n_bins, const int32_t *s_tilde, int max_kept,
                      int precision, const double *E, int64_t e_stride,
                      const int64_t *off, void *A, int *fault, hipStream_t s,
                      const PsfClassArgs &pc, int steering, int diag)
{
    if (n_bins == 0 || max_kept == 0)
        return hipSuccess;
    const int64_t tiles = psf_tiles(max_kept, steering);
    dim3 grid((unsigned)tiles, n_bins);
    PsfExtra ex{nullptr, nullptr, tiles};
    if (precision == DAMAS_PREC_FP64)
        return launch_psf_t<double>(grid, s, steering, diag, M, s_tilde, max_kept, E, e_stride,
                                    off, (double *)A, fault, ex);
    ex.lo = pc.lo;
    ex.tsum = pc.cls ? pc.tsum : nullptr;
    hipError_t e = launch_psf_t<float>(grid, s, steering, diag, M, s_tilde, max_kept, E,
                                       e_stride, off, (float *)A, fault, ex);
    if (e != hipSuccess || !pc.cls)
        return e;
    hipLaunchKernelGGL(class_kernel, dim3(n_bins), dim3(64), 0, s, s_tilde, max_kept, pc.tsum,
                       tiles, pc.rho_wide, pc.rho_f32, pc.wide_cap,
                       steering == DAMAS_STEER_PAPER ? 1 : 0, pc.cls);
    return hipGetLastError();
}

} // namespace damas
