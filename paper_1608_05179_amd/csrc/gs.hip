// DAMAS sweeps (section "DAMAS"): projected Gauss-Seidel on A~ x~ = b~,
//   r_i = sum_j A_ij x_j - b~_i   (x_j already updated for j < i)
//   x_i = max(x_i - r_i / A_ii, 0),  i = 0 .. S~-1, for every sweep,
// followed by the scatter of x~ back onto the full grid (zero elsewhere).
//
// One workgroup owns one bin for all its sweeps; x~ lives in LDS in double,
// whatever A's storage type: the sweep state, b~ and every sum are double,
// and float storage of A only rounds its entries once.
//
// Rows go in tiles of 64, and the tiles of all sweeps form one stream
// q = 0, 1, ... (tile q mod T of sweep q div T).  Two roles run side by side:
//   wave 0 (serial): updates the 64 rows of tile q in order.  Lane l holds
//     the residual of row l; after row i moves by d_i every later row l
//     adds A_li d_i, so row l sees the new value of each earlier row of the
//     tile.  The same broadcast d_i also accumulates, for the next tile's
//     rows, the change A_{q+1,i} d_i of their residuals.
//   waves 1-4 (stream): meanwhile compute the residuals of tile q+1 over
//     every column, taking tile q's columns at their values before this
//     tile's update (a snapshot, so the serial wave may overwrite them), and
//     by symmetry reading row r's sum down column r: each j is a contiguous
//     64-column strip, 16 bytes per lane.  The same reads hand wave 0, through
//     double-buffered LDS, the next tile's diagonal block and its coupling
//     to the tile after it, so the serial wave never waits on A.
// The residual of tile q+1 is then exactly the sum over the new values of
// every row before it and the previous sweep's values of itself and the rows
// after it: the same iteration as the row-by-row scheme; only the order in
// which each r_i's terms are summed (and, for a diagonal other than 1, the
// scaling by 1 / A_ii) differ.
#include "common.h"

namespace damas {

constexpr int kGsTile = 64;
constexpr int kGsStreamWaves = 4;
constexpr int kGsThreads = 64 * (1 + kGsStreamWaves);
constexpr int kGsCtPitch = kGsTile + 1; // rows of the coupling block
constexpr int kGsBatch = 8;             // loads in flight per stream lane

// 16 bytes of A per lane: CPL = 4 floats or 2 doubles.
template <typename TA> struct Vec16;
template <> struct Vec16<float> {
    typedef float4 type;
    static constexpr int n = 4;
    __device__ static float at(const float4 &v, int s)
    {
        return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
    }
    __device__ static float4 make(const float *a) { return make_float4(a[0], a[1], a[2], a[3]); }
};
template <> struct Vec16<double> {
    typedef double2 type;
    static constexpr int n = 2;
    __device__ static double at(const double2 &v, int s) { return s == 0 ? v.x : v.y; }
    __device__ static double2 make(const double *a) { return make_double2(a[0], a[1]); }
};

// LDS blocks handed from the stream waves to the serial wave for tile t
// (tn = the tile after it):
//   U[i][l]       = A_{t0+i, t0+l} for l > i, 0 for l <= i (strict upper)
//   dg[l]         = A_{t0+l, t0+l}
//   Ct[l][i]      = A_{tn0+l, t0+i} (pitch 65: lane l reads row l)
template <typename TA> struct TileBlocks {
    TA U[kGsTile * kGsTile];
    TA Ct[kGsTile * kGsCtPitch];
    TA dg[kGsTile];
};

// Stream role, one of kGsStreamWaves waves (sw = 0..): partial residual
// sums of the 64 rows of tile T (columns T0..T0+63 of every row j of A, A
// being symmetric) over the row groups this wave owns.  Rows j of the tile
// being updated, [X0, X0 + 64), take x from the snapshot xold.  Rows j in
// [T0, T0 + 64) also fill U and dg, rows j in [TN0, TN0 + 64) fill Ct.
// part[sw][r] receives the partial sum of row T0 + r.
//
// The sum runs branch-free over batches of kGsBatch loads, two batches in
// flight (rows past the wave's last group are read clamped and weighted 0),
// so the loads of one batch overlap the arithmetic of the other.
template <typename TA>
__device__ __forceinline__ void stream_strip(const TA *__restrict__ A, int64_t ld,
                                             const double *xs, const double *xold,
                                             const double *zero, int St, int T0, int X0,
                                             int TN0, double *part, TileBlocks<TA> *blk,
                                             int sw, int lane)
{
    typedef Vec16<TA> VA;
    typedef typename VA::type VT;
    constexpr int CPL = VA::n;         // columns per lane
    constexpr int LPJ = kGsTile / CPL; // lanes per row j
    constexpr int NW = kGsStreamWaves;
    const int jp = lane / LPJ;         // which of the CPL rows of a group
    const int cl = (lane % LPJ) * CPL; // first tile column of this lane
    const int64_t csrc = min((int64_t)(T0 + cl), ld - CPL);
    const TA *Ac = A + csrc;
    // Row groups of CPL consecutive j; this wave owns g = sw + NW k.
    const int ngroup = (St + CPL - 1) / CPL;
    const int nk = ngroup > sw ? (ngroup - sw + NW - 1) / NW : 0;
    const int gmax = ngroup - 1;

    double acc[CPL];
#pragma unroll
    for (int s = 0; s < CPL; ++s)
        acc[s] = 0.0;

    // Addresses split into a wave-uniform part (the group, scalar registers)
    // and a fixed per-lane byte offset (row jp of the group, column cl), so a
    // load costs no vector address arithmetic.
    const char *Ab = reinterpret_cast<const char *>(A);
    const uint32_t voff = (uint32_t)(((int64_t)jp * ld + csrc) * sizeof(TA));
    const int64_t gstride = (int64_t)CPL * ld * sizeof(TA); // bytes per group
    auto load = [&](VT *dst, int k0) {
#pragma unroll
        for (int n = 0; n < kGsBatch; ++n) {
            const int g = min(sw + NW * (k0 + n), gmax); // wave-uniform
            dst[n] = *reinterpret_cast<const VT *>(Ab + g * gstride + voff);
        }
    };
    auto accumulate = [&](const VT *src, int k0) {
#pragma unroll
        for (int n = 0; n < kGsBatch; ++n) {
            const int jb = (sw + NW * (k0 + n)) * CPL; // wave-uniform
            // x of row jb + jp: the snapshot inside the tile being updated,
            // the zero word past the wave's last group.
            const double *xb = k0 + n >= nk                 ? zero - jp
                               : jb >= X0 && jb < X0 + kGsTile ? xold + (jb - X0)
                                                               : xs + jb;
            const double xj = xb[jp];
#pragma unroll
            for (int s = 0; s < CPL; ++s)
                acc[s] += (double)VA::at(src[n], s) * xj;
        }
    };
    // sched_barrier keeps each batch's loads issued ahead of the arithmetic
    // on the other batch (the scheduler would otherwise sink them to their
    // uses and leave one or two loads in flight).
    if (nk > 0) {
        VT b0[kGsBatch], b1[kGsBatch];
        load(b0, 0);
        for (int k0 = 0; k0 < nk; k0 += 2 * kGsBatch) {
            load(b1, k0 + kGsBatch);
            __builtin_amdgcn_sched_barrier(0);
            accumulate(b0, k0);
            __builtin_amdgcn_sched_barrier(0);
            load(b0, k0 + 2 * kGsBatch);
            __builtin_amdgcn_sched_barrier(0);
            accumulate(b1, k0 + kGsBatch);
            __builtin_amdgcn_sched_barrier(0);
        }
    }

    // Hand-over blocks: the rows j of tiles T and TN that this wave owns
    // (re-read; they were just fetched).
    {
        const int n = kGsTile / CPL / NW + 1; // groups per wave in a tile, at most
        VT u[n], c[n];
#pragma unroll
        for (int m = 0; m < n; ++m) {
            const int gu = T0 / CPL + sw + NW * m, gc = TN0 / CPL + sw + NW * m;
            const int64_t ju = min((int64_t)gu * CPL + jp, ld - 1);
            const int64_t jc = min((int64_t)gc * CPL + jp, ld - 1);
            u[m] = *reinterpret_cast<const VT *>(&Ac[ju * ld]);
            c[m] = *reinterpret_cast<const VT *>(&Ac[jc * ld]);
        }
#pragma unroll
        for (int m = 0; m < n; ++m) {
            const int g = sw + NW * m; // group within the tile
            if (g * CPL < kGsTile) {
                const int i = g * CPL + jp;
                TA uu[CPL];
#pragma unroll
                for (int s = 0; s < CPL; ++s) {
                    const TA v = VA::at(u[m], s);
                    uu[s] = cl + s > i ? v : (TA)0;
                    if (cl + s == i)
                        blk->dg[i] = v;
                }
                *reinterpret_cast<VT *>(&blk->U[i * kGsTile + cl]) = VA::make(uu);
#pragma unroll
                for (int s = 0; s < CPL; ++s)
                    blk->Ct[i * kGsCtPitch + cl + s] = VA::at(c[m], s);
            }
        }
    }

    // Sum the CPL row groups (lanes l, l + LPJ, ...), then lanes 0..LPJ-1
    // hold the partial sums of the tile's 64 rows.
#pragma unroll
    for (int m = LPJ; m < 64; m <<= 1)
#pragma unroll
        for (int s = 0; s < CPL; ++s)
            acc[s] += __shfl_xor(acc[s], m);
    if (lane < LPJ)
#pragma unroll
        for (int s = 0; s < CPL; ++s)
            part[sw * kGsTile + cl + s] = acc[s];
}

// Serial role (one wave): the rows of each tile in order.  With the scaled
// residual rho_l = r_l / A_ll, row i's change is d_i = max(-rho_i, -x_i)
// (x_i + d_i = max(x_i - r_i / A_ii, 0)), and every later row l of the
// tile takes rho_l += (A_li / A_ll) d_i.  U is zero on and below the
// diagonal, so lane l's rho stops changing once its own row is done and its
// new value is formed once after the loop.  UNIT: A_ii = 1, no scaling.
template <typename TA, bool UNIT>
__device__ __forceinline__ void serial_role(double *xs, const double *parts, double *xold,
                                            const TileBlocks<TA> *blks,
                                            const int32_t *__restrict__ id,
                                            const double *__restrict__ bf, int St, int ntile,
                                            long long total, int lane)
{
    __builtin_amdgcn_s_setprio(3);
    int t = 0;
    double bt = lane < St ? bf[id[lane]] : 0.0;
    double rn = 0.0; // change of the next tile's residuals from this tile
    for (long long q = 0; q < total; ++q) {
        const int t0 = t * kGsTile;
        const int tn = t + 1 == ntile ? 0 : t + 1;
        const int tn0 = tn * kGsTile;
        const int rows = min(kGsTile, St - t0);
        const bool mine = lane < rows;
        const TileBlocks<TA> &bk = blks[q & 1];
        const double *pt = parts + (q & 1) * kGsStreamWaves * kGsTile;
        // b~ of the next tile's rows, needed one tile from now.
        const double bt_next = tn0 + lane < St ? bf[id[tn0 + lane]] : 0.0;
        double r = -bt + rn;
#pragma unroll
        for (int k = 0; k < kGsStreamWaves; ++k)
            r += pt[k * kGsTile + lane];
        double il = 1.0;
        if (!UNIT)
            il = mine ? 1.0 / (double)bk.dg[lane] : 0.0;
        const double xl = mine ? xs[min(t0 + lane, St - 1)] : 0.0;
        double rho = UNIT ? r : r * il;
        // Software pipeline: the block entries of step i + kPre are read
        // from LDS during step i (raw storage type), and those of step i + 1
        // are widened to double at the end of step i, off the serial chain
        //   max -> readlane -> fma;
        // sched_barrier keeps each step's instructions together, and the
        // four independent coupling sums fill the chain's latency.
        constexpr int kPre = 8;
        TA ur[kPre], cr[kPre];
#pragma unroll
        for (int i = 0; i < kPre; ++i) {
            ur[i] = bk.U[i * kGsTile + lane];
            cr[i] = bk.Ct[lane * kGsCtPitch + i];
        }
        double ud = UNIT ? (double)ur[0] : (double)ur[0] * il, cd = (double)cr[0];
        double rn4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < kGsTile; ++i) {
            const double d = lane_bcast(fmax(-rho, -xl), i);
            rho += ud * d;
            // Pin the chain update first in the step, then the coupling sum
            // (otherwise it is sunk past the loop and all 64 broadcasts stay
            // live in scalar registers).
            asm volatile("" : "+v"(rho));
            rn4[i & 3] += cd * d;
            asm volatile("" : "+v"(rn4[i & 3]));
            if (i + kPre < kGsTile) {
                ur[i % kPre] = bk.U[(i + kPre) * kGsTile + lane];
                cr[i % kPre] = bk.Ct[lane * kGsCtPitch + i + kPre];
            }
            if (i + 1 < kGsTile) {
                ud = (double)ur[(i + 1) % kPre];
                if (!UNIT)
                    ud *= il;
                cd = (double)cr[(i + 1) % kPre];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        rn = (rn4[0] + rn4[1]) + (rn4[2] + rn4[3]);
        if (mine)
            xs[t0 + lane] = xl + fmax(-rho, -xl);
        // Snapshot of the next tile's values for the stream waves, which
        // read it while this wave overwrites that tile.
        xold[((q + 1) & 1) * kGsTile + lane] =
            tn0 + lane < St ? xs[min(tn0 + lane, St - 1)] : 0.0;
        bt = bt_next;
        t = tn;
        __syncthreads();
    }
}

template <typename TA> constexpr size_t gs_lds_fixed()
{
    return sizeof(double) * (2 * kGsStreamWaves * kGsTile + 2 * kGsTile + 8) +
           2 * sizeof(TileBlocks<TA>);
}

template <typename TA, typename TX, bool UNIT>
__global__ __launch_bounds__(kGsThreads) void gs_kernel(
    int N, const int32_t *__restrict__ s_tilde, int max_kept,
    const int32_t *__restrict__ idx, const int64_t *__restrict__ off,
    const TA *__restrict__ A_all, const double *__restrict__ b, int iters,
    const TX *__restrict__ x_init, TX *__restrict__ x_map, int *fault)
{
    // LDS: x~ [ld_cap] | partial sums [2][NW][64] | snapshots [2][64] |
    //      zero words [8] | tile blocks [2]
    extern __shared__ double xs[];
    const int64_t ld_cap = ld_of(max_kept);
    double *parts = xs + ld_cap;
    double *xold = parts + 2 * kGsStreamWaves * kGsTile;
    double *zero = xold + 2 * kGsTile;
    TileBlocks<TA> *blks = reinterpret_cast<TileBlocks<TA> *>(zero + 8);

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
    if (tid < 8)
        zero[tid] = 0.0;
    {
        TA *z = reinterpret_cast<TA *>(blks);
        for (int i = tid; i < (int)(2 * sizeof(TileBlocks<TA>) / sizeof(TA)); i += kGsThreads)
            z[i] = (TA)0;
    }
    __syncthreads();

    const int ntile = (St + kGsTile - 1) / kGsTile;
    const long long total = (long long)iters * ntile;
    if (total > 0) {
        // Prologue: residuals and blocks of tile 0; snapshot of tile 0.
        const int t1 = ntile > 1 ? kGsTile : 0;
        if (w > 0)
            stream_strip<TA>(A, ld, xs, xold, zero, St, 0, -2 * kGsTile, t1, parts,
                             &blks[0], w - 1, lane);
        else
            xold[lane] = lane < St ? xs[min(lane, St - 1)] : 0.0;
        __syncthreads();
        // The two roles run separate loops (w is wave-uniform) so that each
        // allocates only its own registers; both pass exactly one barrier
        // per tile.
        if (w == 0) {
            serial_role<TA, UNIT>(xs, parts, xold, blks, id, bf, St, ntile, total, lane);
        } else {
            int t = 0;
            for (long long q = 0; q < total; ++q) {
                const int tn = t + 1 == ntile ? 0 : t + 1;
                const int tnn = tn + 1 == ntile ? 0 : tn + 1;
                if (q + 1 < total)
                    stream_strip<TA>(A, ld, xs, xold + (q & 1) * kGsTile, zero, St,
                                     tn * kGsTile, t * kGsTile, tnn * kGsTile,
                                     parts + ((q + 1) & 1) * kGsStreamWaves * kGsTile,
                                     &blks[(q + 1) & 1], w - 1, lane);
                t = tn;
                __syncthreads();
            }
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

static size_t gs_lds_bytes(int precision, int max_kept)
{
    const size_t fixed = precision == DAMAS_PREC_FP64 ? gs_lds_fixed<double>()
                                                      : gs_lds_fixed<float>();
    return fixed + sizeof(double) * (size_t)ld_of(max_kept);
}

int gs_max_kept(int precision)
{
    // Everything in the 160 KB of LDS of one CU, less a margin.
    const size_t lds = 160 * 1024 - 512;
    const size_t fixed = gs_lds_bytes(precision, 0);
    return (int)(((lds - fixed) / sizeof(double)) & ~(size_t)7);
}

template <typename TA, typename TX, bool UNIT>
static hipError_t launch_gs_t(int N, int n_bins, const int32_t *s_tilde, int max_kept,
                              const int32_t *idx, const int64_t *off, const void *A,
                              const double *b, int iterations, const void *x_init,
                              void *x_map, int *fault, hipStream_t s)
{
    static const hipError_t attr = allow_big_lds((const void *)gs_kernel<TA, TX, UNIT>);
    if (attr != hipSuccess)
        return attr;
    const size_t lds = gs_lds_fixed<TA>() + sizeof(double) * (size_t)ld_of(max_kept);
    hipLaunchKernelGGL((gs_kernel<TA, TX, UNIT>), dim3(n_bins), dim3(kGsThreads), lds, s, N,
                       s_tilde, max_kept, idx, off, (const TA *)A, b, iterations,
                       (const TX *)x_init, (TX *)x_map, fault);
    return hipGetLastError();
}

hipError_t launch_gs(int N, int n_bins, const int32_t *s_tilde, int max_kept,
                     const int32_t *idx, const int64_t *off, int precision,
                     int unit_diagonal, const void *A, const double *b, int iterations,
                     const void *x_init, void *x_map, int *fault, hipStream_t s)
{
    if (n_bins == 0)
        return hipSuccess;
    if (precision == DAMAS_PREC_FP64)
        return unit_diagonal
                   ? launch_gs_t<double, double, true>(N, n_bins, s_tilde, max_kept, idx, off,
                                                       A, b, iterations, x_init, x_map, fault, s)
                   : launch_gs_t<double, double, false>(N, n_bins, s_tilde, max_kept, idx, off,
                                                        A, b, iterations, x_init, x_map, fault, s);
    return unit_diagonal
               ? launch_gs_t<float, float, true>(N, n_bins, s_tilde, max_kept, idx, off, A, b,
                                                 iterations, x_init, x_map, fault, s)
               : launch_gs_t<float, float, false>(N, n_bins, s_tilde, max_kept, idx, off, A, b,
                                                  iterations, x_init, x_map, fault, s);
}

} // namespace damas
