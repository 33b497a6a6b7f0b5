// Wavelet-compressed computational grid (Algorithm 1) and the packed layout
// of the per-bin compressed systems.
//
// Algorithm 1 with an interpolating predictor: on an N x N grid,
// J = floor(log2 N) and G^j = {points whose two indices are multiples of
// 2^(J-j)}.  A point first appearing on level j+1 >= 1 is predicted from
// G^j and its wavelet detail is d = b(p) - prediction.  Order 0 (HAAR): the
// lower-left neighbour on G^j.  LINEAR: with h the point's own spacing, the
// mean of its two neighbours at distance h along its odd axis, or of its
// four diagonal neighbours when both axes are odd (bilinear interpolation
// on G^j), a neighbour past the last grid line replaced by its mirror; the
// sums are formed in the order written below, in double.
// G^0 is always kept.  The union over levels is written in ascending grid
// order.
//
// One workgroup (1024 threads) per bin.  Every decision is an exact
// function of b: |b(p) - b(q)| and eps * max|b| are single correctly
// rounded operations and the rest is comparison and integer logic, so no
// operation here may be fused.  Keep-count selection finds the K'-th
// largest |d| exactly by an MSB-first radix select on the IEEE bit pattern
// (order-preserving for non-negative doubles), and breaks ties by grid index.
#include "common.h"

#pragma clang fp contract(off)

namespace damas {

constexpr int kSelThreads = 1024;
constexpr int kSelWaves = kSelThreads / 64;

__device__ inline int finest_level(int N)
{
    int J = 0;
    while ((2 << J) <= N)
        ++J;
    return J;
}

// Level of (ix, iy) and, for level >= 1, the flat index of its parent.
__device__ inline int point_level(int N, int J, int p, int *parent)
{
    int ix = p % N, iy = p / N;
    int vx = ix == 0 ? J : min(__builtin_ctz((unsigned)ix), J);
    int vy = iy == 0 ? J : min(__builtin_ctz((unsigned)iy), J);
    int level = J - min(vx, vy);
    if (level >= 1) {
        int H = 1 << (J - level + 1);
        *parent = (iy / H) * H * N + (ix / H) * H;
    } else {
        *parent = p;
    }
    return level;
}

// |d(p)| as an order-preserving 64-bit key (0 for level-0 points, which are
// flagged through *coarse).
__device__ inline unsigned long long detail_key(const double *bb, int N, int J,
                                                int predictor, int p, bool *coarse)
{
    int q;
    int lv = point_level(N, J, p, &q);
    *coarse = lv == 0;
    if (lv == 0)
        return 0ull;
    double pred;
    if (predictor == DAMAS_PRED_LINEAR) {
        const int ix = p % N, iy = p / N, h = 1 << (J - lv);
        const bool ox = ix % (2 * h) != 0, oy = iy % (2 * h) != 0;
        const int xl = ix - h, xr = ix + h <= N - 1 ? ix + h : ix - h;
        const int yl = iy - h, yr = iy + h <= N - 1 ? iy + h : iy - h;
        if (ox && !oy)
            pred = 0.5 * (bb[iy * N + xl] + bb[iy * N + xr]);
        else if (oy && !ox)
            pred = 0.5 * (bb[yl * N + ix] + bb[yr * N + ix]);
        else
            pred = 0.25 * ((bb[yl * N + xl] + bb[yl * N + xr]) +
                           (bb[yr * N + xl] + bb[yr * N + xr]));
    } else {
        pred = bb[q];
    }
    double d = fabs(bb[p] - pred);
    return __builtin_bit_cast(unsigned long long, d);
}

// Exclusive prefix of a 0/1 flag over the block in thread order, plus the
// block total.  scratch: kSelWaves ints of LDS.
__device__ inline int block_flag_scan(bool flag, int *scratch, int *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    unsigned long long bal = __ballot(flag);
    int in_wave = __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                            __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0));
    if (lane == 0)
        scratch[w] = __popcll(bal);
    __syncthreads();
    int before = 0, all = 0;
    for (int i = 0; i < kSelWaves; ++i) {
        int c = scratch[i];
        before += i < w ? c : 0;
        all += c;
    }
    __syncthreads();
    *total = all;
    return before + in_wave;
}

__global__ __launch_bounds__(kSelThreads) void select_kernel(
    int N, const double *__restrict__ b, int mode, double eps, int predictor,
    const int32_t *__restrict__ keep_count, int32_t *__restrict__ idx,
    int32_t *__restrict__ s_tilde)
{
    __shared__ int scan_scratch[kSelWaves];
    __shared__ unsigned int hist[256];
    __shared__ double red[kSelWaves];
    __shared__ unsigned long long s_prefix;
    __shared__ int s_need, s_digit, s_above;

    const int f = blockIdx.x;
    const int S = N * N;
    const int J = finest_level(N);
    const double *bb = b + (size_t)f * S;
    int32_t *out = idx + (size_t)f * S;
    const int tid = threadIdx.x;

    // Number of level-0 points and of candidates (levels >= 1).
    const int g0side = (1 << J) < N ? 2 : 1;
    const int n0 = g0side * g0side;
    const int ncand = S - n0;

    // Decide what a candidate needs to be kept.
    // kind 0: keep all; kind 1: |d| >= tau; kind 2: key > pivot, or
    // key == pivot and tie rank < need; kind 3: keep only G^0.
    int kind = 0;
    double tau = 0.0;
    unsigned long long pivot = 0;
    int need = 0;

    if (mode == DAMAS_SEL_EPS_REL) {
        double m = 0.0;
        for (int p = tid; p < S; p += kSelThreads)
            m = fmax(m, fabs(bb[p]));
        for (int o = 32; o > 0; o >>= 1)
            m = fmax(m, __shfl_xor(m, o));
        if ((tid & 63) == 0)
            red[tid >> 6] = m;
        __syncthreads();
        double bmax = 0.0;
        for (int i = 0; i < kSelWaves; ++i)
            bmax = fmax(bmax, red[i]);
        tau = eps * bmax;
        kind = 1;
    } else if (mode == DAMAS_SEL_KEEP_COUNT) {
        int K = keep_count[f];
        int kp = K - n0;
        if (kp <= 0) {
            kind = 3;
        } else if (kp >= ncand) {
            kind = 0;
        } else {
            kind = 2;
            // Radix select of the kp-th largest key, 8 bits at a time.
            if (tid == 0) {
                s_prefix = 0ull;
                s_need = kp;
            }
            for (int shift = 56; shift >= 0; shift -= 8) {
                for (int i = tid; i < 256; i += kSelThreads)
                    hist[i] = 0u;
                __syncthreads();
                const unsigned long long pre = s_prefix;
                const unsigned long long hi_mask =
                    shift == 56 ? 0ull : (~0ull << (shift + 8));
                for (int p = tid; p < S; p += kSelThreads) {
                    bool coarse;
                    unsigned long long key = detail_key(bb, N, J, predictor, p, &coarse);
                    if (!coarse && (key & hi_mask) == pre)
                        atomicAdd(&hist[(key >> shift) & 255u], 1u);
                }
                __syncthreads();
                if (tid < 64) {
                    // Descending digits: lane l owns digits 255-4l .. 252-4l.
                    unsigned int c[4], sum = 0;
                    for (int q = 0; q < 4; ++q) {
                        c[q] = hist[255 - (4 * tid + q)];
                        sum += c[q];
                    }
                    unsigned int incl = sum;
                    for (int o = 1; o < 64; o <<= 1) {
                        unsigned int v = __shfl_up(incl, o);
                        if (tid >= o)
                            incl += v;
                    }
                    unsigned int excl = incl - sum;
                    const unsigned int nd = (unsigned int)s_need;
                    unsigned int run = excl;
                    for (int q = 0; q < 4; ++q) {
                        if (run < nd && nd <= run + c[q]) {
                            s_digit = 255 - (4 * tid + q);
                            s_above = (int)run;
                        }
                        run += c[q];
                    }
                }
                __syncthreads();
                if (tid == 0) {
                    s_prefix |= (unsigned long long)s_digit << shift;
                    s_need -= s_above;
                }
                __syncthreads();
            }
            pivot = s_prefix;
            need = s_need;
        }
    }

    // Compaction in ascending grid order, 1024 points per round.
    int written = 0, ties_seen = 0;
    for (int base = 0; base < S; base += kSelThreads) {
        const int p = base + tid;
        bool keep = false, tie = false;
        if (p < S) {
            bool coarse;
            unsigned long long key = detail_key(bb, N, J, predictor, p, &coarse);
            if (coarse || kind == 0) {
                keep = true;
            } else if (kind == 1) {
                keep = __builtin_bit_cast(double, key) >= tau;
            } else if (kind == 2) {
                keep = key > pivot;
                tie = key == pivot;
            }
        }
        if (kind == 2) {
            int nt;
            int rank = ties_seen + block_flag_scan(tie, scan_scratch, &nt);
            ties_seen += nt;
            if (tie && rank < need)
                keep = true;
        }
        int nk;
        int pos = written + block_flag_scan(keep, scan_scratch, &nk);
        if (keep)
            out[pos] = p;
        written += nk;
    }
    if (tid == 0)
        s_tilde[f] = written;
}

// Packed layout: off[f] = sum_{g<f} ld(s_tilde[g])^2, off[n_bins] = total.
// A bin that kept more than max_kept points, or whose system would end past
// `capacity` elements, gets s_tilde = 0 (later steps skip it) and raises the
// fault word.  One workgroup: counts are staged in LDS and one thread runs
// the (short) prefix sum.
constexpr int kLayoutChunk = 4096;

__global__ __launch_bounds__(1024) void layout_kernel(
    int n_bins, int32_t *__restrict__ s_tilde, int max_kept, int64_t capacity,
    int64_t *__restrict__ off, int *fault)
{
    __shared__ int32_t st[kLayoutChunk];
    __shared__ int64_t of[kLayoutChunk];
    __shared__ int64_t carry;
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) {
        carry = 0;
        bad = 0;
    }
    for (int base = 0; base < n_bins; base += kLayoutChunk) {
        const int n = min(kLayoutChunk, n_bins - base);
        __syncthreads();
        for (int i = tid; i < n; i += 1024)
            st[i] = s_tilde[base + i];
        __syncthreads();
        if (tid == 0) {
            int64_t run = carry;
            for (int i = 0; i < n; ++i) {
                const int64_t l = ld_of(st[i]);
                int64_t sz = l * l;
                if (st[i] > max_kept || run + sz > capacity) {
                    st[i] = -1;
                    sz = 0;
                    bad = 1;
                }
                of[i] = run;
                run += sz;
            }
            carry = run;
        }
        __syncthreads();
        for (int i = tid; i < n; i += 1024) {
            off[base + i] = of[i];
            if (st[i] < 0)
                s_tilde[base + i] = 0;
        }
    }
    __syncthreads();
    if (tid == 0) {
        off[n_bins] = carry;
        if (bad)
            atomicOr(fault, 8);
    }
}

hipError_t launch_select(int N, int n_bins, const double *b, int mode,
                         double eps, int predictor, const int32_t *keep_count, int32_t *idx,
                         int32_t *s_tilde, hipStream_t s)
{
    if (n_bins == 0)
        return hipSuccess;
    hipLaunchKernelGGL(select_kernel, dim3(n_bins), dim3(kSelThreads), 0, s, N,
                       b, mode, eps, predictor, keep_count, idx, s_tilde);
    return hipGetLastError();
}

hipError_t launch_layout(int n_bins, int32_t *s_tilde, int max_kept,
                         int64_t capacity, int64_t *off, int *fault,
                         hipStream_t s)
{
    hipLaunchKernelGGL(layout_kernel, dim3(1), dim3(1024), 0, s, n_bins,
                       s_tilde, max_kept, capacity, off, fault);
    return hipGetLastError();
}

} // namespace damas
