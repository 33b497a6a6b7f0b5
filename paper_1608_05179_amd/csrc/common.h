// Shared declarations of the HIP library: kernel-side geometry, small
// device helpers and the host launchers of every kernel.  gfx950 only
// (wave64, MFMA, 160 KB LDS per CU).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "damas.h"

namespace damas {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Geometry passed by value to kernels (section "Beamforming").
struct Geom {
    int M;
    const double *mic; // device, M x 3
    int N;
    double x0, dx, y0, dy, z0;
    double c;
};

inline Geom make_geom(const damas_geometry &g)
{
    Geom k;
    k.M = g.M;
    k.mic = g.mic;
    k.N = g.N;
    k.x0 = g.x0;
    k.y0 = g.y0;
    k.dx = g.N > 1 ? (g.x1 - g.x0) / (double)(g.N - 1) : 0.0;
    k.dy = g.N > 1 ? (g.y1 - g.y0) / (double)(g.N - 1) : 0.0;
    k.z0 = g.z0;
    k.c = g.c;
    return k;
}

// bfloat16 storage word (the upper half of an IEEE single).
struct bf16s {
    uint16_t u;
};
__host__ __device__ inline float bf16_to_float(bf16s v)
{
    return __builtin_bit_cast(float, (uint32_t)v.u << 16);
}

// Row stride of a compressed system: s_tilde rounded up to 32 elements.
// Arenas start on 256-byte boundaries and the per-bin offsets are sums of
// ld^2, so every row of a float or double arena starts on a 128-byte line
// and the 64-column piece of a row that a sweep strip reads covers whole
// lines: no line is fetched for a neighbouring strip (with 8-element rows
// three lines in four straddled, and the streamed bands fetched 1.35-1.4
// times their algorithmic bytes).  bf16 rows start on 64-byte halves; 64
// elements would align them too but pad the small cache-resident systems
// out of L2 (measured: no faster on the bf16 sweeps, 11 % slower on 337-row
// bins).
constexpr int kLdAlign = 32;
__host__ __device__ inline int64_t ld_of(int32_t st)
{
    return ((int64_t)st + kLdAlign - 1) & ~(int64_t)(kLdAlign - 1);
}

// Distance from grid point n to microphone m, in double.
__device__ inline double point_mic_dist(const Geom &g, int n, int m)
{
    int ix = n % g.N, iy = n / g.N;
    double px = g.x0 + (double)ix * g.dx;
    double py = g.y0 + (double)iy * g.dy;
    double ddx = px - g.mic[3 * m + 0];
    double ddy = py - g.mic[3 * m + 1];
    double ddz = g.z0 - g.mic[3 * m + 2];
    return sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
}

// Distance from grid point n to the array centre (the origin), in double.
__device__ inline double point_origin_dist(const Geom &g, int n)
{
    int ix = n % g.N, iy = n / g.N;
    double px = g.x0 + (double)ix * g.dx;
    double py = g.y0 + (double)iy * g.dy;
    return sqrt(px * px + py * py + g.z0 * g.z0);
}

// Lane-uniform broadcast of lane `src` (wave64); src must be uniform.
__device__ inline float lane_bcast(float v, int src)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}
__device__ inline double lane_bcast(double v, int src)
{
    long long u = __builtin_bit_cast(long long, v);
    int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), src);
    int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// ---- launchers (each returns the launch status) ------------------------
// fault: device word set non-zero by a kernel that met a capacity violation.

hipError_t launch_csm(int M, int K, int n_bins, const double *snap, double *csm,
                      hipStream_t s);
int csm_upper_blocks(int M);

// steering: DAMAS_STEER_UNIT or DAMAS_STEER_PAPER; diag: remove the CSM
// diagonal.
hipError_t launch_das(const Geom &g, int n_bins, const double *freq,
                      const double *csm, double *b, hipStream_t s,
                      int steering = DAMAS_STEER_UNIT, int diag = 0);

hipError_t launch_select(int N, int n_bins, const double *b, int mode,
                         double eps, int predictor, const int32_t *keep_count, int32_t *idx,
                         int32_t *s_tilde, hipStream_t s);

hipError_t launch_layout(int n_bins, int32_t *s_tilde, int max_kept,
                         int64_t capacity, int64_t *off, int *fault,
                         hipStream_t s);

// Lift the dynamic-LDS limit of a kernel to the whole 160 KB of a CU
// (once per kernel).
hipError_t allow_big_lds(const void *kernel);

// steering DAMAS_STEER_PAPER writes two row sets per bin: the beamformer
// vectors in rows [0, ld), the propagation vectors in rows [ld, 2 ld).
hipError_t launch_steer(const Geom &g, int n_bins, const double *freq,
                        const int32_t *idx, const int32_t *s_tilde,
                        int max_kept, double *E, int64_t e_stride, int *fault,
                        hipStream_t s, int steering = DAMAS_STEER_UNIT);

// Storage classes of a bin (see PsfClassArgs and GsClassArgs).
constexpr int kClsF32 = 1, kClsWide = 2;

// Per-bin storage classes chosen after a float PSF: lo (device, or null)
// receives the bf16 residuals bf16(A - float(A)) of every bin; with cls
// non-null, tsum (device, n_bins x psf_tiles(max_kept) doubles) receives
// the tile sums of A and cls (device, n_bins bytes) the class of each bin
// (kClsWide: mean row sum over the kept points above rho_wide and at most
// wide_cap kept; else kClsF32 above rho_f32; else 0).
struct PsfClassArgs {
    uint16_t *lo = nullptr;
    double *tsum = nullptr;
    uint8_t *cls = nullptr;
    double rho_wide = 0.0, rho_f32 = 0.0;
    int wide_cap = 0;
};
// Tiles of a bin's PSF launch grid: the upper triangle, or every tile for
// the paper's (non-symmetric) pair.
int64_t psf_tiles(int max_kept, int steering = DAMAS_STEER_UNIT);
// steering: the paper's pair stores A transposed (see psf.hip); diag: the
// CSM diagonal removed, A = (|G|^2 - sum |v|^2 |g|^2) / (M^2 - M).
hipError_t launch_psf(int M, int n_bins, const int32_t *s_tilde, int max_kept,
                      int precision, const double *E, int64_t e_stride,
                      const int64_t *off, void *A, int *fault, hipStream_t s,
                      const PsfClassArgs &pc = PsfClassArgs(),
                      int steering = DAMAS_STEER_UNIT, int diag = 0);

// bf16 steering rows (half-width MP = M rounded up to 16) and the PSF on the
// bf16 matrix cores.
int mp_of(int M);
hipError_t launch_steer16(const Geom &g, int n_bins, const double *freq, const int32_t *idx,
                          const int32_t *s_tilde, int max_kept, uint16_t *E, int64_t e_stride,
                          int *fault, hipStream_t s);
hipError_t launch_psf16(int M, int n_bins, const int32_t *s_tilde, int max_kept,
                        const uint16_t *E, int64_t e_stride, const int64_t *off, uint16_t *A,
                        int *fault, hipStream_t s, int diag = 0);

// Per-bin storage classes of a sweep launch: cls (per bin, device, or
// null: every bin of class 0) with kClsF32 = every sweep on the float
// system, kClsWide = every sweep on float hi + bf16 lo; lo (device) the
// bf16 residual arena of wide bins, at the float arena's offsets; iters_cls
// the sweeps of a bin whose class is not 0.
struct GsClassArgs {
    const uint8_t *cls = nullptr;
    const uint16_t *lo = nullptr;
    int iters_cls = 0;
    double *power = nullptr; // device, per bin: sum of x over the bin (output)
    // device, per bin (base, S): where bin f's maps (idx, b, x_init, x_map)
    // start and how many grid points they hold, for a batch of different
    // grids; null: f N^2 and N^2
    const int64_t *map = nullptr;
};

hipError_t launch_gs(int N, int n_bins, const int32_t *s_tilde, int max_kept,
                     const int32_t *idx, const int64_t *off, int precision,
                     int unit_diagonal, const void *A, const double *b, int iterations,
                     const void *x_init, void *x_map, int *fault, hipStream_t s,
                     const GsClassArgs &gc = GsClassArgs());

// Largest kept count of a wide bin (float hi + bf16 lo sweeps).
int gs_wide_capacity();

// Largest s_tilde the sweep kernel holds on chip for a precision.
int gs_max_kept(int precision);

// Cooperative sweeps (several workgroups per bin, several bins per
// workgroup).  tab (device int32): a header (queue length Q, offset of the
// ranges, offset of the jobs), a queue of Q bins that run alone (taken by
// workgroups once their static jobs are done, in queue order), per
// workgroup the [first, end) of its static jobs, then per job the bin, its
// rank and the bin's rank count; a job with ranks > 1 must be the first of
// its workgroup;
// groups_per_wave: the most row groups any stream wave sums per strip;
// streamed: A exceeds kGsStreamBytes (see there);
// ws: gs_coop_ws_bytes of device workspace.  Every bin needs >= 2 tiles.
size_t gs_coop_ws_bytes(int n_bins, int max_kept);
int gs_max_ranks();
int gs_groups_per_wave(int precision, int s_tilde, int ranks);
// Workgroups of the cooperative kernel that can be resident at once (lo:
// with wide bins possible).
int gs_coop_capacity(int precision, int max_kept, bool lo = false);
hipError_t launch_gs_coop(int N, int n_bins, const int32_t *s_tilde, int max_kept,
                          const int32_t *idx, const int64_t *off, int precision,
                          int unit_diagonal, const void *A, const double *b, int iterations,
                          const void *x_init, void *x_map, int *fault, const int32_t *tab,
                          int n_wg, int groups_per_wave, bool streamed, void *ws,
                          const GsClassArgs &gc, hipStream_t s);
// Bytes of A (all bins of a launch) above which the cooperative sweeps
// load it with the non-temporal hint and read each row once per sweep (the
// hand-over rows left out of the strip loads): twice the 256 MB last-level
// cache, so such a band is streamed from HBM every sweep and gains nothing
// from being cached, while a smaller one stays (partly) in cache between
// sweeps, where a second read of the hand-over rows hits in L2.
constexpr double kGsStreamBytes = 512.0 * 1024 * 1024;
// Whether fn is one of the cooperative kernel's instances (graph capture
// turns their cooperative launches into plain kernel nodes).
bool gs_is_coop_kernel(const void *fn);

} // namespace damas
