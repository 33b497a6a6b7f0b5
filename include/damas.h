/*
 * damas.h -- C ABI of the MI355X (gfx950) library for DAMAS on a
 * wavelet-compressed computational grid (W. Ma, X. Liu, "Improving the
 * Efficiency of DAMAS for Sound Source Localization via Wavelet Compression
 * Computational Grid").
 *
 * The path, per frequency bin f:
 *   1. delay-and-sum map  b_n = e_n^H C_f e_n / M^2 at every grid point
 *      (section "Beamforming", Eq. dirty_map_1);
 *   2. Algorithm 1: wavelet detail of b on nested dyadic grids, threshold,
 *      kept set G>= (section "Wavelet Compression Computational Grid");
 *   3. point-spread matrix over the kept points,
 *      A_ij = |e_i^H e_j|^2 / M^2 (section "DAMAS", PSF and Eq. Axb);
 *   4. non-negative Gauss-Seidel sweeps on A~ x~ = b~ (section "DAMAS",
 *      the DAMAS iteration, and Eq. Axb_CG), x = 0 off the kept set.
 *
 * Conventions shared by every call.
 *  - Return value: DAMAS_OK (0) or a negative DAMAS_E* code.  No C++
 *    exception crosses this boundary.  damas_last_error() describes the most
 *    recent failure of the calling thread.
 *  - Arguments are validated on the host before any device work; when
 *    validation fails nothing is launched and no output is written.  After a
 *    device error (DAMAS_EDEVICE) outputs are undefined.
 *  - "device" pointers are HIP device allocations on the current device
 *    (for example torch tensors' data_ptr()); "host" pointers are ordinary
 *    memory.  The library never frees memory it did not allocate and keeps
 *    no pointer to caller memory after a call returns (asynchronous calls:
 *    after the enqueued work completes).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls that take a stream only enqueue work on it and return.
 *  - Grid indexing: point n = iy*N + ix, ix along x, both 0-based; the scan
 *    plane is z = z0 with x = x0 + ix (x1-x0)/(N-1), y likewise, end points
 *    included (section "Beamforming": S = N x N equidistant points).
 *  - Complex numbers are interleaved (re, im) pairs of doubles.
 *  - Steering component of microphone m at point r: exp(-i k |r - r_m|),
 *    k = 2 pi f / c, unit magnitude, used both for the beamformer and for
 *    the source model, so A is symmetric with unit diagonal.
 */
#ifndef DAMAS_H
#define DAMAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------- */
#define DAMAS_OK 0
#define DAMAS_EINVAL (-1)    /* invalid argument                          */
#define DAMAS_ENOMEM (-2)    /* device or host allocation failed          */
#define DAMAS_EDEVICE (-3)   /* HIP runtime or kernel error               */
#define DAMAS_EADMIT (-4)    /* request can never fit the memory budget   */
#define DAMAS_EBUSY (-5)     /* queue full, or a resource in use (graph)  */
#define DAMAS_ETIMEDOUT (-6) /* wait timed out                            */
#define DAMAS_ECAPACITY (-7) /* a device-side capacity bound was exceeded */

/* ---- grid-compression modes (Algorithm 1) --------------------------- */
#define DAMAS_SEL_KEEP_ALL 0   /* no compression: every grid point        */
#define DAMAS_SEL_EPS_REL 1    /* keep level-0 points and every point whose
                                  wavelet detail |d| >= eps * max_n |b_n|   */
#define DAMAS_SEL_KEEP_COUNT 2 /* keep level-0 points plus the points of
                                  largest |d| (ties: lower grid index first)
                                  up to keep_count points in total          */
#define DAMAS_SEL_KEEP_FRAC 3  /* the KEEP_COUNT rule with the same count for
                                  every bin, ceil(keep_frac * N*N) (the
                                  ceiling of that double product; level-0
                                  points included); whole-path solves and
                                  the server only, the step-level
                                  damas_select takes counts                */

/* ---- predictors of Algorithm 1's interpolating wavelet ------------- */
#define DAMAS_PRED_HAAR 0   /* order 0: the lower-left neighbour on G^j     */
#define DAMAS_PRED_LINEAR 1 /* linear: with h the point's own spacing, the
                               mean of its two neighbours at distance h
                               along its odd axis, or of its four diagonal
                               neighbours when both axes are odd; a
                               neighbour past the last grid line replaced by
                               its mirror; 0.5 (a + b) and
                               0.25 ((a + b) + (c + d)) in double           */

/* ---- arithmetic of the compressed system ---------------------------- */
#define DAMAS_PREC_FP64 0 /* A stored in double                          */
#define DAMAS_PREC_FP32 1 /* A stored in float (half the bytes the sweeps
                             stream); steering, the PSF products, b, x and
                             the row residuals stay double; the partial
                             residual sums over a wave's share of a strip
                             are accumulated in FP32                       */
#define DAMAS_PREC_BF16 2 /* bulk sweeps on A stored in bf16 (a quarter of
                             the bytes of double), built on the bf16 matrix
                             cores with FP32 accumulation; then the last
                             refine_sweeps sweeps on an FP32 copy of A built
                             as for DAMAS_PREC_FP32.  x maps are float;
                             the sweep state and row residuals stay
                             double, partial sums FP32 as above            */

/* ---- steering forms (section "Beamforming" v_m, section "DAMAS" g_m) ---- */
#define DAMAS_STEER_UNIT 0  /* v_m(r) = g_m(r) = exp(-i k |r - r_m|): A is
                               symmetric with A_nn = 1 (the default)        */
#define DAMAS_STEER_PAPER 1 /* the paper's pair: beamformer
                               v_m(r) = (|r - r_m| / |r|) exp(-i k |r - r_m|),
                               source model
                               g_m(r) = (|r| / |r - r_m|) exp(-i k |r - r_m|),
                               |r| the distance to the array centre; A is
                               not symmetric, A_nn = 1                      */

/* ---- per-bin precision policy of a whole-path solve ------------------ */
#define DAMAS_POLICY_AUTO 0  /* per bin, the storage of A that keeps the
                                iterate within about 1e-4 of the FP64
                                iteration, chosen on the device from the
                                bin's mean PSF row sum over its kept points,
                                rho = (1/S~) sum_ij A_ij (about the kept
                                points inside one main lobe):
                                - DAMAS_PREC_FP32: a bin with rho > rho_wide
                                  (and at most damas_wide_capacity() kept)
                                  is "wide": A is held as float hi plus a
                                  bf16 residual lo = bf16(A - hi), and its
                                  sweeps form every residual from hi + lo in
                                  double (A to about 2^-33);
                                - DAMAS_PREC_BF16: a bin with rho > rho_f32
                                  runs every sweep on the FP32 system (wide
                                  above rho_wide as for FP32), the others
                                  the bf16 bulk plus refine_sweeps FP32
                                  sweeps;
                                - DAMAS_PREC_FP64: no classes.            */
#define DAMAS_POLICY_FIXED 1 /* every bin at `precision` as stated       */
#define DAMAS_RHO_WIDE_DEFAULT 100.0
#define DAMAS_RHO_F32_DEFAULT 12.0

/* Scan geometry (section "Beamforming").  The struct itself is host memory;
 * `mic` is a DEVICE pointer to M x 3 doubles (metres, row-major, array in
 * the plane z = 0 centred on the origin). */
typedef struct {
    int32_t M;
    const double *mic;
    int32_t N;
    double x0, x1, y0, y1, z0;
    double c; /* speed of sound, m/s */
} damas_geometry;

/* ---- helpers (host only, no device work) ----------------------------- */

/* Message for a status code. */
const char *damas_strerror(int code);

/* Description of the calling thread's last failure ("" if none). */
const char *damas_last_error(void);

/* Leading dimension (row stride, in elements) of a compressed system with
 * s_tilde unknowns: s_tilde rounded up to a multiple of 32 (so float rows
 * start on whole 128-byte lines).  Rows and the columns j >= s_tilde of the
 * padding are zero. */
int64_t damas_ld(int32_t s_tilde);

/* The largest max_kept the sweeps accept at `precision` (DAMAS_PREC_*):
 * the unknowns one sweep workgroup holds in LDS beside its partial sums
 * and hand-over blocks, whichever of the one-workgroup and cooperative
 * kernels needs more; for DAMAS_PREC_BF16 also within what the FP32
 * refinement sweeps hold.  0 for an unknown precision.  Host only, no
 * device work. */
int32_t damas_gs_capacity(int32_t precision);

/* The largest kept count of a wide bin (DAMAS_POLICY_AUTO): the unknowns a
 * sweep workgroup holds in LDS beside the wide (hi + lo) hand-over blocks.
 * A bin above it stays narrow.  Host only. */
int32_t damas_wide_capacity(void);

/* Number of points on the coarsest grid G^0 of Algorithm 1 for an N x N
 * grid; every compressed grid keeps them, so KEEP_COUNT keeps
 * clamp(keep_count, |G^0|, N*N) points. */
int32_t damas_coarse_count(int32_t N);

/* ---- step-level calls (device pointers, enqueue on `stream`) --------- */

/* The step before step 1, Eq. (1): the cross-spectral matrix of each bin
 * as the average of p p^H over its snapshots,
 *   csm[f][m][q] = (1/n_snap) sum_k p_{f,k}[m] conj(p_{f,k}[q]).
 *   snap  device, n_bins x n_snap x M complex (snapshot k of bin f: its M
 *         microphone spectra, contiguous), interleaved (re, im) doubles
 *   csm   device, n_bins x M x M complex, row-major, interleaved (output)
 * Products and sums in double precision on the FP64 matrix cores.  Each
 * entry with m < q is written with its conjugate at (q, m) and the diagonal
 * with a zero imaginary part, so csm is exactly Hermitian.
 * DAMAS_EINVAL: M outside [1, 8192], n_snap < 1, n_bins < 0, or a NULL
 * pointer with n_bins > 0.  n_bins = 0 enqueues nothing. */
int damas_csm(int32_t M, int32_t n_snap, int32_t n_bins, const double *snap, double *csm,
              void *stream);

/* Step 1, Eq. dirty_map_1: b[f*S + n] = Re(e_n^H C_f e_n) / M^2 for every
 * bin f < n_bins and grid point n < S = N*N.
 *   freq  device, n_bins doubles (Hz, > 0)
 *   csm   device, n_bins x M x M complex (row-major, Hermitian)
 *   b     device, n_bins x S doubles (output)
 * Phase k|r - r_m| and all sums in double precision. */
int damas_das_map(const damas_geometry *g, int32_t n_bins, const double *freq,
                  const double *csm, double *b, void *stream);

/* Step 2, Algorithm 1 with the order-0 interpolating predictor: per bin,
 * J = floor(log2 N); grid G^j holds the points whose indices are both
 * multiples of 2^(J-j); a point first appearing on level j+1 >= 1 has
 * detail d = b(p) - b(parent), parent = its lower-left neighbour on G^j.
 * Kept points are written in ascending grid order.
 *   b           device, n_bins x S doubles
 *   keep_count  device, n_bins int32 (KEEP_COUNT only; may be NULL otherwise)
 *   idx         device, n_bins x S int32 (output; entries past s_tilde[f]
 *               are left untouched)
 *   s_tilde     device, n_bins int32 (output: kept points per bin)
 * The decisions are exact functions of b: the same b gives the same idx on
 * any IEEE machine (no fused operations in the comparisons). */
int damas_select(int32_t N, int32_t n_bins, const double *b, int32_t mode,
                 double eps, const int32_t *keep_count, int32_t *idx,
                 int32_t *s_tilde, void *stream);

/* damas_select with a choice of predictor (DAMAS_PRED_*; the detail is
 * d = b(p) - prediction from G^j), the same arguments otherwise;
 * DAMAS_EINVAL for an unknown predictor.  damas_select is this call with
 * DAMAS_PRED_HAAR. */
int damas_select_pred(int32_t N, int32_t n_bins, const double *b, int32_t mode,
                      double eps, int32_t predictor, const int32_t *keep_count,
                      int32_t *idx, int32_t *s_tilde, void *stream);

/* Packed layout of the per-bin compressed systems: off[f] = sum over g < f
 * of damas_ld(s_tilde[g])^2, off[n_bins] = total elements.
 *   s_tilde   device, n_bins int32 (in/out)
 *   max_kept  host bound on s_tilde[f]
 *   capacity  elements available in the A arena
 *   off       device, n_bins + 1 int64 (output)
 * A bin with s_tilde[f] > max_kept, or whose system would end beyond
 * `capacity`, is set to s_tilde[f] = 0 (the later steps then skip it and
 * its map is all zero) and damas_check reports DAMAS_ECAPACITY. */
int damas_layout(int32_t n_bins, int32_t *s_tilde, int32_t max_kept,
                 int64_t capacity, int64_t *off, void *stream);

/* Steering rows of the kept points (section "Beamforming", v_m(r) with unit
 * magnitude), in double: for bin f and i < s_tilde[f], with
 * n = idx[f*S + i],
 *   E[f*e_stride + i*2M + m]     = cos(k |r_n - r_m|)
 *   E[f*e_stride + i*2M + M + m] = -sin(k |r_n - r_m|)
 * rows s_tilde[f] <= i < damas_ld(s_tilde[f]) are zero.
 *   idx      device, n_bins x S int32, as written by damas_select
 *   s_tilde  device, n_bins int32; bins above max_kept are skipped and
 *            raise the fault that damas_check reports
 *   E        device, n_bins x e_stride doubles (output)
 *   e_stride elements per bin, >= damas_ld(max_kept) * 2M when n_bins > 1 */
int damas_steer(const damas_geometry *g, int32_t n_bins, const double *freq,
                const int32_t *idx, const int32_t *s_tilde, int32_t max_kept,
                double *E, int64_t e_stride, void *stream);

/* damas_das_map with a steering form (DAMAS_STEER_*) and, with
 * diag_removal = 1, the CSM diagonal removed (section "Beamforming": the
 * m = m' terms dropped, the map normalised by M^2 - M):
 *   b[f*S + n] = Re(v_n^H C_f v_n - diag * sum_m |v_nm|^2 C_f,mm) /
 *                (M^2 - diag * M),
 * v_n the unit steering vector or the paper's beamformer vector.  Same
 * arguments and errors as damas_das_map otherwise. */
int damas_das_map_ex(const damas_geometry *g, int32_t n_bins, const double *freq,
                     const double *csm, int32_t steering, int32_t diag_removal, double *b,
                     void *stream);

/* damas_steer with a steering form: DAMAS_STEER_UNIT as damas_steer;
 * DAMAS_STEER_PAPER writes two row sets per bin, rows [0, ld) the
 * beamformer vectors v = (|r - r_m| / |r|) e and rows [ld, 2 ld) the
 * propagation vectors g = (|r| / |r - r_m|) e (ld = damas_ld(s_tilde[f]);
 * e_stride >= 2 damas_ld(max_kept) 2M when n_bins > 1). */
int damas_steer_ex(const damas_geometry *g, int32_t n_bins, const double *freq,
                   const int32_t *idx, const int32_t *s_tilde, int32_t max_kept,
                   int32_t steering, double *E, int64_t e_stride, void *stream);

/* damas_psf with a steering form and diagonal removal, from the rows of
 * damas_steer_ex.  DAMAS_STEER_UNIT: A as damas_psf, symmetric.
 * DAMAS_STEER_PAPER: A is not symmetric and the arena holds it TRANSPOSED,
 * row r = source point, column c = beam point:
 *   A_f[r*ld + c] = PSF(r_c | r_r) = |v_c^H g_r|^2 / M^2,
 * which is the layout damas_gs reads (a strip of 64 columns holds the
 * coefficients of 64 rows of A x).  diag_removal = 1: every entry becomes
 * (|.|^2 - sum_m |v_m|^2 |g_m|^2) / (M^2 - M) (M for unit steering), the
 * diagonal stays 1 exactly and padding 0. */
int damas_psf_ex(int32_t M, int32_t n_bins, const int32_t *s_tilde, int32_t max_kept,
                 int32_t precision, int32_t steering, int32_t diag_removal, const double *E,
                 int64_t e_stride, const int64_t *off, void *A, void *stream);

/* Half-width of a bf16 steering row: M rounded up to 16. */
int32_t damas_mp(int32_t M);

/* Steering rows of the kept points in bf16 (round to nearest even of the
 * double values), for damas_psf_bf16: for bin f and i < s_tilde[f],
 *   E16[f*e16_stride + i*2MP + m]      = bf16(cos(k |r_n - r_m|))
 *   E16[f*e16_stride + i*2MP + MP + m] = bf16(-sin(k |r_n - r_m|))
 * with MP = damas_mp(M); entries m >= M and rows s_tilde[f] <= i <
 * damas_ld(s_tilde[f]) are zero.  Phases in double as for damas_steer.
 *   E16       device, n_bins x e16_stride uint16 (bf16 bit patterns)
 *   e16_stride elements per bin, >= damas_ld(max_kept) * 2MP when n_bins > 1 */
int damas_steer_bf16(const damas_geometry *g, int32_t n_bins, const double *freq,
                     const int32_t *idx, const int32_t *s_tilde, int32_t max_kept,
                     uint16_t *E16, int64_t e16_stride, void *stream);

/* Step 3 on the bf16 matrix cores (section "DAMAS", PSF):
 *   A16_f[i*ld + j] = bf16(((Re G_ij)^2 + (Im G_ij)^2) / M^2),
 *   G_ij = sum_m conj(e_im) e_jm over the bf16 steering rows E16
 * (damas_steer_bf16), both real products with FP32 accumulation, the value
 * rounded once to bf16 (nearest even).  Same packed layout as damas_psf
 * (A16_f = A16 + off[f], ld = damas_ld(s_tilde[f])); A16 is bitwise
 * symmetric, A_ii = 1 exactly, padding rows and columns are 0.
 *   A16  device, bf16 bit patterns (output) */
int damas_psf_bf16(int32_t M, int32_t n_bins, const int32_t *s_tilde,
                   int32_t max_kept, const uint16_t *E16, int64_t e16_stride,
                   const int64_t *off, uint16_t *A16, void *stream);

/* Step 3 (section "DAMAS", PSF): A_f[i*ld + j] = |sum_m conj(e_im) e_jm|^2 / M^2
 * over the kept points of bin f, ld = damas_ld(s_tilde[f]), A_f = A + off[f].
 * Built from the double steering rows E (damas_steer) as two real products
 * on the f64 matrix cores and rounded once to the storage type (double for
 * DAMAS_PREC_FP64, float for DAMAS_PREC_FP32).  Every off-diagonal value is
 * computed once and written to (i,j) and (j,i), so A is bitwise symmetric;
 * A_ii = 1 exactly (unit-magnitude steering); padding rows and columns
 * are 0. */
int damas_psf(int32_t M, int32_t n_bins, const int32_t *s_tilde,
              int32_t max_kept, int32_t precision, const double *E,
              int64_t e_stride, const int64_t *off, void *A, void *stream);

/* Step 4 (section "DAMAS", the DAMAS iteration): for bin f, with
 * b~_i = b[f*S + idx[f*S + i]], x~ starting at x_init[f*S + idx[..]] (or 0
 * when x_init is NULL), `iterations` full sweeps over i = 0 .. s_tilde-1:
 *   r_i = sum_j A_ij x_j - b~_i  (x_j already updated for j < i)
 *   x_i = max(x_i - r_i / A_ii, 0)
 * then x_map[f*S + n] = x~_i at n = idx[f*S + i] and 0 at every other n.
 *   A       device arena of damas_psf's layout (element type by precision:
 *           double, float, or bf16 bit patterns for DAMAS_PREC_BF16)
 *   b       device, n_bins x S doubles
 *   x_init  device, n_bins x S (double for FP64, float otherwise), or NULL;
 *           it may be the same buffer as x_map (each bin reads its x_init
 *           before it writes its x_map)
 *   x_map   device, n_bins x S, same type (output)
 *   unit_diagonal  non-zero promises A_ii = 1 for every kept row (true of
 *                  damas_psf's output); the sweeps then skip the scaling by
 *                  1 / A_ii.  Zero accepts any positive diagonal.
 * A must be symmetric (as the PSF matrix is).  The sweep state x~, b~ and
 * the row residuals are double at every precision; the partial sums a
 * stream wave forms over its share of a strip are FP32 for a float or bf16
 * A, double for a double A.  max_kept may not exceed
 * damas_gs_capacity(precision).  One workgroup owns one bin for all its
 * sweeps; bins run concurrently (the context's solves may also split a
 * long bin over several workgroups). */
int damas_gs(int32_t N, int32_t n_bins, const int32_t *s_tilde,
             int32_t max_kept, const int32_t *idx, const int64_t *off,
             int32_t precision, int32_t unit_diagonal, const void *A,
             const double *b, int32_t iterations, const void *x_init,
             void *x_map, void *stream);

/* ---- the whole path -------------------------------------------------- */

typedef struct damas_ctx damas_ctx;

/* A context owns the device workspace (kept points, steering rows, the
 * packed A arena), grown on demand and reused across calls, for one device.
 * Not thread-safe.  damas_ctx_create(device, out) is damas_ctx_create_ex
 * with every option at its default. */
int damas_ctx_create(int32_t device, damas_ctx **out);
void damas_ctx_destroy(damas_ctx *ctx);

/* Options of a context (damas_ctx_create_ex; host memory, read during the
 * call; tune_cache is copied). */
typedef struct {
    int32_t device;          /* HIP device ordinal                          */
    uint64_t hbm_budget;     /* bytes the context's workspace may hold; a
                                solve that would grow it beyond fails with
                                DAMAS_EADMIT, its outputs undefined (0: no
                                limit; damas_query_footprint bounds a
                                solve's need)                              */
    const char *tune_cache;  /* path of a text file of autotune choices, or
                                NULL: damas_ctx_autotune first looks its
                                problem up there (and applies the stored
                                choice without trial solves), else tunes
                                and appends the choice; the file is read
                                at creation, and lines that do not parse
                                or hold knobs damas_ctx_set_schedule would
                                refuse are skipped                         */
    int32_t deterministic;   /* 1: sweeps run one workgroup per bin (no
                                cooperative schedule), so results depend
                                only on the inputs, not on tuning or on
                                the device's compute-unit count;
                                damas_ctx_set_coop then accepts only 0     */
} damas_ctx_opts;
int damas_ctx_create_ex(const damas_ctx_opts *opts, damas_ctx **out);

/* Description of the last failure of a call made on this context, from any
 * thread ("" if none; NULL ctx: ""); the text is copied to storage of the
 * calling thread, valid until that thread's next call to this function. */
const char *damas_ctx_last_error(const damas_ctx *ctx);

/* Timing of the phases of a solve: when enabled, each damas_solve_dev
 * records HIP events on the solve's stream around
 *   DAMAS_PHASE_SWEEPS  its Gauss-Seidel launch(es) (bulk and refinement),
 *   DAMAS_PHASE_SYSTEM  its steering and PSF launches (the system build),
 * once per batched solve or once per bin of a plain solve.
 * damas_ctx_phase_time returns the summed milliseconds and count of the
 * recorded intervals of one phase (it synchronises on them) and clears that
 * phase's record; damas_ctx_gs_time is the sweeps phase. */
#define DAMAS_PHASE_SWEEPS 0
#define DAMAS_PHASE_SYSTEM 1
#define DAMAS_PHASES 2
int damas_ctx_set_timing(damas_ctx *ctx, int32_t enabled);
int damas_ctx_phase_time(damas_ctx *ctx, int32_t phase, double *ms, int64_t *launches);
int damas_ctx_gs_time(damas_ctx *ctx, double *ms, int64_t *launches);

/* Cooperative sweeps: in a batched solve whose kept counts the host knows
 * (KEEP_ALL, KEEP_COUNT), bins with long strips get several workgroups that
 * share each sweep's sums (one owner runs the rows; helpers sum slices of
 * every strip and exchange through device memory), so few or uneven bins
 * still use the whole chip.  The same iteration; only the summation order
 * of each residual changes.  max_workgroups bounds the workgroups one solve
 * launches: -1 (default) what the device holds at once, 0 never cooperate,
 * n > 0 at most n (several contexts sharing a device at once should split
 * it).  Cooperation is used only where it helps (at least 320 rows per
 * workgroup and three tiles per bin). */
int damas_ctx_set_coop(damas_ctx *ctx, int32_t max_workgroups);

/* Workgroups of the context's last sweep launch (the bins' count when no
 * bin cooperated). */
int damas_ctx_last_workgroups(const damas_ctx *ctx, int32_t *workgroups);

/* Parameters of a solve (host struct). */
typedef struct damas_params damas_params;

/* Outcome of damas_ctx_autotune. */
typedef struct {
    int32_t coop;            /* cooperative sweeps chosen (1) or not (0)   */
    int32_t coop_min_rows;   /* rows per rank at least                     */
    double coop_split;       /* bins above coop_split x the mean work per
                                workgroup get ranks                        */
    double coop_overhead;    /* assumed cost per element of a rank
                                relative to a bin alone (schedule choice) */
    double best_ms_per_sweep;    /* sweep time of the choice              */
    double default_ms_per_sweep; /* of the untuned knobs                  */
    int32_t candidates_timed;    /* distinct schedules timed              */
    int32_t coop_floor_rows;     /* cost model of a bin's (or a rank's)
                                    tile: max(floor, rows it sums), so that
                                    short bins, bound by the row chain, are
                                    not under-weighted; 0: rows alone     */
    double wide_cost;            /* cost per element of a wide bin relative
                                    to a narrow one in the schedule
                                    (DAMAS_POLICY_AUTO)                    */
} damas_tune_result;

struct damas_params {
    int32_t select_mode;       /* DAMAS_SEL_*                               */
    double eps;                /* EPS_REL threshold (relative to max |b|)   */
    const int32_t *keep_count; /* HOST, n_bins int32 (KEEP_COUNT), or NULL:
                                  then keep_count_all applies to every bin  */
    int32_t keep_count_all;
    int32_t iterations;        /* Gauss-Seidel sweeps, >= 0                 */
    int32_t precision;         /* DAMAS_PREC_*                              */
    int32_t batched;           /* 0: one launch per step per bin ("plain");
                                  1: one launch per step for all bins       */
    int32_t max_kept;          /* EPS_REL: host bound on kept points per bin
                                  (0 = N*N); exceeding it fails with
                                  DAMAS_ECAPACITY                           */
    int32_t refine_sweeps;     /* DAMAS_PREC_BF16: how many of the
                                  `iterations` sweeps run last, on the FP32
                                  copy of A (0 .. iterations); ignored
                                  otherwise                                 */
    int32_t predictor;         /* DAMAS_PRED_* of Algorithm 1 (0 = HAAR)    */
    int32_t policy;            /* DAMAS_POLICY_* (0 = AUTO)                 */
    double rho_wide;           /* AUTO: widening threshold (0: default)     */
    double rho_f32;            /* AUTO, BF16: bf16 bulk only at rho <= this
                                  (0: default)                              */
    int32_t steering;          /* DAMAS_STEER_* (0 = UNIT); PAPER needs
                                  FP64 or FP32 precision                    */
    int32_t diag_removal;      /* 1: remove the CSM diagonal from the map
                                  (section "Beamforming") and use the
                                  matching PSF, A = (|v^H g|^2 -
                                  sum_m |v_m|^2 |g_m|^2) / (M^2 - M); the
                                  map may then be negative                  */
    double *power;             /* optional output, n_bins doubles: each
                                  bin's integrated power sum_n x_n (the
                                  paper's Table 1 quantity P), summed in
                                  double from the sweep state in a fixed
                                  order; DEVICE memory for damas_solve_dev
                                  and damas_solve_static, HOST memory for
                                  damas_solve; ignored by the server      */
    double keep_frac;          /* KEEP_FRAC: fraction of the N*N grid
                                  points to keep, in (0, 1]               */
};

/* Storage class of each bin in the context's last batched solve under
 * DAMAS_POLICY_AUTO (0: the solve's precision, 1: every sweep on the FP32
 * system, 2: wide), copied to host `out` (n_bins bytes) after a device
 * synchronisation.  DAMAS_EINVAL if the context holds no classes of that
 * many bins. */
#define DAMAS_CLASS_NARROW 0
#define DAMAS_CLASS_FP32 1
#define DAMAS_CLASS_WIDE 2
int damas_ctx_classes(damas_ctx *ctx, int32_t n_bins, uint8_t *out);

/* Every step for every bin, device-resident, enqueued on `stream`.
 *   freq, csm   device, as for damas_das_map
 *   x_init      device map (n_bins x S, the precision's type) or NULL
 *   x_map       device, n_bins x S, the precision's type (output)
 *   b_map       device, n_bins x S doubles, or NULL (then kept internally)
 *   idx         device, n_bins x S int32, or NULL
 *   s_tilde     device, n_bins int32, or NULL
 * Device-side capacity failures are reported by damas_check(ctx). */
int damas_solve_dev(damas_ctx *ctx, const damas_geometry *g, int32_t n_bins,
                    const double *freq, const double *csm,
                    const damas_params *p, const void *x_init, void *x_map,
                    double *b_map, int32_t *idx, int32_t *s_tilde,
                    void *stream);

/* Synchronise `stream` and report a device-side capacity failure
 * (DAMAS_ECAPACITY) or a HIP error.  Every context has a fault word of its
 * own that only its solves set; damas_check(ctx, ...) reads and clears that
 * word, so a fault in one context (one request of the server) is never
 * charged to, or cleared by, another.  damas_check(NULL, stream) reads and
 * clears the device's word shared by the step-level calls. */
int damas_check(damas_ctx *ctx, void *stream);

/* damas_solve_dev on HOST memory, synchronously: every pointer, g->mic
 * included, is host memory of the sizes damas_solve_dev states.  The call
 * allocates device staging buffers on the context's device, copies the
 * inputs over, runs the solve on the null stream, waits for it (reporting
 * any fault damas_check would) and copies x_map and the non-NULL b_map,
 * idx and s_tilde back; outputs are not written when it fails.  The
 * PCIe copies are part of its time. */
int damas_solve(damas_ctx *ctx, const damas_geometry *g, int32_t n_bins, const double *freq,
                const double *csm, const damas_params *p, const void *x_init, void *x_map,
                double *b_map, int32_t *idx, int32_t *s_tilde);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * batched whole-path solve of damas_solve_dev with no context, its whole
 * workspace (b, kept indices, offsets, steering rows, the A arena and, under
 * DAMAS_POLICY_AUTO, the lo residuals, tile sums and classes, plus a fault
 * word) carved from one static device array per GPU of
 * damas_static_scratch_bytes() bytes (96 MiB), held by the library for the
 * process's lifetime.  The call allocates nothing (no hipMalloc, hipFree or
 * pinned staging) and only enqueues kernels on `stream`, the fault word
 * included (cleared by a kernel, not a memset).
 *   g, freq, csm, x_init, x_map, b_map, idx, s_tilde  as for damas_solve_dev
 *   p           precision DAMAS_PREC_FP64 or DAMAS_PREC_FP32; p->batched,
 *               p->keep_count, p->keep_count_all and refine_sweeps are
 *               ignored; p->max_kept bounds the kept points per bin for
 *               EPS_REL and KEEP_COUNT (0: N*N) and sizes the workspace
 *   keep_count  DEVICE, n_bins int32 (KEEP_COUNT; may be NULL otherwise)
 * Sweeps run one workgroup per bin (no cooperative schedule).  A solve whose
 * workspace exceeds the array fails with DAMAS_EINVAL before any launch
 * (supply b_map, idx and s_tilde, or a smaller max_kept, to shrink it).
 * Device-side faults are reported by damas_check(NULL, stream).  Every call
 * on a device shares that device's array: calls that overlap on one device
 * (concurrent streams or threads) race, and must be serialised by the
 * caller. */
int damas_solve_static(const damas_geometry *g, int32_t n_bins, const double *freq,
                       const double *csm, const damas_params *p, const int32_t *keep_count,
                       const void *x_init, void *x_map, double *b_map, int32_t *idx,
                       int32_t *s_tilde, void *stream);
int64_t damas_static_scratch_bytes(void);

/* Autotuner of the cooperative sweep schedule: times trial solves of this
 * problem (batched, trial_sweeps sweeps each, into a scratch map; for BF16
 * the bulk sweeps on the bf16 system) for one workgroup per bin and for a
 * grid of schedule knobs (minimum rows per rank, split threshold, rank
 * cost; with wide bins under DAMAS_POLICY_AUTO, then their cost factor),
 * timing each distinct schedule once, keeps the fastest on the context for
 * its later solves and reports it.  Under the policy, cooperative batched
 * solves read the bins' classes back before planning (one synchronisation
 * of the solve's stream) so the schedule weighs wide bins by that factor.  Inputs as for damas_solve_dev;
 * synchronises on `stream`. */
int damas_ctx_autotune(damas_ctx *ctx, const damas_geometry *g, int32_t n_bins,
                       const double *freq, const double *csm, const damas_params *p,
                       int32_t trial_sweeps, void *stream, damas_tune_result *out);

/* Apply schedule knobs (the coop .. wide_cost fields of a
 * damas_tune_result, as damas_ctx_autotune reports them; the timing fields
 * are ignored) to the context's later solves, without trial solves.
 * DAMAS_EINVAL for knobs out of range (coop not 0/1, coop_min_rows < 64,
 * coop_split, coop_overhead or wide_cost not > 0, coop_floor_rows < 0). */
int damas_ctx_set_schedule(damas_ctx *ctx, const damas_tune_result *knobs);

/* ---- graphs: one whole-path solve captured, replayed on any stream ------ */

/* Capture the batched launches of damas_solve_dev with these arguments into
 * a HIP graph (after one eager solve that sizes the workspace).  Every
 * replay runs the same launches on the same buffers, so it reads the
 * current contents of freq, csm and x_init: a new CSM in place gives a new
 * solve.  The sweeps replay the schedule the eager solve chose: cooperative
 * (several workgroups per long bin, one launch for the band) when it was,
 * from a copy of the schedule table the graph owns, as kernel nodes carrying
 * the cooperative launch attribute; with per-bin classes the
 * schedule weighs the classes of that eager solve, and a replay whose
 * classes differ (a new CSM that changes the kept sets) is still exact, only
 * balanced for the old ones.  While a graph exists its context refuses
 * solves that would grow the workspace (DAMAS_EBUSY).  The launch sequence
 * holds no memset nodes.  A replay must not run concurrently with other
 * work on the context, nor, when cooperative, with work that would keep its
 * workgroups from being resident together (its bounded waits would then
 * report fault bit 8 through damas_check). */
typedef struct damas_graph damas_graph;
int damas_graph_capture(damas_ctx *ctx, const damas_geometry *g, int32_t n_bins,
                        const double *freq, const double *csm, const damas_params *p,
                        const void *x_init, void *x_map, double *b_map, int32_t *idx,
                        int32_t *s_tilde, damas_graph **out);
int damas_graph_launch(damas_graph *gr, void *stream);
/* Workgroups of the graph's sweep launches (n_bins when one per bin); 0 for
 * NULL. */
int32_t damas_graph_workgroups(const damas_graph *gr);
void damas_graph_destroy(damas_graph *gr);

/* Device bytes a whole-path solve of this shape holds (host only, no device
 * work): inputs (mic, freq, CSM), the x map and s_tilde, and a context's
 * workspace (b, kept indices, offsets, steering rows, the A arena(s)).
 * EPS_REL is sized by params->max_kept (0 = N*N).  The request server
 * admits requests by this figure. */
int damas_query_footprint(int32_t M, int32_t N, int32_t n_bins, const damas_params *p,
                          uint64_t *bytes);

/* ---- request server ---------------------------------------------------- */

/* A server runs whole-path solves submitted from any host thread.  Worker
 * threads, one per stream slot, take requests in arrival order; a request
 * starts when its footprint (damas_query_footprint) fits the HBM budget
 * beside the workspaces the slots hold and the PSF cache (least recently
 * used cache entries are dropped, and idle slots release their workspaces,
 * to make room).  Slots keep their device workspace (the A arenas) between
 * requests.  The PSF cache keeps built systems in HBM, keyed by geometry,
 * frequencies, precision and the kept points of every bin, so a repeated
 * scene skips its steering and PSF launches (the key needs the kept points
 * on the host: one stream synchronisation per cached request).  Batched
 * solves only.  The server is thread-safe.  The slots' sweep launches pass
 * a gate one at a time (each waits on the device for the previous ones), so
 * every cooperative sweep grid has the whole device, while the uploads,
 * system builds and downloads of the other slots overlap it.
 *
 * Batch former (max_batch > 1): a worker that takes a request whose kept
 * counts the host knows (KEEP_ALL, KEEP_COUNT, KEEP_FRAC) also takes up to
 * max_batch - 1 later queued requests with the same precision, sweep counts
 * and policy, whatever their array, grid size or kept counts, while their
 * summed footprints fit the budget, and runs them as one batch: each
 * request's DAS map, selection and system build on its own grid, then one
 * sweep launch over every bin of the batch (cooperative job lists), so small
 * requests share the chip instead of queueing behind each other.  Merged
 * requests bypass the PSF cache, finish together, and share one fault
 * word: a device fault fails every request of its batch. */
typedef struct damas_server damas_server;

typedef struct {
    int32_t device;        /* HIP device ordinal                            */
    uint64_t hbm_budget;   /* bytes the server may hold on the device
                              (workspaces, in-flight inputs and the cache)   */
    uint64_t cache_budget; /* bytes of the PSF cache (0 disables it)         */
    int32_t slots;         /* concurrent requests (streams), >= 1            */
    int32_t max_queue;     /* waiting requests at most (DAMAS_EBUSY beyond)  */
    int32_t max_batch;     /* requests merged into one batch at most (0 or 1:
                              every request runs alone)                      */
} damas_server_opts;

/* One solve request; every pointer is HOST memory.  Inputs are copied at
 * submission.  The outputs are written by the server and must stay valid
 * until damas_wait retires the ticket (or damas_poll reports it done). */
typedef struct {
    int32_t M;
    const double *mic; /* M x 3 */
    int32_t N;
    double x0, x1, y0, y1, z0, c;
    int32_t n_bins;
    const double *freq; /* n_bins */
    const double *csm;  /* n_bins x M x M complex, interleaved */
    damas_params params; /* params.keep_count, if set, is copied too;
                            params.batched is ignored (always batched)    */
    void *x_map;         /* output, n_bins x N*N (double for FP64, else float) */
    int32_t *s_tilde;    /* output, n_bins kept counts, or NULL           */
} damas_request;

/* Timing and outcome of a finished request. */
typedef struct {
    int32_t status;    /* DAMAS_OK or the solve's error code              */
    int32_t cache_hit; /* the systems came from the PSF cache             */
    double queue_ms;   /* submission to start                            */
    double run_ms;     /* start to results on the host                   */
    double total_ms;   /* submission to results on the host              */
} damas_request_info;

typedef struct {
    uint64_t submitted, completed, rejected;
    uint64_t cache_hits, cache_misses;
    uint64_t held_bytes;  /* workspaces and inputs held by the slots       */
    uint64_t cache_bytes; /* bytes in the PSF cache                       */
    int32_t queued, running;
    uint64_t batches;     /* batches run (a request alone is one batch)     */
    uint64_t merged;      /* requests that ran in a batch of two or more    */
} damas_server_stats;

int damas_server_create(const damas_server_opts *o, damas_server **out);

/* Stops the workers after the running requests; waiting requests finish
 * with status DAMAS_EBUSY.  Frees every device buffer of the server and
 * every ticket not yet collected by damas_wait: no other call on the
 * server may run during or after it (collect the tickets first). */
void damas_server_destroy(damas_server *srv);

/* Queue a request.  DAMAS_EINVAL: invalid request (validated as for
 * damas_solve_dev); DAMAS_EADMIT: its footprint exceeds the HBM budget, so
 * it can never run; DAMAS_EBUSY: the queue is full.  On success *ticket
 * identifies the request. */
int damas_submit(damas_server *srv, const damas_request *req, uint64_t *ticket);

/* Wait up to timeout_ms (< 0: no limit) for a request.  Returns the
 * request's status and retires the ticket, DAMAS_ETIMEDOUT if it is still
 * queued or running (the ticket stays valid), DAMAS_EINVAL for an unknown
 * ticket.  `info` (may be NULL) receives its timing. */
int damas_wait(damas_server *srv, uint64_t ticket, int32_t timeout_ms,
               damas_request_info *info);

/* 1 if the request has finished, 0 if it is queued or running, DAMAS_EINVAL
 * for an unknown ticket.  Does not retire the ticket. */
int damas_poll(damas_server *srv, uint64_t ticket);

int damas_server_get_stats(damas_server *srv, damas_server_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* DAMAS_H */
