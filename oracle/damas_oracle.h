/*
 * FP64 CPU oracle of DAMAS on a wavelet-compressed computational grid
 * (W. Ma, X. Liu, "Improving the Efficiency of DAMAS for Sound Source
 * Localization via Wavelet Compression Computational Grid").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no source, header, table or helper with the GPU
 * library, and it never calls it.
 *
 * Every routine is a plain, slow, literal transcription of the paper's
 * definitions in double precision, with sums in ascending index order and
 * no blocking or reordering.  Build with -ffp-contract=off so that no
 * multiply-add is fused behind the reader's back.
 */
#ifndef DAMAS_ORACLE_H
#define DAMAS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Array and scan-grid geometry (section "Beamforming").  Microphones lie in
 * the plane z = 0 with the origin at the array centre; the scan plane is
 * z = z0 with N x N equidistant points, n = iy*N + ix, covering
 * [x0, x1] x [y0, y1] with both end points included. */
typedef struct {
    int M;              /* number of microphones                         */
    const double *mic;  /* M x 3 positions, metres, row-major            */
    int N;              /* grid points per side, S = N*N                 */
    double x0, x1;      /* scan-plane extent along x                     */
    double y0, y1;      /* scan-plane extent along y                     */
    double z0;          /* distance between array plane and scan plane   */
    double c;           /* speed of sound, m/s                           */
} orc_geom;

/* Selection modes for the wavelet-compressed grid. */
enum {
    ORC_SEL_KEEP_ALL = 0,   /* no compression: every grid point            */
    ORC_SEL_EPS_REL = 1,    /* Algorithm 1 with threshold eps * max|b|     */
    ORC_SEL_KEEP_COUNT = 2  /* the K points of largest |d| (G0 included)   */
};

/* Coordinates of grid point n. */
void orc_grid_point(const orc_geom *g, int n, double r[3]);

/* Steering vectors e_nm = exp(-i k |r_n - r_m|), k = 2 pi f / c, for the
 * n_pts grid points listed in pts.  Output e is n_pts x M complex numbers
 * stored as interleaved (re, im) pairs. */
void orc_steering(const orc_geom *g, double freq, int n_pts, const int *pts,
                  double *e);

/* Cross-spectral matrix, Eq. (1): the average over n_snap snapshots of
 * p p^H, C[m][m'] = (1/n_snap) sum_k p_k[m] conj(p_k[m']).  snap is
 * n_snap x M complex (snapshot k's M microphone spectra contiguous),
 * interleaved; csm is M x M complex, row-major, interleaved.  Every entry is
 * its own sum, so C is exactly Hermitian with a real diagonal. */
void orc_csm(int M, int n_snap, const double *snap, double *csm);

/* Delay-and-sum map, Eq. (2): b_n = Re(e_n^H C e_n) / M^2 for every grid
 * point.  csm is M x M complex, row-major, interleaved (re, im). */
void orc_das_map(const orc_geom *g, double freq, const double *csm,
                 double *b);

/* Resolution level of grid point (ix, iy) in the nested dyadic grids G^j of
 * Algorithm 1, and (for level >= 1) its parent on the next-coarser grid,
 * whose value predicts it (order-0 interpolation).  Returns the level. */
int orc_level(int N, int ix, int iy, int *parent_ix, int *parent_iy);

/* Wavelet-compressed grid (Algorithm 1).  Writes the kept grid indices in
 * ascending order to idx (capacity N*N) and returns their number.  detail
 * (nullable, N*N) receives |d(p)| (0 on the coarsest grid).  margin
 * (nullable) receives the relative distance of the closest decision to its
 * threshold: min |(|d| - tau)| / tau for EPS_REL, the relative gap between
 * the K'-th and (K'+1)-th largest |d| for KEEP_COUNT, +inf otherwise. */
int orc_select(int N, const double *b, int mode, double eps, int keep_count,
               int *idx, double *detail, double *margin);

/* Predictors of a point from the next-coarser grid G^(l-1) (Algorithm 1's
 * interpolating wavelet): ORC_PRED_HAAR, the ancestor at the lower-left
 * corner (order 0, what orc_select uses); ORC_PRED_LINEAR, the mean of the
 * two (one odd axis) or four (both odd) neighbours at the point's own
 * spacing, a neighbour past the last grid line replaced by its mirror. */
enum { ORC_PRED_HAAR = 0, ORC_PRED_LINEAR = 1 };
int orc_select_pred(int N, const double *b, int mode, double eps, int keep_count,
                    int predictor, int *idx, double *detail, double *margin);

/* Point-spread matrix over St points, A_ij = |e_i^H e_j|^2 / M^2 (section
 * "DAMAS", PSF definition), from their steering vectors e (St x M complex,
 * interleaved).  A is St x St row-major.  Entries with j >= i are computed
 * and mirrored, so A is exactly symmetric. */
void orc_psf(int M, int St, const double *e, double *A);

/* DAMAS Gauss-Seidel with the non-negativity clamp: iters full sweeps over
 * rows 0..St-1 of A x = b, starting from the values in x, updated in place. */
void orc_gs(int St, const double *A, const double *b, int iters, double *x);

/* ---- options beside the default readings --------------------------- */

/* Steering forms (section "Beamforming", the beamformer vector v, and
 * section "DAMAS", the propagation vector g):
 *  ORC_STEER_UNIT   v_m(r) = g_m(r) = exp(-i k |r - r_m|)  (the default);
 *  ORC_STEER_PAPER  v_m(r) = (|r - r_m| / |r|) exp(-i k |r - r_m|),
 *                   g_m(r) = (|r| / |r - r_m|) exp(-i k |r - r_m|),
 *                   |r| the distance from the point to the array centre. */
enum { ORC_STEER_UNIT = 0, ORC_STEER_PAPER = 1 };

/* Beamformer vectors v (n_pts x M) and propagation vectors w (the paper's
 * g, n_pts x M) of the listed points, complex interleaved; either output
 * may be NULL. */
void orc_steering_form(const orc_geom *g, double freq, int form, int n_pts, const int *pts,
                       double *v, double *w);

/* Delay-and-sum map with a steering form and optional removal of the CSM
 * diagonal (section "Beamforming": diagonal removal is usually applied):
 *   b_n = (v_n^H C v_n - diag * sum_m |v_nm|^2 C_mm) / (M^2 - diag * M). */
void orc_das_map_ex(const orc_geom *g, double freq, const double *csm, int form, int diag,
                    double *b);

/* Point-spread matrix of beamformer vectors v and propagation vectors w
 * (St x M each): A[i][j] = PSF(r_i | r_j), the map at point i of a unit
 * source at point j, with the same diagonal removal as the map:
 *   A[i][j] = (|v_i^H w_j|^2 - diag * sum_m |v_im|^2 |w_jm|^2) / (M^2 - diag M).
 * Every entry is computed on its own (A is not symmetric for the paper's
 * pair). */
void orc_psf_ex(int M, int St, const double *v, const double *w, int diag, double *A);

/* orc_solve_bin with a steering form and diagonal removal. */
int orc_solve_bin_ex(const orc_geom *g, double freq, const double *csm, int form, int diag,
                     int mode, double eps, int keep_count, int iters, const double *x_init,
                     double *b_map, int *idx, double *x_map, double *margin);

/* The whole path for one frequency bin: DAS map, selection, compressed
 * system, sweeps.  x_init (nullable) is a full N*N map whose kept entries
 * start the sweeps (zero otherwise).  Outputs (all nullable except idx):
 * b_map (N*N), idx (N*N capacity), x_map (N*N, zero off the kept set),
 * margin.  Returns the number of kept points, or -1 on allocation failure. */
int orc_solve_bin(const orc_geom *g, double freq, const double *csm,
                  int mode, double eps, int keep_count, int iters,
                  const double *x_init, double *b_map, int *idx,
                  double *x_map, double *margin);

#ifdef __cplusplus
}
#endif
#endif
