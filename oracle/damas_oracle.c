/*
 * FP64 CPU oracle of DAMAS on a wavelet-compressed computational grid.
 *
 * TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares nothing
 * with the GPU library.
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * project's design notes):
 *  - steering: unit-magnitude free-field vectors e_m = exp(-i k |r - r_m|),
 *    used both for the beamformer and for the source model, so A is
 *    symmetric with A_nn = 1;
 *  - wavelet: Algorithm 1 with the order-0 (Haar) interpolating predictor,
 *    i.e. a point on level j+1 is predicted by the value at its lower-left
 *    ancestor on grid G^j; no averaging, no update step;
 *  - threshold: |d| >= eps * max|b| keeps a point (ties kept);
 *  - ordering of the compressed unknowns: ascending original index;
 *  - Gauss-Seidel: rows in ascending order, fixed sweep count, no early stop.
 */
#include "damas_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double ORC_PI = 3.14159265358979323846;

/* ---------------------------------------------------------------------- */
/* Geometry: section "Beamforming" (scan plane of N x N equidistant points). */

void orc_grid_point(const orc_geom *g, int n, double r[3])
{
    int ix = n % g->N;
    int iy = n / g->N;
    double dx = g->N > 1 ? (g->x1 - g->x0) / (double)(g->N - 1) : 0.0;
    double dy = g->N > 1 ? (g->y1 - g->y0) / (double)(g->N - 1) : 0.0;
    r[0] = g->x0 + (double)ix * dx;
    r[1] = g->y0 + (double)iy * dy;
    r[2] = g->z0;
}

static double wavenumber(const orc_geom *g, double freq)
{
    /* k = omega / c0 with omega = 2 pi f (section "Beamforming"). */
    return 2.0 * ORC_PI * freq / g->c;
}

/* e_m(r) = exp(-i k |r - r_m|), the unit-magnitude steering component. */
static void steer_point(const orc_geom *g, double k, const double r[3],
                        double *e)
{
    for (int m = 0; m < g->M; ++m) {
        double ddx = r[0] - g->mic[3 * m + 0];
        double ddy = r[1] - g->mic[3 * m + 1];
        double ddz = r[2] - g->mic[3 * m + 2];
        double d = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
        double ph = k * d;
        e[2 * m + 0] = cos(ph);
        e[2 * m + 1] = -sin(ph);
    }
}

void orc_steering(const orc_geom *g, double freq, int n_pts, const int *pts,
                  double *e)
{
    double k = wavenumber(g, freq);
    for (int p = 0; p < n_pts; ++p) {
        double r[3];
        orc_grid_point(g, pts[p], r);
        steer_point(g, k, r, e + (size_t)2 * g->M * p);
    }
}

/* ---------------------------------------------------------------------- */
/* Cross-spectral matrix, Eq. (1): C = (1/K) sum_k p_k p_k^H.              */

void orc_csm(int M, int n_snap, const double *snap, double *csm)
{
    for (int m = 0; m < M; ++m)
        for (int q = 0; q < M; ++q) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < n_snap; ++k) {
                /* p_k[m] conj(p_k[q]) with p_k[m] = a + ib, p_k[q] = c + id */
                const double a = snap[2 * ((long)k * M + m)];
                const double b = snap[2 * ((long)k * M + m) + 1];
                const double c = snap[2 * ((long)k * M + q)];
                const double d = snap[2 * ((long)k * M + q) + 1];
                re += a * c + b * d;
                im += b * c - a * d;
            }
            csm[2 * ((long)m * M + q)] = re / n_snap;
            csm[2 * ((long)m * M + q) + 1] = im / n_snap;
        }
}

/* ---------------------------------------------------------------------- */
/* Delay-and-sum beamforming, Eq. (2): b(r) = v(r)^H C v(r) / M^2.        */

void orc_das_map(const orc_geom *g, double freq, const double *csm, double *b)
{
    int M = g->M;
    int S = g->N * g->N;
    double k = wavenumber(g, freq);
    double *e = (double *)malloc(sizeof(double) * 2 * (size_t)M);
    for (int n = 0; n < S; ++n) {
        double r[3];
        orc_grid_point(g, n, r);
        steer_point(g, k, r, e);
        /* sum_m sum_m' conj(e_m) C_mm' e_m' ; only the real part survives
         * for a Hermitian C, and the real part is what the map keeps. */
        double acc = 0.0;
        for (int m = 0; m < M; ++m) {
            double er = e[2 * m], ei = -e[2 * m + 1]; /* conj(e_m) */
            for (int mp = 0; mp < M; ++mp) {
                const double *c = csm + 2 * ((size_t)m * M + mp);
                double cr = c[0], ci = c[1];
                double fr = e[2 * mp], fi = e[2 * mp + 1];
                /* (er + i ei) * (cr + i ci) * (fr + i fi), real part */
                double tr = er * cr - ei * ci;
                double ti = er * ci + ei * cr;
                acc += tr * fr - ti * fi;
            }
        }
        b[n] = acc / ((double)M * (double)M);
    }
    free(e);
}

/* ---------------------------------------------------------------------- */
/* Nested dyadic grids of Algorithm 1.                                    */

/* J = floor(log2 N), the finest level (the original grid). */
static int finest_level(int N)
{
    int J = 0;
    while ((2 << J) <= N) /* 2^(J+1) <= N */
        ++J;
    return J;
}

/* Largest e <= cap with 2^e dividing v; v = 0 is divisible by everything. */
static int dyadic_valuation(int v, int cap)
{
    int e = 0;
    if (v == 0)
        return cap;
    while (e < cap && (v % (2 << e)) == 0) /* 2^(e+1) divides v */
        ++e;
    return e;
}

int orc_level(int N, int ix, int iy, int *parent_ix, int *parent_iy)
{
    /* G^j holds the points whose two indices are multiples of 2^(J-j)
     * (the restriction x_k^j = x_{2k}^{j+1} applied J-j times from the
     * finest grid G^J).  A point's level is the smallest j with the point in
     * G^j. */
    int J = finest_level(N);
    int vx = dyadic_valuation(ix, J);
    int vy = dyadic_valuation(iy, J);
    int v = vx < vy ? vx : vy;
    int level = J - v;
    if (level >= 1) {
        /* Predict from G^(level-1): its spacing is H = 2^(J-level+1); the
         * order-0 interpolant takes the ancestor at the lower-left corner. */
        int H = 1 << (J - level + 1);
        *parent_ix = (ix / H) * H;
        *parent_iy = (iy / H) * H;
    } else {
        *parent_ix = ix;
        *parent_iy = iy;
    }
    return level;
}

typedef struct {
    double d;
    int n;
} orc_cand;

/* Order: |d| descending, then grid index ascending. */
static int cand_cmp(const void *a, const void *b)
{
    const orc_cand *x = (const orc_cand *)a;
    const orc_cand *y = (const orc_cand *)b;
    if (x->d > y->d)
        return -1;
    if (x->d < y->d)
        return 1;
    return (x->n > y->n) - (x->n < y->n);
}

/* Linear interpolating prediction of a point of level l >= 1 from
 * G^(l-1): with h the spacing of G^l, the mean of its two neighbours at
 * distance h along its one odd axis, or of its four diagonal neighbours when
 * both axes are odd (bilinear interpolation on the coarser grid).  A
 * neighbour past the last grid line is replaced by its mirror on the other
 * side. */
static double linear_prediction(int N, const double *b, int ix, int iy, int level)
{
    int h = 1 << (finest_level(N) - level);
    int ox = ix % (2 * h) != 0, oy = iy % (2 * h) != 0;
    int xl = ix - h, xr = ix + h <= N - 1 ? ix + h : ix - h;
    int yl = iy - h, yr = iy + h <= N - 1 ? iy + h : iy - h;
    if (ox && !oy)
        return 0.5 * (b[iy * N + xl] + b[iy * N + xr]);
    if (oy && !ox)
        return 0.5 * (b[yl * N + ix] + b[yr * N + ix]);
    return 0.25 * ((b[yl * N + xl] + b[yl * N + xr]) + (b[yr * N + xl] + b[yr * N + xr]));
}

int orc_select(int N, const double *b, int mode, double eps, int keep_count,
               int *idx, double *detail, double *margin)
{
    return orc_select_pred(N, b, mode, eps, keep_count, ORC_PRED_HAAR, idx, detail, margin);
}

int orc_select_pred(int N, const double *b, int mode, double eps, int keep_count,
                    int predictor, int *idx, double *detail, double *margin)
{
    int S = N * N;
    unsigned char *keep = (unsigned char *)calloc((size_t)S, 1);
    double *d = (double *)calloc((size_t)S, sizeof(double));
    int *lvl = (int *)calloc((size_t)S, sizeof(int));
    double mg = INFINITY;

    /* Wavelet coefficient of every point: its value minus the value
     * interpolated from the next-coarser grid (interpolating-wavelet
     * detail).  Coarsest-grid points carry scaling coefficients only. */
    for (int p = 0; p < S; ++p) {
        int ix = p % N, iy = p / N, px, py;
        lvl[p] = orc_level(N, ix, iy, &px, &py);
        if (lvl[p] == 0)
            d[p] = 0.0;
        else if (predictor == ORC_PRED_LINEAR)
            d[p] = fabs(b[p] - linear_prediction(N, b, ix, iy, lvl[p]));
        else
            d[p] = fabs(b[p] - b[py * N + px]);
        if (lvl[p] == 0)
            keep[p] = 1; /* G^0 is always part of the compressed grid */
    }

    if (mode == ORC_SEL_KEEP_ALL) {
        for (int p = 0; p < S; ++p)
            keep[p] = 1;
    } else if (mode == ORC_SEL_EPS_REL) {
        double bmax = 0.0;
        for (int p = 0; p < S; ++p)
            if (fabs(b[p]) > bmax)
                bmax = fabs(b[p]);
        double tau = eps * bmax;
        for (int p = 0; p < S; ++p) {
            if (lvl[p] == 0)
                continue;
            if (d[p] >= tau)
                keep[p] = 1;
            if (tau > 0.0) {
                double r = fabs(d[p] - tau) / tau;
                if (r < mg)
                    mg = r;
            }
        }
    } else { /* ORC_SEL_KEEP_COUNT */
        int n0 = 0, nc = 0;
        for (int p = 0; p < S; ++p)
            n0 += lvl[p] == 0;
        orc_cand *c = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)(S - n0 + 1));
        for (int p = 0; p < S; ++p)
            if (lvl[p] != 0) {
                c[nc].d = d[p];
                c[nc].n = p;
                ++nc;
            }
        qsort(c, (size_t)nc, sizeof(orc_cand), cand_cmp);
        int take = keep_count - n0;
        if (take < 0)
            take = 0;
        if (take > nc)
            take = nc;
        for (int i = 0; i < take; ++i)
            keep[c[i].n] = 1;
        if (take >= 1 && take < nc && c[take - 1].d > 0.0)
            mg = (c[take - 1].d - c[take].d) / c[take - 1].d;
        free(c);
    }

    int St = 0;
    for (int p = 0; p < S; ++p)
        if (keep[p])
            idx[St++] = p;
    if (detail)
        memcpy(detail, d, sizeof(double) * (size_t)S);
    if (margin)
        *margin = mg;
    free(keep);
    free(d);
    free(lvl);
    return St;
}

/* ---------------------------------------------------------------------- */
/* Point-spread matrix (section "DAMAS"): column s of A is the beamformer
 * response to a unit source at r_s, A[n][s] = |e_n^H e_s|^2 / M^2.       */

void orc_psf(int M, int St, const double *e, double *A)
{
    double inv = 1.0 / ((double)M * (double)M);
    for (int i = 0; i < St; ++i) {
        const double *ei = e + (size_t)2 * M * i;
        for (int j = i; j < St; ++j) {
            const double *ej = e + (size_t)2 * M * j;
            double re = 0.0, im = 0.0;
            for (int m = 0; m < M; ++m) {
                /* conj(ei_m) * ej_m */
                double ar = ei[2 * m], ai = -ei[2 * m + 1];
                double br = ej[2 * m], bi = ej[2 * m + 1];
                re += ar * br - ai * bi;
                im += ar * bi + ai * br;
            }
            double v = (re * re + im * im) * inv;
            A[(size_t)i * St + j] = v;
            A[(size_t)j * St + i] = v;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* DAMAS iteration (section "DAMAS"): successive relaxation over the rows,
 * r_i = sum_j A_ij x_j - b_i with x_j already updated for j < i, then
 * x_i = max(x_i - r_i / A_ii, 0).                                        */

void orc_gs(int St, const double *A, const double *b, int iters, double *x)
{
    for (int it = 0; it < iters; ++it) {
        for (int i = 0; i < St; ++i) {
            const double *a = A + (size_t)i * St;
            double s = 0.0;
            for (int j = 0; j < St; ++j)
                s += a[j] * x[j];
            double r = s - b[i];
            double v = x[i] - r / a[i];
            x[i] = v > 0.0 ? v : 0.0;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* One frequency bin end to end: DAS map on the full grid, compression of
 * the grid from that map, DAMAS on the compressed system (Eq. Axb_CG).   */

int orc_solve_bin(const orc_geom *g, double freq, const double *csm,
                  int mode, double eps, int keep_count, int iters,
                  const double *x_init, double *b_map, int *idx,
                  double *x_map, double *margin)
{
    int S = g->N * g->N;
    int M = g->M;
    double *b = (double *)malloc(sizeof(double) * (size_t)S);
    if (!b)
        return -1;
    orc_das_map(g, freq, csm, b);
    int St = orc_select(g->N, b, mode, eps, keep_count, idx, NULL, margin);

    double *e = (double *)malloc(sizeof(double) * 2 * (size_t)M * (size_t)St);
    double *A = (double *)malloc(sizeof(double) * (size_t)St * (size_t)St);
    double *bt = (double *)malloc(sizeof(double) * (size_t)St);
    double *xt = (double *)malloc(sizeof(double) * (size_t)St);
    if ((St && (!e || !A || !bt || !xt))) {
        free(b); free(e); free(A); free(bt); free(xt);
        return -1;
    }
    orc_steering(g, freq, St, idx, e);
    orc_psf(M, St, e, A);
    for (int i = 0; i < St; ++i) {
        bt[i] = b[idx[i]];
        xt[i] = x_init ? x_init[idx[i]] : 0.0;
    }
    orc_gs(St, A, bt, iters, xt);

    if (b_map)
        memcpy(b_map, b, sizeof(double) * (size_t)S);
    if (x_map) {
        for (int n = 0; n < S; ++n)
            x_map[n] = 0.0;
        for (int i = 0; i < St; ++i)
            x_map[idx[i]] = xt[i];
    }
    free(b); free(e); free(A); free(bt); free(xt);
    return St;
}

/* ---------------------------------------------------------------------- */
/* Steering forms and CSM diagonal removal.                               */

void orc_steering_form(const orc_geom *g, double freq, int form, int n_pts, const int *pts,
                       double *v, double *w)
{
    double k = wavenumber(g, freq);
    for (int p = 0; p < n_pts; ++p) {
        double r[3];
        orc_grid_point(g, pts[p], r);
        /* |r|: distance from the point to the array centre (the origin). */
        double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        for (int m = 0; m < g->M; ++m) {
            double ddx = r[0] - g->mic[3 * m + 0];
            double ddy = r[1] - g->mic[3 * m + 1];
            double ddz = r[2] - g->mic[3 * m + 2];
            double d = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
            double c = cos(k * d), s = -sin(k * d);
            /* v_m = (d / |r|) e_m, g_m = (|r| / d) e_m (paper); both e_m
             * in the unit form */
            double av = form == ORC_STEER_PAPER ? d / rn : 1.0;
            double ag = form == ORC_STEER_PAPER ? rn / d : 1.0;
            size_t o = (size_t)2 * ((size_t)p * g->M + m);
            if (v) {
                v[o] = av * c;
                v[o + 1] = av * s;
            }
            if (w) {
                w[o] = ag * c;
                w[o + 1] = ag * s;
            }
        }
    }
}

void orc_das_map_ex(const orc_geom *g, double freq, const double *csm, int form, int diag,
                    double *b)
{
    int M = g->M;
    int S = g->N * g->N;
    double *v = (double *)malloc(sizeof(double) * 2 * (size_t)M);
    double norm = (double)M * (double)M - (diag ? (double)M : 0.0);
    for (int n = 0; n < S; ++n) {
        orc_steering_form(g, freq, form, 1, &n, v, NULL);
        /* sum_m sum_m' conj(v_m) C_mm' v_m', real part, without the m = m'
         * terms when the diagonal is removed */
        double acc = 0.0;
        for (int m = 0; m < M; ++m) {
            double ar = v[2 * m], ai = -v[2 * m + 1]; /* conj(v_m) */
            for (int mp = 0; mp < M; ++mp) {
                if (diag && mp == m)
                    continue;
                const double *c = csm + 2 * ((size_t)m * M + mp);
                double tr = ar * c[0] - ai * c[1];
                double ti = ar * c[1] + ai * c[0];
                acc += tr * v[2 * mp] - ti * v[2 * mp + 1];
            }
        }
        b[n] = acc / norm;
    }
    free(v);
}

void orc_psf_ex(int M, int St, const double *v, const double *w, int diag, double *A)
{
    /* the reciprocal, as orc_psf scales by 1 / M^2 */
    double inv = 1.0 / ((double)M * (double)M - (diag ? (double)M : 0.0));
    for (int i = 0; i < St; ++i) {
        const double *vi = v + (size_t)2 * M * i;
        for (int j = 0; j < St; ++j) {
            const double *wj = w + (size_t)2 * M * j;
            double re = 0.0, im = 0.0, dd = 0.0;
            for (int m = 0; m < M; ++m) {
                /* conj(v_im) * w_jm */
                double ar = vi[2 * m], ai = -vi[2 * m + 1];
                double br = wj[2 * m], bi = wj[2 * m + 1];
                re += ar * br - ai * bi;
                im += ar * bi + ai * br;
                /* |v_im|^2 |w_jm|^2: the m = m' term of |v_i^H w_j|^2 */
                dd += (ar * ar + ai * ai) * (br * br + bi * bi);
            }
            A[(size_t)i * St + j] = (re * re + im * im - (diag ? dd : 0.0)) * inv;
        }
    }
}

int orc_solve_bin_ex(const orc_geom *g, double freq, const double *csm, int form, int diag,
                     int mode, double eps, int keep_count, int iters, const double *x_init,
                     double *b_map, int *idx, double *x_map, double *margin)
{
    int S = g->N * g->N;
    int M = g->M;
    double *b = (double *)malloc(sizeof(double) * (size_t)S);
    if (!b)
        return -1;
    orc_das_map_ex(g, freq, csm, form, diag, b);
    int St = orc_select(g->N, b, mode, eps, keep_count, idx, NULL, margin);

    double *v = (double *)malloc(sizeof(double) * 2 * (size_t)M * (size_t)St);
    double *w = (double *)malloc(sizeof(double) * 2 * (size_t)M * (size_t)St);
    double *A = (double *)malloc(sizeof(double) * (size_t)St * (size_t)St);
    double *bt = (double *)malloc(sizeof(double) * (size_t)St);
    double *xt = (double *)malloc(sizeof(double) * (size_t)St);
    if (St && (!v || !w || !A || !bt || !xt)) {
        free(b); free(v); free(w); free(A); free(bt); free(xt);
        return -1;
    }
    orc_steering_form(g, freq, form, St, idx, v, w);
    orc_psf_ex(M, St, v, w, diag, A);
    for (int i = 0; i < St; ++i) {
        bt[i] = b[idx[i]];
        xt[i] = x_init ? x_init[idx[i]] : 0.0;
    }
    orc_gs(St, A, bt, iters, xt);

    if (b_map)
        memcpy(b_map, b, sizeof(double) * (size_t)S);
    if (x_map) {
        for (int n = 0; n < S; ++n)
            x_map[n] = 0.0;
        for (int i = 0; i < St; ++i)
            x_map[idx[i]] = xt[i];
    }
    free(b); free(v); free(w); free(A); free(bt); free(xt);
    return St;
}
