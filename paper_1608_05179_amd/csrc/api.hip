// C ABI of the library: argument validation, the device workspace of a
// context, and the order of the launches that make up one solve.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <set>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "ctx_internal.h"

using namespace damas;

namespace {

thread_local std::string g_err;
thread_local damas_ctx *g_ctx_cur = nullptr; // see CtxScope

void record(const char *msg)
{
    g_err = msg;
    if (g_ctx_cur) {
        std::lock_guard<std::mutex> lk(g_ctx_cur->err_mu);
        g_ctx_cur->err = msg;
    }
}

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    record(buf);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(DAMAS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                                                    \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess)                                                  \
            return hip_fail(e_, what);                                         \
    } while (0)

// One zero-initialised fault word per device for the step-level calls,
// which run without a context (a context's solves use its own word).
std::mutex g_fault_mu;
std::unordered_map<int, int *> g_fault;

int fault_word(int **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_fault_mu);
    auto it = g_fault.find(dev);
    if (it != g_fault.end()) {
        *out = it->second;
        return DAMAS_OK;
    }
    int *p = nullptr;
    HIP_TRY(hipMalloc(&p, sizeof(int)), "hipMalloc(fault word)");
    HIP_TRY(hipMemset(p, 0, sizeof(int)), "hipMemset(fault word)");
    g_fault[dev] = p;
    *out = p;
    return DAMAS_OK;
}

bool finite(double v) { return isfinite(v) != 0; }

int check_geometry(const damas_geometry *g)
{
    if (!g)
        return fail(DAMAS_EINVAL, "geometry is NULL");
    if (g->M < 1 || g->M > 128)
        return fail(DAMAS_EINVAL, "M = %d outside [1, 128]", g->M);
    if (!g->mic)
        return fail(DAMAS_EINVAL, "mic positions are NULL");
    if (g->N < 1 || g->N > 46340)
        return fail(DAMAS_EINVAL, "N = %d outside [1, 46340]", g->N);
    if (!finite(g->x0) || !finite(g->x1) || !finite(g->y0) || !finite(g->y1) ||
        !finite(g->z0))
        return fail(DAMAS_EINVAL, "scan-plane extent is not finite");
    if (!(g->c > 0.0) || !finite(g->c))
        return fail(DAMAS_EINVAL, "speed of sound must be positive and finite");
    return DAMAS_OK;
}

int check_precision(int32_t p)
{
    if (p != DAMAS_PREC_FP64 && p != DAMAS_PREC_FP32 && p != DAMAS_PREC_BF16)
        return fail(DAMAS_EINVAL, "unknown precision %d", p);
    return DAMAS_OK;
}

// Storage precisions of damas_psf (double steering rows in).
int check_psf_precision(int32_t p)
{
    if (p != DAMAS_PREC_FP64 && p != DAMAS_PREC_FP32)
        return fail(DAMAS_EINVAL, "damas_psf stores FP64 or FP32 (precision %d); "
                                  "bf16 systems come from damas_psf_bf16", p);
    return DAMAS_OK;
}

// Steering form and diagonal removal of a solve (the paper's pair needs the
// double steering rows of the f64 PSF: FP64 or FP32 storage).
int check_form(int32_t steering, int32_t diag, int32_t precision)
{
    if (steering != DAMAS_STEER_UNIT && steering != DAMAS_STEER_PAPER)
        return fail(DAMAS_EINVAL, "steering = %d is not a DAMAS_STEER_* value", steering);
    if (diag != 0 && diag != 1)
        return fail(DAMAS_EINVAL, "diag_removal must be 0 or 1");
    if (steering == DAMAS_STEER_PAPER && precision == DAMAS_PREC_BF16)
        return fail(DAMAS_EINVAL, "the paper's steering pair is built at FP64 or FP32");
    return DAMAS_OK;
}

int check_mode(int32_t mode, double eps)
{
    if (mode != DAMAS_SEL_KEEP_ALL && mode != DAMAS_SEL_EPS_REL &&
        mode != DAMAS_SEL_KEEP_COUNT)
        return fail(DAMAS_EINVAL, "unknown selection mode %d", mode);
    if (mode == DAMAS_SEL_EPS_REL && (!(eps >= 0.0) || !finite(eps)))
        return fail(DAMAS_EINVAL, "eps must be finite and >= 0");
    return DAMAS_OK;
}

} // namespace

// KEEP_FRAC is KEEP_COUNT with one count for every bin, ceil(keep_frac *
// N^2): *q becomes `tmp`, a copy of *p in that form, or stays p for the
// other modes.
int damas::resolve_frac(const damas_params *p, int32_t N, damas_params &tmp,
                        const damas_params **q)
{
    *q = p;
    if (!p || p->select_mode != DAMAS_SEL_KEEP_FRAC)
        return DAMAS_OK;
    const double f = p->keep_frac;
    if (!(f > 0.0 && f <= 1.0))
        return fail(DAMAS_EINVAL, "keep_frac = %g outside (0, 1]", f);
    tmp = *p;
    tmp.select_mode = DAMAS_SEL_KEEP_COUNT;
    tmp.keep_count = nullptr;
    tmp.keep_count_all = (int32_t)std::ceil(f * (double)N * (double)N);
    *q = &tmp;
    return DAMAS_OK;
}

namespace {

int check_kept(int32_t max_kept, int32_t S, int32_t precision)
{
    if (max_kept < 0 || max_kept > S)
        return fail(DAMAS_EINVAL, "max_kept = %d outside [0, N*N = %d]", max_kept, S);
    // The bf16 path ends with FP32 sweeps: both must fit.
    if (precision == DAMAS_PREC_BF16 && max_kept > gs_max_kept(DAMAS_PREC_FP32))
        return fail(DAMAS_EINVAL,
                    "max_kept = %d exceeds the %d unknowns a sweep workgroup "
                    "holds on chip for the FP32 refinement sweeps",
                    max_kept, gs_max_kept(DAMAS_PREC_FP32));
    if (max_kept > gs_max_kept(precision))
        return fail(DAMAS_EINVAL,
                    "max_kept = %d exceeds the %d unknowns a sweep workgroup "
                    "holds on chip at this precision",
                    max_kept, gs_max_kept(precision));
    return DAMAS_OK;
}

size_t elem_size(int32_t precision)
{
    return precision == DAMAS_PREC_FP64   ? sizeof(double)
           : precision == DAMAS_PREC_FP32 ? sizeof(float)
                                          : sizeof(uint16_t);
}

// Element size of the x maps.
size_t x_size(int32_t precision)
{
    return precision == DAMAS_PREC_FP64 ? sizeof(double) : sizeof(float);
}

int coarse_count(int32_t N)
{
    int J = 0;
    while ((2 << J) <= N)
        ++J;
    int side = (1 << J) < N ? 2 : 1;
    return side * side;
}

} // namespace

hipError_t damas::allow_big_lds(const void *kernel)
{
    // Raise the kernel's dynamic-LDS limit to what a workgroup may hold on
    // this device.  A runtime that needs no opt-in may refuse the call;
    // the launch itself then reports any real shortfall, so the status is
    // cleared here rather than left for the next error check.
    int dev = 0, max_lds = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
            hipSuccess &&
        max_lds > 0)
        (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    (void)hipGetLastError();
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// helpers

extern "C" const char *damas_strerror(int code)
{
    switch (code) {
    case DAMAS_OK: return "success";
    case DAMAS_EINVAL: return "invalid argument";
    case DAMAS_ENOMEM: return "out of memory";
    case DAMAS_EDEVICE: return "device error";
    case DAMAS_EADMIT: return "request exceeds the memory budget";
    case DAMAS_EBUSY: return "busy (queue full or resource in use)";
    case DAMAS_ETIMEDOUT: return "timed out";
    case DAMAS_ECAPACITY: return "device-side capacity exceeded";
    default: return "unknown status";
    }
}

extern "C" const char *damas_last_error(void) { return g_err.c_str(); }

extern "C" int64_t damas_ld(int32_t s_tilde) { return s_tilde < 0 ? 0 : ld_of(s_tilde); }

extern "C" int32_t damas_coarse_count(int32_t N) { return N < 1 ? 0 : coarse_count(N); }

extern "C" int32_t damas_mp(int32_t M) { return M < 1 ? 0 : mp_of(M); }

extern "C" int32_t damas_wide_capacity(void) { return gs_wide_capacity(); }

extern "C" int32_t damas_gs_capacity(int32_t precision)
{
    if (precision != DAMAS_PREC_FP64 && precision != DAMAS_PREC_FP32 &&
        precision != DAMAS_PREC_BF16)
        return 0;
    const int c = gs_max_kept(precision);
    return precision == DAMAS_PREC_BF16 ? std::min(c, gs_max_kept(DAMAS_PREC_FP32)) : c;
}

// ---------------------------------------------------------------------------
// step-level calls

extern "C" int damas_csm(int32_t M, int32_t n_snap, int32_t n_bins, const double *snap,
                         double *csm, void *stream)
{
    if (M < 1 || M > 8192)
        return fail(DAMAS_EINVAL, "M = %d outside [1, 8192]", M);
    if (n_snap < 1)
        return fail(DAMAS_EINVAL, "n_snap = %d < 1", n_snap);
    if (n_bins < 0)
        return fail(DAMAS_EINVAL, "n_bins < 0");
    if (n_bins > 0 && (!snap || !csm))
        return fail(DAMAS_EINVAL, "snap and csm must be non-NULL");
    if ((int64_t)n_bins * csm_upper_blocks(M) > (int64_t)1 << 33)
        return fail(DAMAS_EINVAL, "n_bins = %d too large for M = %d", n_bins, M);
    HIP_TRY(launch_csm(M, n_snap, n_bins, snap, csm, (hipStream_t)stream), "csm launch");
    return DAMAS_OK;
}

extern "C" int damas_das_map(const damas_geometry *g, int32_t n_bins,
                             const double *freq, const double *csm, double *b,
                             void *stream)
{
    int rc = check_geometry(g);
    if (rc)
        return rc;
    if (n_bins < 0)
        return fail(DAMAS_EINVAL, "n_bins < 0");
    if (n_bins > 0 && (!freq || !csm || !b))
        return fail(DAMAS_EINVAL, "freq, csm and b must be non-NULL");
    HIP_TRY(launch_das(make_geom(*g), n_bins, freq, csm, b, (hipStream_t)stream),
            "das launch");
    return DAMAS_OK;
}

extern "C" int damas_select_pred(int32_t N, int32_t n_bins, const double *b,
                                 int32_t mode, double eps, int32_t predictor,
                                 const int32_t *keep_count, int32_t *idx,
                                 int32_t *s_tilde, void *stream)
{
    if (N < 1 || N > 46340)
        return fail(DAMAS_EINVAL, "N = %d outside [1, 46340]", N);
    if (predictor != DAMAS_PRED_HAAR && predictor != DAMAS_PRED_LINEAR)
        return fail(DAMAS_EINVAL, "predictor = %d is not a DAMAS_PRED_* value", predictor);
    if (n_bins < 0)
        return fail(DAMAS_EINVAL, "n_bins < 0");
    int rc = check_mode(mode, eps);
    if (rc)
        return rc;
    if (n_bins > 0 && (!b || !idx || !s_tilde))
        return fail(DAMAS_EINVAL, "b, idx and s_tilde must be non-NULL");
    if (n_bins > 0 && mode == DAMAS_SEL_KEEP_COUNT && !keep_count)
        return fail(DAMAS_EINVAL, "KEEP_COUNT needs keep_count");
    HIP_TRY(launch_select(N, n_bins, b, mode, eps, predictor, keep_count, idx, s_tilde,
                          (hipStream_t)stream),
            "select launch");
    return DAMAS_OK;
}

extern "C" int damas_select(int32_t N, int32_t n_bins, const double *b, int32_t mode,
                            double eps, const int32_t *keep_count, int32_t *idx,
                            int32_t *s_tilde, void *stream)
{
    return damas_select_pred(N, n_bins, b, mode, eps, DAMAS_PRED_HAAR, keep_count, idx,
                             s_tilde, stream);
}

extern "C" int damas_layout(int32_t n_bins, int32_t *s_tilde, int32_t max_kept,
                            int64_t capacity, int64_t *off, void *stream)
{
    if (n_bins < 0 || max_kept < 0 || capacity < 0)
        return fail(DAMAS_EINVAL, "n_bins, max_kept and capacity must be >= 0");
    if (!off || (n_bins > 0 && !s_tilde))
        return fail(DAMAS_EINVAL, "s_tilde and off must be non-NULL");
    int *fault;
    int rc = fault_word(&fault);
    if (rc)
        return rc;
    HIP_TRY(launch_layout(n_bins, s_tilde, max_kept, capacity, off, fault,
                          (hipStream_t)stream),
            "layout launch");
    return DAMAS_OK;
}

extern "C" int damas_steer(const damas_geometry *g, int32_t n_bins,
                           const double *freq, const int32_t *idx,
                           const int32_t *s_tilde, int32_t max_kept, double *E,
                           int64_t e_stride, void *stream)
{
    int rc = check_geometry(g);
    if (rc)
        return rc;
    const int32_t S = g->N * g->N;
    if (n_bins < 0)
        return fail(DAMAS_EINVAL, "n_bins < 0");
    if (max_kept < 0 || max_kept > S)
        return fail(DAMAS_EINVAL, "max_kept = %d outside [0, N*N]", max_kept);
    if (n_bins > 0 && (!freq || !idx || !s_tilde || !E))
        return fail(DAMAS_EINVAL, "freq, idx, s_tilde and E must be non-NULL");
    if (n_bins > 1 && e_stride < ld_of(max_kept) * 2 * g->M)
        return fail(DAMAS_EINVAL, "e_stride < damas_ld(max_kept) * 2M");
    int *fault;
    if ((rc = fault_word(&fault)))
        return rc;
    HIP_TRY(launch_steer(make_geom(*g), n_bins, freq, idx, s_tilde, max_kept, E,
                         e_stride, fault, (hipStream_t)stream),
            "steer launch");
    return DAMAS_OK;
}

extern "C" int damas_psf(int32_t M, int32_t n_bins, const int32_t *s_tilde,
                         int32_t max_kept, int32_t precision, const double *E,
                         int64_t e_stride, const int64_t *off, void *A,
                         void *stream)
{
    int rc = check_psf_precision(precision);
    if (rc)
        return rc;
    if (M < 1 || M > 128)
        return fail(DAMAS_EINVAL, "M = %d outside [1, 128]", M);
    if (n_bins < 0 || max_kept < 0)
        return fail(DAMAS_EINVAL, "n_bins and max_kept must be >= 0");
    if (n_bins > 0 && (!s_tilde || !E || !off || !A))
        return fail(DAMAS_EINVAL, "s_tilde, E, off and A must be non-NULL");
    if (n_bins > 1 && e_stride < ld_of(max_kept) * 2 * M)
        return fail(DAMAS_EINVAL, "e_stride < damas_ld(max_kept) * 2M");
    int *fault;
    if ((rc = fault_word(&fault)))
        return rc;
    HIP_TRY(launch_psf(M, n_bins, s_tilde, max_kept, precision, E, e_stride, off,
                       A, fault, (hipStream_t)stream),
            "psf launch");
    return DAMAS_OK;
}

extern "C" int damas_das_map_ex(const damas_geometry *g, int32_t n_bins, const double *freq,
                                const double *csm, int32_t steering, int32_t diag_removal,
                                double *b, void *stream)
{
    int rc = check_geometry(g);
    if (rc || (rc = check_form(steering, diag_removal, DAMAS_PREC_FP64)))
        return rc;
    if (n_bins < 0)
        return fail(DAMAS_EINVAL, "n_bins < 0");
    if (n_bins > 0 && (!freq || !csm || !b))
        return fail(DAMAS_EINVAL, "freq, csm and b must be non-NULL");
    HIP_TRY(launch_das(make_geom(*g), n_bins, freq, csm, b, (hipStream_t)stream, steering,
                       diag_removal),
            "das launch");
    return DAMAS_OK;
}

extern "C" int damas_steer_ex(const damas_geometry *g, int32_t n_bins, const double *freq,
                              const int32_t *idx, const int32_t *s_tilde, int32_t max_kept,
                              int32_t steering, double *E, int64_t e_stride, void *stream)
{
    int rc = check_geometry(g);
    if (rc || (rc = check_form(steering, 0, DAMAS_PREC_FP64)))
        return rc;
    const int32_t S = g->N * g->N;
    if (n_bins < 0)
        return fail(DAMAS_EINVAL, "n_bins < 0");
    if (max_kept < 0 || max_kept > S)
        return fail(DAMAS_EINVAL, "max_kept = %d outside [0, N*N]", max_kept);
    if (n_bins > 0 && (!freq || !idx || !s_tilde || !E))
        return fail(DAMAS_EINVAL, "freq, idx, s_tilde and E must be non-NULL");
    const int64_t rows = ld_of(max_kept) * (steering == DAMAS_STEER_PAPER ? 2 : 1);
    if (n_bins > 1 && e_stride < rows * 2 * g->M)
        return fail(DAMAS_EINVAL, "e_stride < rows * 2M (two row sets for the paper's pair)");
    int *fault;
    if ((rc = fault_word(&fault)))
        return rc;
    HIP_TRY(launch_steer(make_geom(*g), n_bins, freq, idx, s_tilde, max_kept, E, e_stride,
                         fault, (hipStream_t)stream, steering),
            "steer launch");
    return DAMAS_OK;
}

extern "C" int damas_psf_ex(int32_t M, int32_t n_bins, const int32_t *s_tilde,
                            int32_t max_kept, int32_t precision, int32_t steering,
                            int32_t diag_removal, const double *E, int64_t e_stride,
                            const int64_t *off, void *A, void *stream)
{
    int rc = check_psf_precision(precision);
    if (rc || (rc = check_form(steering, diag_removal, precision)))
        return rc;
    if (M < 1 || M > 128)
        return fail(DAMAS_EINVAL, "M = %d outside [1, 128]", M);
    if (n_bins < 0 || max_kept < 0)
        return fail(DAMAS_EINVAL, "n_bins and max_kept must be >= 0");
    if (n_bins > 0 && (!s_tilde || !E || !off || !A))
        return fail(DAMAS_EINVAL, "s_tilde, E, off and A must be non-NULL");
    const int64_t rows = ld_of(max_kept) * (steering == DAMAS_STEER_PAPER ? 2 : 1);
    if (n_bins > 1 && e_stride < rows * 2 * M)
        return fail(DAMAS_EINVAL, "e_stride < rows * 2M (two row sets for the paper's pair)");
    int *fault;
    if ((rc = fault_word(&fault)))
        return rc;
    HIP_TRY(launch_psf(M, n_bins, s_tilde, max_kept, precision, E, e_stride, off, A, fault,
                       (hipStream_t)stream, PsfClassArgs(), steering, diag_removal),
            "psf launch");
    return DAMAS_OK;
}

extern "C" int damas_steer_bf16(const damas_geometry *g, int32_t n_bins,
                                const double *freq, const int32_t *idx,
                                const int32_t *s_tilde, int32_t max_kept, uint16_t *E16,
                                int64_t e16_stride, void *stream)
{
    int rc = check_geometry(g);
    if (rc)
        return rc;
    const int32_t S = g->N * g->N;
    if (n_bins < 0)
        return fail(DAMAS_EINVAL, "n_bins < 0");
    if (max_kept < 0 || max_kept > S)
        return fail(DAMAS_EINVAL, "max_kept = %d outside [0, N*N]", max_kept);
    if (n_bins > 0 && (!freq || !idx || !s_tilde || !E16))
        return fail(DAMAS_EINVAL, "freq, idx, s_tilde and E16 must be non-NULL");
    if (n_bins > 1 && e16_stride < ld_of(max_kept) * 2 * mp_of(g->M))
        return fail(DAMAS_EINVAL, "e16_stride < damas_ld(max_kept) * 2 * damas_mp(M)");
    int *fault;
    if ((rc = fault_word(&fault)))
        return rc;
    HIP_TRY(launch_steer16(make_geom(*g), n_bins, freq, idx, s_tilde, max_kept, E16,
                           e16_stride, fault, (hipStream_t)stream),
            "steer16 launch");
    return DAMAS_OK;
}

extern "C" int damas_psf_bf16(int32_t M, int32_t n_bins, const int32_t *s_tilde,
                              int32_t max_kept, const uint16_t *E16, int64_t e16_stride,
                              const int64_t *off, uint16_t *A16, void *stream)
{
    if (M < 1 || M > 128)
        return fail(DAMAS_EINVAL, "M = %d outside [1, 128]", M);
    if (n_bins < 0 || max_kept < 0)
        return fail(DAMAS_EINVAL, "n_bins and max_kept must be >= 0");
    if (n_bins > 0 && (!s_tilde || !E16 || !off || !A16))
        return fail(DAMAS_EINVAL, "s_tilde, E16, off and A16 must be non-NULL");
    if (n_bins > 1 && e16_stride < ld_of(max_kept) * 2 * mp_of(M))
        return fail(DAMAS_EINVAL, "e16_stride < damas_ld(max_kept) * 2 * damas_mp(M)");
    int *fault;
    int rc = fault_word(&fault);
    if (rc)
        return rc;
    HIP_TRY(launch_psf16(M, n_bins, s_tilde, max_kept, E16, e16_stride, off, A16, fault,
                         (hipStream_t)stream),
            "psf16 launch");
    return DAMAS_OK;
}

extern "C" int damas_gs(int32_t N, int32_t n_bins, const int32_t *s_tilde,
                        int32_t max_kept, const int32_t *idx,
                        const int64_t *off, int32_t precision, int32_t unit_diagonal,
                        const void *A, const double *b, int32_t iterations,
                        const void *x_init, void *x_map, void *stream)
{
    int rc = check_precision(precision);
    if (rc)
        return rc;
    if (N < 1 || N > 46340)
        return fail(DAMAS_EINVAL, "N = %d outside [1, 46340]", N);
    if (n_bins < 0 || iterations < 0)
        return fail(DAMAS_EINVAL, "n_bins and iterations must be >= 0");
    if ((rc = check_kept(max_kept, N * N, precision)))
        return rc;
    if (n_bins > 0 && (!s_tilde || !idx || !off || !A || !b || !x_map))
        return fail(DAMAS_EINVAL, "s_tilde, idx, off, A, b and x_map must be non-NULL");
    int *fault;
    if ((rc = fault_word(&fault)))
        return rc;
    HIP_TRY(launch_gs(N, n_bins, s_tilde, max_kept, idx, off, precision, unit_diagonal != 0,
                      A, b, iterations, x_init, x_map, fault, (hipStream_t)stream),
            "gs launch");
    return DAMAS_OK;
}

// ---------------------------------------------------------------------------
// context

namespace {

int ensure(damas_ctx *ctx, Buffer &buf, size_t bytes, hipStream_t s, const char *what)
{
    if (buf.bytes >= bytes)
        return DAMAS_OK;
    if (ctx->graphs > 0 || ctx->in_capture)
        return fail(DAMAS_EBUSY,
                    "%s would grow while a graph captured on this context exists", what);
    if (ctx->hbm_budget) {
        const size_t after = ctx_bytes(ctx) - buf.bytes + std::max(bytes, (size_t)256);
        if (after > ctx->hbm_budget)
            return fail(DAMAS_EADMIT,
                        "%s would take the context's workspace to %zu bytes, beyond its "
                        "budget of %llu",
                        what, after, (unsigned long long)ctx->hbm_budget);
    }
    if (buf.p) {
        // Work already enqueued may still read the old buffer.
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
        HIP_TRY(hipFree(buf.p), "hipFree");
        buf.p = nullptr;
        buf.bytes = 0;
    }
    size_t want = std::max(bytes, (size_t)256);
    if (hipMalloc(&buf.p, want) != hipSuccess) {
        (void)hipGetLastError();
        buf.p = nullptr;
        return fail(DAMAS_ENOMEM, "cannot allocate %zu bytes for %s", want, what);
    }
    buf.bytes = want;
    (void)ctx;
    return DAMAS_OK;
}

int pop_events(damas_ctx *ctx, std::pair<hipEvent_t, hipEvent_t> *ev)
{
    if (!ctx->event_pool.empty()) {
        *ev = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return DAMAS_OK;
    }
    HIP_TRY(hipEventCreate(&ev->first), "hipEventCreate");
    HIP_TRY(hipEventCreate(&ev->second), "hipEventCreate");
    return DAMAS_OK;
}

} // namespace

namespace {

// Schedule knobs the cooperative planner accepts (it divides by min_rows
// and weighs work by split, overhead and wide_cost).
bool knobs_valid(int coop, int min_rows, double split, double overhead, int floor_rows,
                 double wide_cost)
{
    return (coop == 0 || coop == 1) && min_rows >= 64 && split > 0.0 && overhead > 0.0 &&
           wide_cost > 0.0 && floor_rows >= 0 && std::isfinite(split) &&
           std::isfinite(overhead) && std::isfinite(wide_cost);
}

// Autotune cache lines: key, then the knobs and the timed ms per sweep;
// a line that does not parse or holds knobs out of range is skipped.
void load_tune_cache(damas_ctx *c)
{
    FILE *fh = fopen(c->tune_cache.c_str(), "r");
    if (!fh)
        return; // a missing file is an empty cache
    char line[1024];
    while (fgets(line, sizeof line, fh)) {
        char key[512];
        int coop = 0, mr = 0, fl = 0;
        double sp = 0, ov = 0, wc = 0, ms = 0;
        if (sscanf(line, "%511s %d %d %lf %lf %d %lf %lf", key, &coop, &mr, &sp, &ov, &fl, &wc,
                   &ms) == 8 &&
            knobs_valid(coop, mr, sp, ov, fl, wc)) {
            TuneKnobs k;
            k.coop = coop != 0;
            k.min_rows = mr;
            k.split = sp;
            k.overhead = ov;
            k.floor_rows = fl;
            k.wide_cost = wc;
            c->tune_entries[key] = {k, ms};
        }
    }
    fclose(fh);
}

} // namespace

extern "C" int damas_ctx_create(int32_t device, damas_ctx **out)
{
    damas_ctx_opts o{};
    o.device = device;
    return damas_ctx_create_ex(&o, out);
}

extern "C" int damas_ctx_create_ex(const damas_ctx_opts *opts, damas_ctx **out)
{
    if (!out || !opts)
        return fail(DAMAS_EINVAL, "opts and out must be non-NULL");
    if (opts->deterministic != 0 && opts->deterministic != 1)
        return fail(DAMAS_EINVAL, "deterministic must be 0 or 1");
    const int32_t device = opts->device;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (device < 0 || device >= n)
        return fail(DAMAS_EINVAL, "device %d outside [0, %d)", device, n);
    HIP_TRY(hipSetDevice(device), "hipSetDevice");
    damas_ctx *c = new (std::nothrow) damas_ctx();
    if (!c)
        return fail(DAMAS_ENOMEM, "context allocation");
    c->device = device;
    if (hipEventCreateWithFlags(&c->kc_done, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->coop_done, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&c->fault, sizeof(int)) != hipSuccess ||
        hipMemset(c->fault, 0, sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        if (c->kc_done)
            (void)hipEventDestroy(c->kc_done);
        if (c->coop_done)
            (void)hipEventDestroy(c->coop_done);
        if (c->fault)
            (void)hipFree(c->fault);
        delete c;
        return fail(DAMAS_EDEVICE, "context set-up (events, fault word)");
    }
    c->hbm_budget = opts->hbm_budget;
    c->deterministic = opts->deterministic == 1;
    if (c->deterministic)
        c->coop_budget = 0;
    if (opts->tune_cache && opts->tune_cache[0]) {
        c->tune_cache = opts->tune_cache;
        load_tune_cache(c);
    }
    *out = c;
    return DAMAS_OK;
}

extern "C" const char *damas_ctx_last_error(const damas_ctx *ctx)
{
    thread_local std::string copy;
    if (!ctx)
        return "";
    std::lock_guard<std::mutex> lk(ctx->err_mu);
    copy = ctx->err;
    return copy.c_str();
}

extern "C" void damas_ctx_destroy(damas_ctx *ctx)
{
    if (!ctx)
        return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (Buffer *b : {&ctx->b, &ctx->idx, &ctx->st, &ctx->kc, &ctx->off, &ctx->E, &ctx->A,
                      &ctx->E16, &ctx->A32, &ctx->Alo, &ctx->tsum, &ctx->cls, &ctx->coop_ws,
                      &ctx->coop_tab, &ctx->mapt})
        if (b->p)
            (void)hipFree(b->p);
    if (ctx->kc_pinned)
        (void)hipHostFree(ctx->kc_pinned);
    if (ctx->mapt_pinned)
        (void)hipHostFree(ctx->mapt_pinned);
    if (ctx->coop_pinned)
        (void)hipHostFree(ctx->coop_pinned);
    if (ctx->cls_pinned)
        (void)hipHostFree(ctx->cls_pinned);
    if (ctx->kc_done)
        (void)hipEventDestroy(ctx->kc_done);
    if (ctx->coop_done)
        (void)hipEventDestroy(ctx->coop_done);
    if (ctx->fault)
        (void)hipFree(ctx->fault);
    for (auto *v : {&ctx->phase_events[0], &ctx->phase_events[1], &ctx->event_pool})
        for (auto &e : *v) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    delete ctx;
}

extern "C" int damas_ctx_set_coop(damas_ctx *ctx, int32_t max_workgroups)
{
    if (!ctx)
        return fail(DAMAS_EINVAL, "ctx is NULL");
    CtxScope scope(ctx);
    if (max_workgroups < -1)
        return fail(DAMAS_EINVAL, "max_workgroups must be >= -1");
    if (ctx->deterministic && max_workgroups != 0)
        return fail(DAMAS_EINVAL, "a deterministic context runs one workgroup per bin");
    ctx->coop_budget = max_workgroups;
    return DAMAS_OK;
}

extern "C" int damas_ctx_last_workgroups(const damas_ctx *ctx, int32_t *workgroups)
{
    CtxScope scope(const_cast<damas_ctx *>(ctx));
    if (!ctx || !workgroups)
        return fail(DAMAS_EINVAL, "NULL argument");
    *workgroups = ctx->last_workgroups;
    return DAMAS_OK;
}

extern "C" int damas_ctx_classes(damas_ctx *ctx, int32_t n_bins, uint8_t *out)
{
    CtxScope scope(ctx);
    if (!ctx || !out || n_bins < 0)
        return fail(DAMAS_EINVAL, "ctx and out must be non-NULL, n_bins >= 0");
    if (n_bins == 0)
        return DAMAS_OK;
    if (!ctx->cls.p || ctx->cls.bytes < (size_t)n_bins)
        return fail(DAMAS_EINVAL, "no classes of %d bins on this context", n_bins);
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    HIP_TRY(hipMemcpy(out, ctx->cls.p, (size_t)n_bins, hipMemcpyDeviceToHost), "read classes");
    return DAMAS_OK;
}

extern "C" int damas_ctx_set_timing(damas_ctx *ctx, int32_t enabled)
{
    CtxScope scope(ctx);
    if (!ctx)
        return fail(DAMAS_EINVAL, "ctx is NULL");
    ctx->timing = enabled != 0;
    return DAMAS_OK;
}

extern "C" int damas_ctx_phase_time(damas_ctx *ctx, int32_t phase, double *ms,
                                    int64_t *launches)
{
    CtxScope scope(ctx);
    if (!ctx || !ms || !launches)
        return fail(DAMAS_EINVAL, "NULL argument");
    if (phase < 0 || phase >= DAMAS_PHASES)
        return fail(DAMAS_EINVAL, "unknown phase %d", phase);
    double total = 0.0;
    int64_t n = 0;
    auto &evs = ctx->phase_events[phase];
    for (auto &e : evs) {
        HIP_TRY(hipEventSynchronize(e.second), "hipEventSynchronize");
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, e.first, e.second), "hipEventElapsedTime");
        total += t;
        ++n;
        ctx->event_pool.push_back(e);
    }
    evs.clear();
    *ms = total;
    *launches = n;
    return DAMAS_OK;
}

extern "C" int damas_ctx_gs_time(damas_ctx *ctx, double *ms, int64_t *launches)
{
    CtxScope scope(ctx);
    return damas_ctx_phase_time(ctx, DAMAS_PHASE_SWEEPS, ms, launches);
}

namespace {
int static_fault(int **out);
}

extern "C" int damas_check(damas_ctx *ctx, void *stream)
{
    CtxScope scope(ctx);
    if (ctx)
        HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize");
    // A context's own word, or the step-level calls' word of the device
    // and, once damas_solve_static has run on it, the static solve's word.
    int *fault = ctx ? ctx->fault : nullptr;
    int *sfault = nullptr;
    if (!fault) {
        int rc = fault_word(&fault);
        if (!rc)
            rc = static_fault(&sfault);
        if (rc)
            return rc;
    }
    int v = 0;
    HIP_TRY(hipMemcpy(&v, fault, sizeof v, hipMemcpyDeviceToHost), "read fault word");
    if (sfault) {
        int w = 0;
        HIP_TRY(hipMemcpy(&w, sfault, sizeof w, hipMemcpyDeviceToHost), "read fault word");
        if (w)
            HIP_TRY(hipMemset(sfault, 0, sizeof(int)), "clear fault word");
        v |= w;
    }
    if (v) {
        HIP_TRY(hipMemset(fault, 0, sizeof(int)), "clear fault word");
        // Bits: 4 a bin kept more points than max_kept; 8 a cooperative
        // exchange gave up waiting; 16 a sweep launch shape did not cover
        // a bin's strip.
        return fail(DAMAS_ECAPACITY,
                    "%s (fault bits 0x%x)",
                    (v & 4) ? "a bin kept more points than max_kept"
                    : (v & 8) ? "a cooperative sweep exchange timed out"
                              : "a sweep launch shape did not cover a bin",
                    v);
    }
    HIP_TRY(hipGetLastError(), "pending HIP error");
    return DAMAS_OK;
}

namespace {

// Validated shape and device buffers of one solve.
struct SolvePlan {
    Geom kg;
    int32_t N, M, S, n_bins;
    const damas_params *p;
    bool batched, bf16, need64, need16;
    int32_t max_kept;
    std::vector<int32_t> st_host; // kept points per bin, where the host knows them
    int32_t bulk, refine;         // sweeps on the storage precision / FP32 copy
    bool classes;                 // per-bin precision classes (DAMAS_POLICY_AUTO)
    int steering, diag;           // steering form, CSM diagonal removal
    double rho_wide, rho_f32;     // their thresholds
    int64_t e_stride, e16_stride;
    int64_t a_elems;
    int nb_ws;                    // bins the workspace holds at once
    size_t es, xs;                // bytes per A element / x element
    double *bm;
    int32_t *ix, *st;
    int64_t *off;
    const int32_t *kc;
    int *fault;
};

// Host-side validation and sizes of a solve (no device work).  The
// geometry's mic pointer is not read here.
int make_plan(int32_t M, int32_t N, int32_t n_bins, const damas_params *p, SolvePlan &P)
{
    int rc;
    if (!p)
        return fail(DAMAS_EINVAL, "params are NULL");
    if ((rc = check_mode(p->select_mode, p->eps)) || (rc = check_precision(p->precision)))
        return rc;
    if (p->predictor != DAMAS_PRED_HAAR && p->predictor != DAMAS_PRED_LINEAR)
        return fail(DAMAS_EINVAL, "predictor = %d is not a DAMAS_PRED_* value", p->predictor);
    if (n_bins < 0 || p->iterations < 0)
        return fail(DAMAS_EINVAL, "n_bins and iterations must be >= 0");
    if (p->policy != DAMAS_POLICY_AUTO && p->policy != DAMAS_POLICY_FIXED)
        return fail(DAMAS_EINVAL, "policy = %d is not a DAMAS_POLICY_* value", p->policy);
    if (!(p->rho_wide >= 0.0) || !(p->rho_f32 >= 0.0))
        return fail(DAMAS_EINVAL, "rho_wide and rho_f32 must be >= 0 (0: defaults)");
    if ((rc = check_form(p->steering, p->diag_removal, p->precision)))
        return rc;
    P.bf16 = p->precision == DAMAS_PREC_BF16;
    if (P.bf16 && (p->refine_sweeps < 0 || p->refine_sweeps > p->iterations))
        return fail(DAMAS_EINVAL, "refine_sweeps = %d outside [0, iterations = %d]",
                    p->refine_sweeps, p->iterations);
    P.N = N;
    P.M = M;
    P.S = N * N;
    P.n_bins = n_bins;
    P.p = p;
    const int n0 = coarse_count(N);
    P.st_host.clear();
    P.max_kept = 0;
    if (p->select_mode == DAMAS_SEL_KEEP_ALL) {
        P.max_kept = P.S;
        P.st_host.assign(n_bins, P.S);
    } else if (p->select_mode == DAMAS_SEL_KEEP_COUNT) {
        P.st_host.resize(n_bins);
        for (int f = 0; f < n_bins; ++f) {
            int32_t K = p->keep_count ? p->keep_count[f] : p->keep_count_all;
            if (K < 0)
                return fail(DAMAS_EINVAL, "keep_count[%d] = %d < 0", f, K);
            P.st_host[f] = std::min(std::max(K, (int32_t)n0), P.S);
            P.max_kept = std::max(P.max_kept, P.st_host[f]);
        }
    } else {
        P.max_kept = p->max_kept > 0 ? std::min(p->max_kept, P.S) : P.S;
    }
    if ((rc = check_kept(P.max_kept, P.S, p->precision)))
        return rc;
    P.batched = p->batched != 0;
    P.es = elem_size(p->precision);
    P.xs = x_size(p->precision);
    const int64_t ldm = ld_of(P.max_kept);
    P.refine = P.bf16 ? p->refine_sweeps : 0;
    P.bulk = p->iterations - P.refine;
    P.steering = p->steering;
    P.diag = p->diag_removal;
    // the paper's pair keeps two row sets (beamformer, propagation) per bin
    P.e_stride = ldm * 2 * M * (P.steering == DAMAS_STEER_PAPER ? 2 : 1);
    P.e16_stride = ldm * 2 * mp_of(M);
    if (!P.batched) {
        P.a_elems = ldm * ldm;
    } else if (!P.st_host.empty()) {
        P.a_elems = 0;
        for (int32_t v : P.st_host)
            P.a_elems += ld_of(v) * ld_of(v);
    } else {
        P.a_elems = (int64_t)n_bins * ldm * ldm;
    }
    P.nb_ws = P.batched ? n_bins : 1;
    P.classes = p->policy == DAMAS_POLICY_AUTO && p->precision != DAMAS_PREC_FP64;
    P.rho_wide = p->rho_wide > 0.0 ? p->rho_wide : DAMAS_RHO_WIDE_DEFAULT;
    P.rho_f32 = p->rho_f32 > 0.0 ? p->rho_f32 : DAMAS_RHO_F32_DEFAULT;
    // With classes a bf16 solve always builds the FP32 system: bins that
    // skip the bf16 bulk run every sweep on it.
    P.need64 = !P.bf16 || P.refine > 0 || P.classes;
    P.need16 = P.bf16 && P.bulk > 0;
    return DAMAS_OK;
}

// Context workspace bytes of a plan: b, idx and s_tilde (when the caller
// does not supply them), keep counts, offsets, steering rows and arenas.
size_t plan_workspace_bytes(const SolvePlan &P, bool own_b, bool own_idx, bool own_st)
{
    size_t t = 0;
    const size_t nb = (size_t)P.n_bins, S = (size_t)P.S;
    if (own_b)
        t += sizeof(double) * nb * S;
    if (own_idx)
        t += sizeof(int32_t) * nb * S;
    if (own_st)
        t += sizeof(int32_t) * nb;
    if (P.p->select_mode == DAMAS_SEL_KEEP_COUNT)
        t += sizeof(int32_t) * nb;
    t += sizeof(int64_t) * (size_t)(P.nb_ws + 1);
    if (P.need64)
        t += sizeof(double) * (size_t)P.e_stride * P.nb_ws;
    if (P.need16)
        t += sizeof(uint16_t) * (size_t)P.e16_stride * P.nb_ws;
    if (P.need16 || !P.bf16)
        t += P.es * (size_t)P.a_elems;
    if (P.bf16 && P.need64)
        t += sizeof(float) * (size_t)P.a_elems;
    if (P.classes)
        t += sizeof(uint16_t) * (size_t)P.a_elems +
             sizeof(double) * (size_t)P.nb_ws * (size_t)psf_tiles(P.max_kept, P.steering) +
             (size_t)P.nb_ws;
    return t;
}

// Workspace, keep counts and the fault word of a plan on the context.
int prepare(damas_ctx *ctx, SolvePlan &P, double *b_map, int32_t *idx, int32_t *s_tilde,
            hipStream_t s)
{
    int rc;
    const damas_params *p = P.p;
    const int32_t n_bins = P.n_bins, S = P.S;
    if (!b_map && (rc = ensure(ctx, ctx->b, sizeof(double) * (size_t)n_bins * S, s, "b")))
        return rc;
    if (!idx && (rc = ensure(ctx, ctx->idx, sizeof(int32_t) * (size_t)n_bins * S, s, "idx")))
        return rc;
    if (!s_tilde && (rc = ensure(ctx, ctx->st, sizeof(int32_t) * (size_t)n_bins, s, "s_tilde")))
        return rc;
    if ((rc = ensure(ctx, ctx->off, sizeof(int64_t) * (size_t)(P.nb_ws + 1), s, "offsets")))
        return rc;
    if (P.need64 && (rc = ensure(ctx, ctx->E, sizeof(double) * (size_t)P.e_stride * P.nb_ws, s,
                                 "steering rows")))
        return rc;
    if (P.need16 && (rc = ensure(ctx, ctx->E16,
                                 sizeof(uint16_t) * (size_t)P.e16_stride * P.nb_ws, s,
                                 "bf16 steering rows")))
        return rc;
    if ((P.need16 || !P.bf16) &&
        (rc = ensure(ctx, ctx->A, P.es * (size_t)P.a_elems, s, "A arena")))
        return rc;
    if (P.bf16 && P.need64 &&
        (rc = ensure(ctx, ctx->A32, sizeof(float) * (size_t)P.a_elems, s, "FP32 A arena")))
        return rc;
    if (P.classes &&
        ((rc = ensure(ctx, ctx->Alo, sizeof(uint16_t) * (size_t)P.a_elems, s, "lo arena")) ||
         (rc = ensure(ctx, ctx->tsum,
                      sizeof(double) * (size_t)P.nb_ws *
                          (size_t)psf_tiles(P.max_kept, P.steering),
                      s, "tile sums")) ||
         (rc = ensure(ctx, ctx->cls, (size_t)P.nb_ws, s, "bin classes"))))
        return rc;
    P.bm = b_map ? b_map : (double *)ctx->b.p;
    P.ix = idx ? idx : (int32_t *)ctx->idx.p;
    P.st = s_tilde ? s_tilde : (int32_t *)ctx->st.p;
    P.off = (int64_t *)ctx->off.p;

    P.kc = nullptr;
    if (p->select_mode == DAMAS_SEL_KEEP_COUNT) {
        std::vector<int32_t> want(n_bins);
        for (int f = 0; f < n_bins; ++f)
            want[f] = p->keep_count ? p->keep_count[f] : p->keep_count_all;
        if (want != ctx->kc_host) {
            if ((rc = ensure(ctx, ctx->kc, sizeof(int32_t) * (size_t)n_bins, s, "keep counts")))
                return rc;
            // The staging buffer may still feed the previous upload.
            HIP_TRY(hipEventSynchronize(ctx->kc_done), "hipEventSynchronize");
            if (ctx->kc_pinned_n < (size_t)n_bins) {
                if (ctx->kc_pinned)
                    HIP_TRY(hipHostFree(ctx->kc_pinned), "hipHostFree");
                ctx->kc_pinned = nullptr;
                ctx->kc_pinned_n = 0;
                HIP_TRY(hipHostMalloc((void **)&ctx->kc_pinned, sizeof(int32_t) * n_bins),
                        "hipHostMalloc");
                ctx->kc_pinned_n = n_bins;
            }
            memcpy(ctx->kc_pinned, want.data(), sizeof(int32_t) * n_bins);
            HIP_TRY(hipMemcpyAsync(ctx->kc.p, ctx->kc_pinned, sizeof(int32_t) * n_bins,
                                   hipMemcpyHostToDevice, s),
                    "upload keep counts");
            HIP_TRY(hipEventRecord(ctx->kc_done, s), "hipEventRecord");
            ctx->kc_host = want;
        }
        P.kc = (const int32_t *)ctx->kc.p;
    }
    P.fault = ctx->fault;
    return DAMAS_OK;
}

// Cooperative schedule of a batched solve, from the kept counts the host
// knows.  The work of a bin is ld^2 (A elements per sweep).  With G
// workgroups (the context's budget within the device's co-resident
// capacity) and T = total work / G, a bin above 1.25 T (the split knob)
// gets ceil(work / T) ranks (at most gs_max_ranks(), at least kCoopMinRows
// rows each, three tiles), each the first job of its own workgroup; the
// other bins, largest
// first, form a queue the workgroups take from when their ranks are done
// (the estimate places them on the least loaded workgroups).  The schedule is
// used only if its estimated makespan (ranks cost kCoopOverhead more per
// element than a bin alone) beats one workgroup per bin by 10 %.
// tab: header (queue length, offset of the ranges, offset of the jobs), the
// queue of bins alone (longest first), [first, end) of the static jobs per
// workgroup, then (bin, rank, ranks) per static job.
int plan_coop(damas_ctx *ctx, const SolvePlan &P, std::vector<int32_t> &tab, int *gpw,
              const uint8_t *cls = nullptr)
{
    if (ctx->coop_budget == 0 || !ctx->tune.coop || ctx->capturing || !P.batched ||
        P.st_host.empty())
        return 0;
    const int kCoopMinRows = ctx->tune.min_rows;
    const double kCoopOverhead = ctx->tune.overhead, kSplit = ctx->tune.split;
    // Cost of a bin: tiles x max(floor, rows summed per tile).  A tile's
    // period is the larger of the row chain (about a fixed time) and the
    // strip sum (proportional to its rows); floor = 0 keeps ld^2.
    const double kFloor = ctx->tune.floor_rows;
    auto cost = [&](int st, double rows) {
        return (double)((st + 63) / 64) * std::max(kFloor, rows);
    };
    // A wide bin's elements cost more (6 bytes, FP64 products): its work is
    // scaled by the context's wide_cost when the classes are known.
    const int nb = P.n_bins;
    auto scale = [&](int f) {
        return cls && cls[f] == kClsWide ? ctx->tune.wide_cost : 1.0;
    };
    int cap = gs_coop_capacity(P.bf16 ? DAMAS_PREC_BF16 : P.p->precision, P.max_kept,
                               P.classes && !P.bf16);
    if (P.bf16 && P.need64)
        cap = std::min(cap, gs_coop_capacity(DAMAS_PREC_FP32, P.max_kept, P.classes));
    const int G = ctx->coop_budget < 0 ? cap : std::min(ctx->coop_budget, cap);
    if (G < 1)
        return 0;
    std::vector<double> work(nb);
    double total = 0.0, plain_span = 0.0;
    for (int f = 0; f < nb; ++f) {
        const double l = (double)ld_of(P.st_host[f]);
        work[f] = (kFloor > 0.0 ? cost(P.st_host[f], l) : l * l) * scale(f);
        total += work[f];
        plain_span = std::max(plain_span, work[f]);
    }
    if (nb <= G && total <= 0.0)
        return 0;
    const double T = total / G;
    std::vector<int> ranks(nb, 1);
    int multi = 0;
    for (int f = 0; f < nb; ++f) {
        const int st = P.st_host[f];
        if (work[f] <= kSplit * T || (st + 63) / 64 < 3)
            continue;
        int r = (int)std::ceil(work[f] / T);
        r = std::min({r, gs_max_ranks(), std::max(st / kCoopMinRows, 1)});
        if (kFloor > 0.0) // ranks past ld / floor would not shorten the tiles
            r = std::min(r, std::max((int)(ld_of(st) / kFloor), 1));
        if (r > 1) {
            ranks[f] = r;
            multi += r;
        }
    }
    // Fit the ranked bins into G workgroups.
    while (multi > G) {
        int best = -1;
        for (int f = 0; f < nb; ++f)
            if (ranks[f] > 1 && (best < 0 || ranks[f] > ranks[best]))
                best = f;
        --ranks[best];
        --multi;
        if (ranks[best] == 1)
            --multi;
    }
    if (multi == 0 && nb <= G)
        return 0; // no bin would get a helper: one workgroup per bin
    // Workgroups: ranked bins' ranks first, each its own workgroup; the
    // bins alone form a queue, longest first, that workgroups take from once
    // their ranks are done.  The estimate of the makespan places them as
    // the queue would under the cost model (longest processing time onto
    // the least loaded workgroup).
    std::vector<double> load(G, 0.0);
    std::vector<int32_t> ranked; // (bin, rank, ranks) per ranked workgroup
    for (int f = 0; f < nb; ++f)
        if (ranks[f] > 1)
            for (int h = 0; h < ranks[f]; ++h) {
                load[ranked.size() / 3] =
                    kCoopOverhead *
                    (kFloor > 0.0 ? cost(P.st_host[f], (double)ld_of(P.st_host[f]) / ranks[f]) *
                                        scale(f)
                                  : work[f] / ranks[f]);
                ranked.insert(ranked.end(), {f, h, ranks[f]});
            }
    std::vector<int> solo;
    for (int f = 0; f < nb; ++f)
        if (ranks[f] == 1)
            solo.push_back(f);
    std::stable_sort(solo.begin(), solo.end(), [&](int a, int b) { return work[a] > work[b]; });
    for (int f : solo) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[k] += work[f];
    }
    const double span = *std::max_element(load.begin(), load.end());
    if (!(span < 0.9 * plain_span) && nb <= G)
        return 0;
    const int n_ranked = (int)(ranked.size() / 3);
    const int n_wg = std::min(G, n_ranked + (int)solo.size());
    const int n_q = (int)solo.size();
    tab.assign(3, 0);
    tab[0] = n_q;
    tab.insert(tab.end(), solo.begin(), solo.end());
    tab[1] = (int32_t)tab.size(); // ranges
    for (int w = 0; w < n_wg; ++w) { // workgroup w < n_ranked: static job w; others: none
        const int32_t first = std::min(w, n_ranked);
        tab.insert(tab.end(), {first, w < n_ranked ? first + 1 : first});
    }
    tab[2] = (int32_t)tab.size(); // jobs
    tab.insert(tab.end(), ranked.begin(), ranked.end());
    int gmax = 0;
    for (int f = 0; f < nb; ++f)
        for (int prec : {P.p->precision, (int)DAMAS_PREC_FP32})
            gmax = std::max(gmax, gs_groups_per_wave(prec, P.st_host[f], ranks[f]));
    *gpw = gmax;
    return n_wg;
}

// Upload a cooperative schedule to the context's table (pinned staging).
int upload_tab(damas_ctx *ctx, const std::vector<int32_t> &tab, hipStream_t s)
{
    int rc;
    if (tab == ctx->coop_tab_host && ctx->coop_tab.p)
        return DAMAS_OK; // the device table already holds it
    if ((rc = ensure(ctx, ctx->coop_tab, sizeof(int32_t) * tab.size(), s, "coop schedule")))
        return rc;
    HIP_TRY(hipEventSynchronize(ctx->coop_done), "hipEventSynchronize");
    if (ctx->coop_pinned_n < tab.size()) {
        if (ctx->coop_pinned)
            HIP_TRY(hipHostFree(ctx->coop_pinned), "hipHostFree");
        ctx->coop_pinned = nullptr;
        ctx->coop_pinned_n = 0;
        HIP_TRY(hipHostMalloc((void **)&ctx->coop_pinned, sizeof(int32_t) * tab.size()),
                "hipHostMalloc");
        ctx->coop_pinned_n = tab.size();
    }
    memcpy(ctx->coop_pinned, tab.data(), sizeof(int32_t) * tab.size());
    HIP_TRY(hipMemcpyAsync(ctx->coop_tab.p, ctx->coop_pinned, sizeof(int32_t) * tab.size(),
                           hipMemcpyHostToDevice, s),
            "upload coop schedule");
    HIP_TRY(hipEventRecord(ctx->coop_done, s), "hipEventRecord");
    ctx->coop_tab_host = tab;
    return DAMAS_OK;
}

// Class arguments of a solve's PSF launches: the lo arena, tile sums and
// class bytes of the context (offset by the caller for a part of a batch).
PsfClassArgs psf_classes(damas_ctx *ctx, const SolvePlan &P)
{
    PsfClassArgs pc;
    if (P.classes) {
        pc.lo = (uint16_t *)ctx->Alo.p;
        pc.tsum = (double *)ctx->tsum.p;
        pc.cls = (uint8_t *)ctx->cls.p;
        pc.rho_wide = P.rho_wide;
        pc.rho_f32 = P.bf16 ? P.rho_f32 : HUGE_VAL; // a float solve has no F32 class
        pc.wide_cap = gs_wide_capacity();
    }
    return pc;
}

// Steering and PSF(s) of bins [0, nb) (arrays, offsets `off`, steering rows
// E / E16 and the class arguments offset by the caller): the
// storage-precision system and, for BF16, the FP32 copy.
int enqueue_system(const SolvePlan &P, int32_t nb, int32_t max_kept, const double *freq,
                   const int32_t *ix, int32_t *st, const int64_t *off, double *E,
                   uint16_t *E16, void *A, void *A32, const PsfClassArgs &pc, hipStream_t s)
{
    if (P.need64) {
        HIP_TRY(launch_steer(P.kg, nb, freq, ix, st, max_kept, E, P.e_stride, P.fault, s,
                             P.steering),
                "steer launch");
        HIP_TRY(launch_psf(P.M, nb, st, max_kept, P.bf16 ? DAMAS_PREC_FP32 : P.p->precision, E,
                           P.e_stride, off, P.bf16 ? A32 : A, P.fault, s, pc, P.steering,
                           P.diag),
                "psf launch");
    }
    if (P.need16) {
        HIP_TRY(launch_steer16(P.kg, nb, freq, ix, st, max_kept, E16, P.e16_stride, P.fault, s),
                "steer16 launch");
        HIP_TRY(launch_psf16(P.M, nb, st, max_kept, E16, P.e16_stride, off, (uint16_t *)A,
                             P.fault, s, P.diag),
                "psf16 launch");
    }
    return DAMAS_OK;
}

// Schedule and sweeps of bins [0, nb) after their systems are built:
// cooperative job lists for a batched solve whose kept counts the host
// knows (P.st_host), else one workgroup per bin; `map` (device, or null)
// places bins of different grids.
int enqueue_sweeps(damas_ctx *ctx, const SolvePlan &P, int32_t nb, int32_t max_kept,
                   const double *bm, const int32_t *ix, const int32_t *st, const void *x_init,
                   void *x_map, hipStream_t s, double *power, const int64_t *map)
{
    const damas_params *p = P.p;
    const bool bf16 = P.bf16;
    int rc;
    GsClassArgs gca;
    gca.map = map;
    if (P.classes) {
        gca.cls = (const uint8_t *)ctx->cls.p;
        gca.lo = (const uint16_t *)ctx->Alo.p;
    }
    // Cooperative schedule (batched solves of host-known kept counts).  With
    // per-bin classes the schedule weighs wide bins by their cost, so the
    // classes the PSF chose come to the host first (one synchronisation of
    // the solve's stream, before the sweeps).  A captured solve neither
    // synchronises nor plans: it runs the schedule its graph holds.
    std::vector<int32_t> tab;
    int gpw = 0;
    const uint8_t *cls_host = nullptr;
    if (P.classes && nb == P.n_bins && ctx->coop_budget != 0 && ctx->tune.coop &&
        !ctx->capturing && P.batched && !P.st_host.empty()) {
        if (ctx->cls_pinned_n < (size_t)nb) {
            if (ctx->cls_pinned)
                HIP_TRY(hipHostFree(ctx->cls_pinned), "hipHostFree");
            ctx->cls_pinned = nullptr;
            ctx->cls_pinned_n = 0;
            HIP_TRY(hipHostMalloc((void **)&ctx->cls_pinned, (size_t)nb), "hipHostMalloc");
            ctx->cls_pinned_n = nb;
        }
        HIP_TRY(hipMemcpyAsync(ctx->cls_pinned, ctx->cls.p, (size_t)nb, hipMemcpyDeviceToHost,
                               s),
                "read classes");
        HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
        cls_host = ctx->cls_pinned;
    }
    int n_wg;
    const int32_t *tab_dev = nullptr;
    if (ctx->capturing) {
        n_wg = nb == P.n_bins && ctx->cap_tab ? ctx->cap_nwg : 0;
        gpw = ctx->cap_gpw;
        tab_dev = ctx->cap_tab;
        if (n_wg > 0 && (rc = ensure(ctx, ctx->coop_ws, gs_coop_ws_bytes(nb, max_kept), s,
                                     "coop exchange")))
            return rc;
    } else {
        n_wg = nb == P.n_bins ? plan_coop(ctx, P, tab, &gpw, cls_host) : 0;
        if (n_wg > 0) {
            if ((rc = upload_tab(ctx, tab, s)) ||
                (rc = ensure(ctx, ctx->coop_ws, gs_coop_ws_bytes(nb, max_kept), s,
                             "coop exchange")))
                return rc;
            tab_dev = (const int32_t *)ctx->coop_tab.p;
        }
    }
    ctx->last_workgroups = n_wg > 0 ? n_wg : nb;
    ctx->last_coop = n_wg > 0;
    ctx->last_gpw = gpw;
    // Gated contexts queue their sweeps behind the previous gated ones.
    std::unique_lock<std::mutex> gate;
    if (ctx->sweep_gate) {
        gate = std::unique_lock<std::mutex>(*ctx->sweep_gate_mu);
        HIP_TRY(hipStreamWaitEvent(s, *ctx->sweep_gate, 0), "hipStreamWaitEvent");
    }
    // Elements of A over the launch's bins (the workspace's capacity where
    // the host does not know the kept counts).
    double a_elems = 0.0;
    if (P.st_host.size() >= (size_t)nb)
        for (int f = 0; f < nb; ++f)
            a_elems += (double)ld_of(P.st_host[f]) * (double)ld_of(P.st_host[f]);
    else
        a_elems = (double)P.a_elems;
    auto sweeps = [&](int prec, const void *Ap, int iters, const void *xi,
                      const GsClassArgs &g) -> hipError_t {
        const double es = prec == DAMAS_PREC_FP64 ? 8.0 : prec == DAMAS_PREC_BF16 ? 2.0 : 4.0;
        const bool streamed = a_elems * es > kGsStreamBytes;
        if (n_wg > 0)
            return launch_gs_coop(P.N, nb, st, max_kept, ix, P.off, prec, 1, Ap, bm, iters, xi,
                                  x_map, P.fault, tab_dev, n_wg, gpw, streamed, ctx->coop_ws.p,
                                  g, s);
        return launch_gs(P.N, nb, st, max_kept, ix, P.off, prec, 1, Ap, bm, iters, xi, x_map,
                         P.fault, s, g);
    };
    // The last sweep launch of a bin writes its integrated power.
    if (!bf16) {
        GsClassArgs g = gca;
        g.iters_cls = p->iterations;
        g.power = power;
        HIP_TRY(sweeps(p->precision, ctx->A.p, p->iterations, x_init, g), "gs launch");
    } else {
        // Bulk sweeps on bf16 A, then the refinement sweeps on the FP32
        // copy, warm-started from the bulk result in place.  With classes,
        // bins of class F32 or wide skip the bulk and run every sweep in
        // the second launch.
        const void *xi = x_init;
        const bool second = P.refine > 0 || P.classes;
        if (P.bulk > 0 || (P.refine == 0 && !P.classes)) {
            GsClassArgs g;
            g.cls = gca.cls;
            g.map = map;
            g.iters_cls = 0;
            g.power = second ? nullptr : power;
            HIP_TRY(sweeps(DAMAS_PREC_BF16, ctx->A.p, P.bulk, xi, g), "gs launch (bf16)");
            xi = x_map;
        }
        if (second) {
            GsClassArgs g = gca;
            g.iters_cls = p->iterations;
            g.power = power;
            HIP_TRY(sweeps(DAMAS_PREC_FP32, ctx->A32.p, P.refine, xi, g),
                    "gs launch (fp32 refinement)");
        }
    }
    if (ctx->sweep_gate)
        HIP_TRY(hipEventRecord(*ctx->sweep_gate, s), "hipEventRecord");
    return DAMAS_OK;
}

// Timed phases of a solve: events around each (when the context times).
struct PhaseTimer {
    damas_ctx *ctx;
    hipStream_t s;
    std::pair<hipEvent_t, hipEvent_t> ev{};
    int begin()
    {
        if (!ctx->timing)
            return DAMAS_OK;
        int rc = pop_events(ctx, &ev);
        if (rc)
            return rc;
        HIP_TRY(hipEventRecord(ev.first, s), "hipEventRecord");
        return DAMAS_OK;
    }
    int end(int phase)
    {
        if (!ctx->timing)
            return DAMAS_OK;
        HIP_TRY(hipEventRecord(ev.second, s), "hipEventRecord");
        ctx->phase_events[phase].push_back(ev);
        return DAMAS_OK;
    }
};

// Everything after the DAS map and the selection for bins [f0, f0 + nb)
// (arrays offset by the caller): layout, steering and PSF(s) when `build`,
// then the sweeps.
int enqueue_system_and_sweeps(damas_ctx *ctx, const SolvePlan &P, int32_t nb,
                              int32_t max_kept, const double *freq, double *bm,
                              int32_t *ix, int32_t *st, const void *x_init, void *x_map,
                              hipStream_t s, bool build = true, double *power = nullptr)
{
    HIP_TRY(launch_layout(nb, st, max_kept, P.a_elems, P.off, P.fault, s), "layout launch");
    int rc;
    PhaseTimer sys{ctx, s}, sw{ctx, s};
    if ((rc = sys.begin()))
        return rc;
    // Per-bin classes: chosen by the float PSF, read by the sweeps.
    if (build && (rc = enqueue_system(P, nb, max_kept, freq, ix, st, P.off, (double *)ctx->E.p,
                                      (uint16_t *)ctx->E16.p, ctx->A.p, ctx->A32.p,
                                      psf_classes(ctx, P), s)))
        return rc;
    if ((rc = sys.end(DAMAS_PHASE_SYSTEM)) || (rc = sw.begin()) ||
        (rc = enqueue_sweeps(ctx, P, nb, max_kept, bm, ix, st, x_init, x_map, s, power,
                             nullptr)))
        return rc;
    return sw.end(DAMAS_PHASE_SWEEPS);
}

// Copy n elements of T from host `src` to device `dst` through a pinned
// staging buffer that the previous upload (event `done`) no longer reads.
template <typename T>
int upload_pinned(T *&pinned, size_t &pinned_n, hipEvent_t done, void *dst, const T *src,
                  size_t n, hipStream_t s, const char *what)
{
    HIP_TRY(hipEventSynchronize(done), "hipEventSynchronize");
    if (pinned_n < n) {
        if (pinned)
            HIP_TRY(hipHostFree(pinned), "hipHostFree");
        pinned = nullptr;
        pinned_n = 0;
        HIP_TRY(hipHostMalloc((void **)&pinned, sizeof(T) * n), "hipHostMalloc");
        pinned_n = n;
    }
    memcpy(pinned, src, sizeof(T) * n);
    HIP_TRY(hipMemcpyAsync(dst, pinned, sizeof(T) * n, hipMemcpyHostToDevice, s), what);
    HIP_TRY(hipEventRecord(done, s), "hipEventRecord");
    return DAMAS_OK;
}

} // namespace

bool damas::merge_compatible(const damas_params &a, const damas_params &b)
{
    auto known = [](const damas_params &q) {
        return q.select_mode == DAMAS_SEL_KEEP_ALL || q.select_mode == DAMAS_SEL_KEEP_COUNT;
    };
    return known(a) && known(b) && a.precision == b.precision && a.iterations == b.iterations &&
           (a.precision != DAMAS_PREC_BF16 || a.refine_sweeps == b.refine_sweeps) &&
           a.policy == b.policy && a.rho_wide == b.rho_wide && a.rho_f32 == b.rho_f32;
}

int damas::merged_sizes(const std::vector<MergedPart> &parts, int64_t *map_elems, int64_t *bins)
{
    int64_t m = 0, b = 0;
    for (const MergedPart &q : parts) {
        m += (int64_t)q.n_bins * q.g.N * q.g.N;
        b += q.n_bins;
    }
    *map_elems = m;
    *bins = b;
    return DAMAS_OK;
}

int damas::solve_merged(damas_ctx *ctx, const std::vector<MergedPart> &parts, void *x_all,
                        int32_t *st_all, std::vector<int64_t> *bin0_out,
                        std::vector<int64_t> *map0_out, hipStream_t s)
{
    CtxScope scope(ctx);
    const int R = (int)parts.size();
    if (R == 0)
        return DAMAS_OK;
    if (!x_all)
        return fail(DAMAS_EINVAL, "x_all is NULL");
    std::vector<damas_params> pp(R);
    std::vector<SolvePlan> Ps(R);
    int rc;
    for (int r = 0; r < R; ++r) {
        const MergedPart &q = parts[r];
        pp[r] = q.p;
        pp[r].batched = 1;
        pp[r].power = nullptr;
        pp[r].keep_count = q.keep_count.empty() ? nullptr : q.keep_count.data();
        if ((rc = check_geometry(&q.g)) || (rc = make_plan(q.g.M, q.g.N, q.n_bins, &pp[r], Ps[r])))
            return rc;
        if (!q.freq || !q.csm || q.n_bins < 1)
            return fail(DAMAS_EINVAL, "part %d: freq, csm and n_bins >= 1 needed", r);
        if (!merge_compatible(pp[0], pp[r]))
            return fail(DAMAS_EINVAL, "part %d's sweep settings or selection mode cannot join "
                                      "the batch", r);
        Ps[r].kg = make_geom(q.g);
        Ps[r].fault = ctx->fault;
    }
    // Bins, maps, steering rows, arena elements and tile sums of each part.
    std::vector<int64_t> bin0(R), map0(R), e0(R), e16_0(R), tile0(R);
    int64_t B = 0, maps = 0, et = 0, e16t = 0, at = 0, tt = 0;
    int32_t max_kept = 0, Nmax = 0;
    std::vector<int32_t> st_all_host, kc_all;
    std::vector<int64_t> table;
    for (int r = 0; r < R; ++r) {
        const SolvePlan &P = Ps[r];
        bin0[r] = B;
        map0[r] = maps;
        e0[r] = et;
        e16_0[r] = e16t;
        tile0[r] = tt;
        for (int f = 0; f < P.n_bins; ++f) {
            table.push_back(maps + (int64_t)f * P.S);
            table.push_back(P.S);
            kc_all.push_back(pp[r].keep_count ? pp[r].keep_count[f] : pp[r].keep_count_all);
        }
        st_all_host.insert(st_all_host.end(), P.st_host.begin(), P.st_host.end());
        B += P.n_bins;
        maps += (int64_t)P.n_bins * P.S;
        if (P.need64)
            et += P.e_stride * P.n_bins;
        if (P.need16)
            e16t += P.e16_stride * P.n_bins;
        at += P.a_elems;
        if (P.classes)
            tt += (int64_t)P.n_bins * psf_tiles(P.max_kept, P.steering);
        max_kept = std::max(max_kept, P.max_kept);
        Nmax = std::max(Nmax, P.N);
    }
    if (B > (int64_t)1 << 24 || maps > ((int64_t)1 << 40))
        return fail(DAMAS_EINVAL, "merged batch too large (%lld bins)", (long long)B);
    // The batch as one plan: part 0's sweep settings, every bin's count.
    SolvePlan Pm = Ps[0];
    Pm.n_bins = (int32_t)B;
    Pm.nb_ws = (int32_t)B;
    Pm.st_host = st_all_host;
    Pm.max_kept = max_kept;
    Pm.a_elems = at;
    Pm.N = Nmax;
    Pm.S = Nmax * Nmax;
    const SolvePlan &P0 = Ps[0];
    if ((rc = ensure(ctx, ctx->b, sizeof(double) * (size_t)maps, s, "b")) ||
        (rc = ensure(ctx, ctx->idx, sizeof(int32_t) * (size_t)maps, s, "idx")) ||
        (!st_all && (rc = ensure(ctx, ctx->st, sizeof(int32_t) * (size_t)B, s, "s_tilde"))) ||
        (rc = ensure(ctx, ctx->kc, sizeof(int32_t) * (size_t)B, s, "keep counts")) ||
        (rc = ensure(ctx, ctx->off, sizeof(int64_t) * (size_t)(B + 1), s, "offsets")) ||
        (rc = ensure(ctx, ctx->mapt, sizeof(int64_t) * (size_t)(2 * B), s, "map table")) ||
        (P0.need64 &&
         (rc = ensure(ctx, ctx->E, sizeof(double) * (size_t)et, s, "steering rows"))) ||
        (P0.need16 &&
         (rc = ensure(ctx, ctx->E16, sizeof(uint16_t) * (size_t)e16t, s, "bf16 steering rows"))) ||
        ((P0.need16 || !P0.bf16) &&
         (rc = ensure(ctx, ctx->A, P0.es * (size_t)at, s, "A arena"))) ||
        (P0.bf16 && P0.need64 &&
         (rc = ensure(ctx, ctx->A32, sizeof(float) * (size_t)at, s, "FP32 A arena"))))
        return rc;
    if (P0.classes &&
        ((rc = ensure(ctx, ctx->Alo, sizeof(uint16_t) * (size_t)at, s, "lo arena")) ||
         (rc = ensure(ctx, ctx->tsum, sizeof(double) * (size_t)tt, s, "tile sums")) ||
         (rc = ensure(ctx, ctx->cls, (size_t)B, s, "bin classes"))))
        return rc;
    // Keep counts and the map table (pinned staging; the kept-count cache
    // of single solves no longer describes ctx->kc).
    ctx->kc_host.clear();
    if ((rc = upload_pinned(ctx->kc_pinned, ctx->kc_pinned_n, ctx->kc_done, ctx->kc.p,
                            kc_all.data(), kc_all.size(), s, "upload keep counts")) ||
        (rc = upload_pinned(ctx->mapt_pinned, ctx->mapt_pinned_n, ctx->kc_done, ctx->mapt.p,
                            table.data(), table.size(), s, "upload map table")))
        return rc;
    double *bm = (double *)ctx->b.p;
    int32_t *ix = (int32_t *)ctx->idx.p;
    int32_t *st = st_all ? st_all : (int32_t *)ctx->st.p;
    int64_t *off = (int64_t *)ctx->off.p;
    const int32_t *kc = (const int32_t *)ctx->kc.p;
    for (int r = 0; r < R; ++r) {
        const SolvePlan &P = Ps[r];
        const MergedPart &q = parts[r];
        HIP_TRY(launch_das(P.kg, P.n_bins, q.freq, q.csm, bm + map0[r], s, P.steering, P.diag),
                "das launch");
        HIP_TRY(launch_select(P.N, P.n_bins, bm + map0[r], pp[r].select_mode, pp[r].eps,
                              pp[r].predictor,
                              pp[r].select_mode == DAMAS_SEL_KEEP_COUNT ? kc + bin0[r] : nullptr,
                              ix + map0[r], st + bin0[r], s),
                "select launch");
    }
    HIP_TRY(launch_layout((int)B, st, max_kept, at, off, ctx->fault, s), "layout launch");
    PhaseTimer sys{ctx, s}, sw{ctx, s};
    if ((rc = sys.begin()))
        return rc;
    for (int r = 0; r < R; ++r) {
        const SolvePlan &P = Ps[r];
        PsfClassArgs pc = psf_classes(ctx, P);
        if (P.classes) {
            pc.tsum += tile0[r];
            pc.cls += bin0[r];
        }
        if ((rc = enqueue_system(P, P.n_bins, P.max_kept, parts[r].freq, ix + map0[r],
                                 st + bin0[r], off + bin0[r], (double *)ctx->E.p + e0[r],
                                 (uint16_t *)ctx->E16.p + e16_0[r], ctx->A.p, ctx->A32.p, pc,
                                 s)))
            return rc;
    }
    Pm.bm = bm;
    Pm.ix = ix;
    Pm.st = st;
    Pm.off = off;
    Pm.kc = kc;
    Pm.fault = ctx->fault;
    if ((rc = sys.end(DAMAS_PHASE_SYSTEM)) || (rc = sw.begin()) ||
        (rc = enqueue_sweeps(ctx, Pm, (int32_t)B, max_kept, bm, ix, st, nullptr, x_all, s,
                             nullptr, (const int64_t *)ctx->mapt.p)) ||
        (rc = sw.end(DAMAS_PHASE_SWEEPS)))
        return rc;
    if (bin0_out)
        *bin0_out = bin0;
    if (map0_out)
        *map0_out = map0;
    return DAMAS_OK;
}

extern "C" int damas_query_footprint(int32_t M, int32_t N, int32_t n_bins,
                                     const damas_params *p, uint64_t *bytes)
{
    if (!bytes)
        return fail(DAMAS_EINVAL, "bytes is NULL");
    if (M < 1 || M > 128)
        return fail(DAMAS_EINVAL, "M = %d outside [1, 128]", M);
    if (N < 1 || N > 46340)
        return fail(DAMAS_EINVAL, "N = %d outside [1, 46340]", N);
    damas_params pn;
    int rc = resolve_frac(p, N, pn, &p);
    if (rc)
        return rc;
    SolvePlan P;
    rc = make_plan(M, N, n_bins, p, P);
    if (rc)
        return rc;
    const size_t nb = (size_t)n_bins, S = (size_t)P.S;
    // Inputs (mic, freq, CSM), the x map and s_tilde, plus the workspace
    // of a context that keeps b and idx itself.
    size_t t = sizeof(double) * (3 * (size_t)M + nb + nb * (size_t)M * M * 2);
    t += P.xs * nb * S + sizeof(int32_t) * nb;
    t += plan_workspace_bytes(P, true, true, false);
    *bytes = t;
    return DAMAS_OK;
}

extern "C" int damas_solve_dev(damas_ctx *ctx, const damas_geometry *g,
                               int32_t n_bins, const double *freq,
                               const double *csm, const damas_params *p,
                               const void *x_init, void *x_map, double *b_map,
                               int32_t *idx, int32_t *s_tilde, void *stream)
{
    CtxScope scope(ctx);
    if (!ctx)
        return fail(DAMAS_EINVAL, "ctx is NULL");
    int rc = check_geometry(g);
    if (rc)
        return rc;
    damas_params pn;
    if ((rc = resolve_frac(p, g->N, pn, &p)))
        return rc;
    SolvePlan P;
    if ((rc = make_plan(g->M, g->N, n_bins, p, P)))
        return rc;
    if (n_bins == 0)
        return DAMAS_OK;
    if (!freq || !csm || !x_map)
        return fail(DAMAS_EINVAL, "freq, csm and x_map must be non-NULL");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    P.kg = make_geom(*g);
    if ((rc = prepare(ctx, P, b_map, idx, s_tilde, s)))
        return rc;
    const int32_t S = P.S, M = P.M;

    if (P.batched) {
        HIP_TRY(launch_das(P.kg, n_bins, freq, csm, P.bm, s, P.steering, P.diag), "das launch");
        HIP_TRY(launch_select(P.N, n_bins, P.bm, p->select_mode, p->eps, p->predictor, P.kc, P.ix,
                              P.st, s),
                "select launch");
        return enqueue_system_and_sweeps(ctx, P, n_bins, P.max_kept, freq, P.bm, P.ix, P.st,
                                         x_init, x_map, s, true, p->power);
    }

    // Plain: each bin on its own, one launch per step; A, E and the layout
    // are reused from bin to bin.
    for (int f = 0; f < n_bins; ++f) {
        const int32_t mk = P.st_host.empty() ? P.max_kept : P.st_host[f];
        const size_t fS = (size_t)f * S;
        const char *xi = x_init ? (const char *)x_init + P.xs * fS : nullptr;
        char *xm = (char *)x_map + P.xs * fS;
        HIP_TRY(launch_das(P.kg, 1, freq + f, csm + (size_t)f * M * M * 2, P.bm + fS, s,
                           P.steering, P.diag),
                "das launch");
        HIP_TRY(launch_select(P.N, 1, P.bm + fS, p->select_mode, p->eps, p->predictor,
                              P.kc ? P.kc + f : nullptr, P.ix + fS, P.st + f, s),
                "select launch");
        if ((rc = enqueue_system_and_sweeps(ctx, P, 1, mk, freq + f, P.bm + fS, P.ix + fS,
                                            P.st + f, xi, xm, s, true,
                                            p->power ? p->power + f : nullptr)))
            return rc;
    }
    return DAMAS_OK;
}

// Host-pointer form of damas_solve_dev: the inputs are staged on the
// context's device, the solve runs on the null stream, and the outputs are
// copied back once damas_check has reported on it.
extern "C" int damas_solve(damas_ctx *ctx, const damas_geometry *g, int32_t n_bins,
                           const double *freq, const double *csm, const damas_params *p,
                           const void *x_init, void *x_map, double *b_map, int32_t *idx,
                           int32_t *s_tilde)
{
    CtxScope scope(ctx);
    if (!ctx || !g || !p)
        return fail(DAMAS_EINVAL, "ctx, g and p must be non-NULL");
    if (n_bins < 0)
        return fail(DAMAS_EINVAL, "n_bins < 0");
    int rc = check_precision(p->precision);
    if (rc)
        return rc;
    if (n_bins > 0 && (!freq || !csm || !x_map || !g->mic))
        return fail(DAMAS_EINVAL, "freq, csm, x_map and g->mic must be non-NULL");
    if (n_bins == 0)
        return DAMAS_OK;
    if (g->M < 1 || g->N < 1 || g->N > 46340)
        return fail(DAMAS_EINVAL, "M = %d or N = %d out of range", g->M, g->N);
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    const size_t nb = (size_t)n_bins, M = (size_t)g->M, S = (size_t)g->N * (size_t)g->N;
    const size_t xs = x_size(p->precision);
    struct Buf {
        void *p = nullptr;
        ~Buf() { if (p) (void)hipFree(p); }
    } dmic, dfreq, dcsm, dxi, dx, db, didx, dst, dpow;
    auto alloc = [](Buf &b, size_t n) { return hipMalloc(&b.p, n ? n : 1); };
    HIP_TRY(alloc(dmic, M * 3 * sizeof(double)), "hipMalloc");
    HIP_TRY(alloc(dfreq, nb * sizeof(double)), "hipMalloc");
    HIP_TRY(alloc(dcsm, nb * M * M * 2 * sizeof(double)), "hipMalloc");
    HIP_TRY(alloc(dx, nb * S * xs), "hipMalloc");
    if (x_init)
        HIP_TRY(alloc(dxi, nb * S * xs), "hipMalloc");
    if (b_map)
        HIP_TRY(alloc(db, nb * S * sizeof(double)), "hipMalloc");
    if (idx)
        HIP_TRY(alloc(didx, nb * S * sizeof(int32_t)), "hipMalloc");
    if (s_tilde)
        HIP_TRY(alloc(dst, nb * sizeof(int32_t)), "hipMalloc");
    if (p->power)
        HIP_TRY(alloc(dpow, nb * sizeof(double)), "hipMalloc");
    HIP_TRY(hipMemcpy(dmic.p, g->mic, M * 3 * sizeof(double), hipMemcpyHostToDevice), "copy");
    HIP_TRY(hipMemcpy(dfreq.p, freq, nb * sizeof(double), hipMemcpyHostToDevice), "copy");
    HIP_TRY(hipMemcpy(dcsm.p, csm, nb * M * M * 2 * sizeof(double), hipMemcpyHostToDevice),
            "copy");
    if (x_init)
        HIP_TRY(hipMemcpy(dxi.p, x_init, nb * S * xs, hipMemcpyHostToDevice), "copy");
    // idx entries past s_tilde are left as the caller had them
    if (idx)
        HIP_TRY(hipMemcpy(didx.p, idx, nb * S * sizeof(int32_t), hipMemcpyHostToDevice), "copy");
    damas_geometry gd = *g;
    gd.mic = (const double *)dmic.p;
    damas_params pd = *p;
    pd.power = (double *)dpow.p; // the host array is filled after the solve
    rc = damas_solve_dev(ctx, &gd, n_bins, (const double *)dfreq.p, (const double *)dcsm.p, &pd,
                         dxi.p, dx.p, (double *)db.p, (int32_t *)didx.p, (int32_t *)dst.p,
                         nullptr);
    if (rc)
        return rc;
    if ((rc = damas_check(ctx, nullptr)))
        return rc;
    HIP_TRY(hipMemcpy(x_map, dx.p, nb * S * xs, hipMemcpyDeviceToHost), "copy");
    if (b_map)
        HIP_TRY(hipMemcpy(b_map, db.p, nb * S * sizeof(double), hipMemcpyDeviceToHost), "copy");
    if (idx)
        HIP_TRY(hipMemcpy(idx, didx.p, nb * S * sizeof(int32_t), hipMemcpyDeviceToHost), "copy");
    if (s_tilde)
        HIP_TRY(hipMemcpy(s_tilde, dst.p, nb * sizeof(int32_t), hipMemcpyDeviceToHost), "copy");
    if (p->power)
        HIP_TRY(hipMemcpy(p->power, dpow.p, nb * sizeof(double), hipMemcpyDeviceToHost), "copy");
    return DAMAS_OK;
}

// ---------------------------------------------------------------------------
// internal: context bytes, trimming, cache, cached solve

size_t damas::ctx_bytes(const damas_ctx *ctx)
{
    size_t t = 0;
    for (const Buffer *b : {&ctx->b, &ctx->idx, &ctx->st, &ctx->kc, &ctx->off, &ctx->E, &ctx->A,
                            &ctx->E16, &ctx->A32, &ctx->Alo, &ctx->tsum, &ctx->cls,
                            &ctx->coop_ws, &ctx->coop_tab, &ctx->mapt})
        t += b->bytes;
    return t;
}

int damas::ctx_trim(damas_ctx *ctx)
{
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (ctx->graphs > 0)
        return fail(DAMAS_EBUSY, "a graph captured on this context still uses its workspace");
    ctx->coop_tab_host.clear();
    for (Buffer *b : {&ctx->b, &ctx->idx, &ctx->st, &ctx->off, &ctx->E, &ctx->A, &ctx->E16,
                      &ctx->A32, &ctx->Alo, &ctx->tsum, &ctx->cls, &ctx->coop_ws,
                      &ctx->coop_tab, &ctx->mapt}) {
        if (b->p)
            HIP_TRY(hipFree(b->p), "hipFree");
        b->p = nullptr;
        b->bytes = 0;
    }
    return DAMAS_OK;
}

int damas::set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    record(buf);
    return code;
}

damas_ctx *damas::ctx_scope_swap(damas_ctx *ctx)
{
    damas_ctx *prev = g_ctx_cur;
    g_ctx_cur = ctx;
    return prev;
}

bool damas::PsfCache::make_room(size_t need)
{
    return need <= budget && shrink_to(budget - need);
}

bool damas::PsfCache::shrink_to(size_t room)
{
    while (used > room && !lru.empty()) {
        const std::string *k = lru.back();
        auto it = map.find(*k);
        lru.pop_back();
        if (it == map.end())
            continue;
        for (Buffer *b : {&it->second.A, &it->second.A32, &it->second.Alo, &it->second.cls})
            if (b->p) {
                (void)hipFree(b->p); // synchronises: no copy still reads it
                used -= b->bytes;
            }
        if (it->second.ready)
            (void)hipEventDestroy(it->second.ready);
        map.erase(it);
    }
    return used <= room;
}

void damas::PsfCache::clear()
{
    for (auto &kv : map) {
        for (Buffer *b : {&kv.second.A, &kv.second.A32, &kv.second.Alo, &kv.second.cls})
            if (b->p)
                (void)hipFree(b->p);
        if (kv.second.ready)
            (void)hipEventDestroy(kv.second.ready);
    }
    map.clear();
    lru.clear();
    used = 0;
}

namespace {

template <typename T> void append(std::string &k, const T *v, size_t n)
{
    k.append(reinterpret_cast<const char *>(v), sizeof(T) * n);
}

} // namespace

int damas::solve_cached(damas_ctx *ctx, const damas_geometry *g, int32_t n_bins,
                        const double *freq, const double *csm, const damas_params *p,
                        void *x_map, int32_t *s_tilde, PsfCache *cache, int *hit, hipStream_t s)
{
    *hit = 0;
    int rc = check_geometry(g);
    if (rc)
        return rc;
    SolvePlan P;
    if ((rc = make_plan(g->M, g->N, n_bins, p, P)))
        return rc;
    if (!P.batched)
        return fail(DAMAS_EINVAL, "cached solves are batched");
    if (n_bins == 0)
        return DAMAS_OK;
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    P.kg = make_geom(*g);
    if ((rc = prepare(ctx, P, nullptr, nullptr, s_tilde, s)))
        return rc;
    HIP_TRY(launch_das(P.kg, n_bins, freq, csm, P.bm, s, P.steering, P.diag), "das launch");
    HIP_TRY(launch_select(P.N, n_bins, P.bm, p->select_mode, p->eps, p->predictor, P.kc, P.ix,
                              P.st, s),
            "select launch");
    if (!cache)
        return enqueue_system_and_sweeps(ctx, P, n_bins, P.max_kept, freq, P.bm, P.ix, P.st,
                                         nullptr, x_map, s);

    // The key: geometry, frequencies, precision and arithmetic split, and
    // every bin's kept points.
    std::vector<int32_t> st(n_bins);
    std::vector<int32_t> ix((size_t)n_bins * P.S);
    std::vector<double> mic(3 * (size_t)g->M), fr(n_bins);
    HIP_TRY(hipMemcpyAsync(st.data(), P.st, sizeof(int32_t) * n_bins, hipMemcpyDeviceToHost, s),
            "read s_tilde");
    HIP_TRY(hipMemcpyAsync(ix.data(), P.ix, sizeof(int32_t) * ix.size(), hipMemcpyDeviceToHost, s),
            "read idx");
    HIP_TRY(hipMemcpyAsync(mic.data(), g->mic, sizeof(double) * mic.size(),
                           hipMemcpyDeviceToHost, s),
            "read mic");
    HIP_TRY(hipMemcpyAsync(fr.data(), freq, sizeof(double) * n_bins, hipMemcpyDeviceToHost, s),
            "read freq");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    std::string key;
    const int32_t hdr[8] = {g->M,      g->N,      p->precision, P.need64,
                            P.need16,  P.classes, P.steering,   P.diag};
    const double box[8] = {g->x0, g->x1, g->y0, g->y1, g->z0, g->c, P.rho_wide, P.rho_f32};
    append(key, hdr, 8);
    append(key, box, P.classes ? 8 : 6);
    append(key, mic.data(), mic.size());
    append(key, fr.data(), fr.size());
    append(key, st.data(), st.size());
    for (int f = 0; f < n_bins; ++f)
        append(key, ix.data() + (size_t)f * P.S, (size_t)std::max(st[f], 0));

    // Bytes of the packed systems of exactly these kept counts (what the
    // layout step will give them; part of the key, so every entry under a
    // key has this size).  A bin over max_kept fails the solve: no caching.
    int64_t packed = 0;
    for (int32_t v : st) {
        if (v < 0 || v > P.max_kept)
            return enqueue_system_and_sweeps(ctx, P, n_bins, P.max_kept, freq, P.bm, P.ix, P.st,
                                             nullptr, x_map, s);
        packed += ld_of(v) * ld_of(v);
    }
    if (packed > P.a_elems)
        return fail(DAMAS_EINVAL, "packed systems (%lld elements) exceed the arena (%lld)",
                    (long long)packed, (long long)P.a_elems);
    const size_t a_bytes = (P.need16 || !P.bf16) ? P.es * (size_t)packed : 0;
    const size_t a32_bytes = (P.bf16 && P.need64) ? sizeof(float) * (size_t)packed : 0;
    const size_t lo_bytes = P.classes ? sizeof(uint16_t) * (size_t)packed : 0;
    const size_t cls_bytes = P.classes ? (size_t)n_bins : 0;
    {
        std::lock_guard<std::mutex> lk(cache->mu);
        auto it = cache->map.find(key);
        if (it != cache->map.end()) {
            ++cache->hits;
            cache->lru.erase(it->second.lru);
            cache->lru.push_front(&it->first);
            it->second.lru = cache->lru.begin();
            // The entry may have been filled on another stream.
            HIP_TRY(hipStreamWaitEvent(s, it->second.ready, 0), "hipStreamWaitEvent");
            if (it->second.A.bytes < a_bytes || it->second.A32.bytes < a32_bytes ||
                it->second.Alo.bytes < lo_bytes || it->second.cls.bytes < cls_bytes)
                return fail(DAMAS_EINVAL, "cached systems smaller than their key states");
            const std::pair<void *, std::pair<const Buffer *, size_t>> cp[] = {
                {ctx->A.p, {&it->second.A, a_bytes}},
                {ctx->A32.p, {&it->second.A32, a32_bytes}},
                {ctx->Alo.p, {&it->second.Alo, lo_bytes}},
                {ctx->cls.p, {&it->second.cls, cls_bytes}}};
            for (const auto &c : cp)
                if (c.second.second)
                    HIP_TRY(hipMemcpyAsync(c.first, c.second.first->p, c.second.second,
                                           hipMemcpyDeviceToDevice, s),
                            "cached systems");
            // The copies must finish before the entry can be evicted.
            HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
            *hit = 1;
        } else {
            ++cache->misses;
        }
    }
    if ((rc = enqueue_system_and_sweeps(ctx, P, n_bins, P.max_kept, freq, P.bm, P.ix, P.st,
                                        nullptr, x_map, s, !*hit)))
        return rc;
    if (*hit)
        return DAMAS_OK;
    // Store a copy of the systems just built, if they fit the budget.
    std::lock_guard<std::mutex> lk(cache->mu);
    const size_t all_bytes = a_bytes + a32_bytes + lo_bytes + cls_bytes;
    if (cache->map.count(key) || !cache->make_room(all_bytes))
        return DAMAS_OK;
    PsfCache::Entry e;
    e.key = key;
    for (auto pr : {std::make_pair(&e.A, std::make_pair(ctx->A.p, a_bytes)),
                    std::make_pair(&e.A32, std::make_pair(ctx->A32.p, a32_bytes)),
                    std::make_pair(&e.Alo, std::make_pair(ctx->Alo.p, lo_bytes)),
                    std::make_pair(&e.cls, std::make_pair(ctx->cls.p, cls_bytes))}) {
        if (!pr.second.second)
            continue;
        if (hipMalloc(&pr.first->p, pr.second.second) != hipSuccess) {
            (void)hipGetLastError();
            for (Buffer *b : {&e.A, &e.A32, &e.Alo, &e.cls})
                if (b->p)
                    (void)hipFree(b->p); // synchronises with its pending copy
            return DAMAS_OK;             // no room on the device: skip caching
        }
        pr.first->bytes = pr.second.second;
        HIP_TRY(hipMemcpyAsync(pr.first->p, pr.second.first, pr.second.second,
                               hipMemcpyDeviceToDevice, s),
                "cache copy");
    }
    if (hipEventCreateWithFlags(&e.ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(e.ready, s) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        for (Buffer *b : {&e.A, &e.A32, &e.Alo, &e.cls})
            if (b->p)
                (void)hipFree(b->p);
        if (e.ready)
            (void)hipEventDestroy(e.ready);
        return DAMAS_OK;
    }
    cache->used += all_bytes;
    auto ins = cache->map.emplace(key, std::move(e));
    cache->lru.push_front(&ins.first->first);
    ins.first->second.lru = cache->lru.begin();
    return DAMAS_OK;
}

// ---------------------------------------------------------------------------
// autotuner: the cooperative schedule's knobs, by timing trial solves

namespace {

// Key of a problem in the autotune cache: what the schedule is a function
// of (shape, precision and policy, the device's compute units, and the kept
// counts, hashed FNV-1a, or the bound on them when the host does not know
// them).
std::string tune_key(const damas_ctx *ctx, const SolvePlan &P)
{
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint32_t v) {
        for (int b = 0; b < 4; ++b) {
            h ^= (v >> (8 * b)) & 0xffu;
            h *= 1099511628211ull;
        }
    };
    if (P.st_host.empty())
        mix((uint32_t)P.max_kept);
    for (int32_t v : P.st_host)
        mix((uint32_t)v);
    char buf[160];
    snprintf(buf, sizeof buf, "M%d:N%d:B%d:P%d:A%d:R%d:cu%d:st%016llx", P.M, P.N, P.n_bins,
             P.p->precision, P.classes ? 1 : 0, P.refine, cus, (unsigned long long)h);
    return buf;
}

} // namespace

extern "C" int damas_ctx_autotune(damas_ctx *ctx, const damas_geometry *g, int32_t n_bins,
                                  const double *freq, const double *csm, const damas_params *p,
                                  int32_t trial_sweeps, void *stream, damas_tune_result *out)
{
    CtxScope scope(ctx);
    if (!ctx || !out || !p)
        return fail(DAMAS_EINVAL, "ctx, params and out must be non-NULL");
    if (trial_sweeps < 1)
        return fail(DAMAS_EINVAL, "trial_sweeps must be >= 1");
    int rc = check_geometry(g);
    if (rc)
        return rc;
    damas_params pn;
    if ((rc = resolve_frac(p, g->N, pn, &p)))
        return rc;
    SolvePlan P;
    if ((rc = make_plan(g->M, g->N, n_bins, p, P)))
        return rc;
    if (n_bins == 0 || !freq || !csm)
        return fail(DAMAS_EINVAL, "nothing to tune (n_bins, freq, csm)");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    auto report = [&](const TuneKnobs &k) {
        out->coop = k.coop;
        out->coop_min_rows = k.min_rows;
        out->coop_split = k.split;
        out->coop_overhead = k.overhead;
        out->coop_floor_rows = k.floor_rows;
        out->wide_cost = k.wide_cost;
    };
    // A problem the cache file holds takes its stored choice, untimed.
    std::string key;
    if (!ctx->tune_cache.empty()) {
        key = tune_key(ctx, P);
        auto it = ctx->tune_entries.find(key);
        if (it != ctx->tune_entries.end()) {
            ctx->tune = it->second.first;
            report(ctx->tune);
            out->best_ms_per_sweep = it->second.second;
            out->default_ms_per_sweep = 0.0;
            out->candidates_timed = 0;
            return DAMAS_OK;
        }
    }
    // Trials: the caller's solve, batched, with trial_sweeps sweeps (for
    // BF16, all on the storage precision), into a scratch map.
    damas_params tp = *p;
    tp.batched = 1;
    tp.iterations = trial_sweeps;
    tp.refine_sweeps = 0;
    void *xm = nullptr;
    const size_t xbytes = P.xs * (size_t)n_bins * P.S;
    if (hipMalloc(&xm, std::max(xbytes, (size_t)256)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DAMAS_ENOMEM, "autotune map (%zu bytes)", xbytes);
    }
    const auto saved = ctx->tune;
    const bool saved_timing = ctx->timing;
    struct Cand {
        bool coop;
        int min_rows;
        double split, overhead;
        int floor_rows;
        double wide_cost;
    };
    const double wc0 = saved.wide_cost;
    std::vector<Cand> cands = {{false, 320, 1.25, 1.3, 0, wc0}, {true, 320, 1.25, 1.3, 0, wc0}};
    for (int fl : {0, 640, 1280})
        for (int mr : {256, 320, 512, 1024})
            for (double sp : {1.0, 1.25, 2.0})
                for (double ov : {1.1, 1.3, 1.6})
                    cands.push_back({true, mr, sp, ov, fl, wc0});
    // One trial solve first: it warms up and, under the per-bin policy,
    // gives the classes the schedules are planned with.
    ctx->timing = true;
    rc = damas_solve_dev(ctx, g, n_bins, freq, csm, &tp, nullptr, xm, nullptr, nullptr,
                         nullptr, s);
    if (rc == DAMAS_OK)
        rc = damas_check(ctx, s);
    std::vector<uint8_t> cls;
    bool any_wide = false;
    if (rc == DAMAS_OK && P.classes) {
        cls.resize(n_bins);
        if (hipMemcpy(cls.data(), ctx->cls.p, (size_t)n_bins, hipMemcpyDeviceToHost) !=
            hipSuccess)
            rc = fail(DAMAS_EDEVICE, "read classes");
        for (uint8_t c : cls)
            any_wide = any_wide || c == kClsWide;
    }
    {
        double t = 0.0;
        int64_t n = 0;
        (void)damas_ctx_phase_time(ctx, DAMAS_PHASE_SWEEPS, &t, &n);
    }
    // Candidates that produce the same schedule are timed once.
    std::map<std::vector<int32_t>, double> timed;
    int ran = 0;
    auto apply = [&](const Cand &c) {
        ctx->tune.coop = c.coop;
        ctx->tune.min_rows = c.min_rows;
        ctx->tune.split = c.split;
        ctx->tune.overhead = c.overhead;
        ctx->tune.floor_rows = c.floor_rows;
        ctx->tune.wide_cost = c.wide_cost;
    };
    auto time_cand = [&](const Cand &c, double *ms, bool again = false) -> int {
        apply(c);
        std::vector<int32_t> tab;
        int gpw = 0;
        if (plan_coop(ctx, P, tab, &gpw, cls.empty() ? nullptr : cls.data()) == 0)
            tab.clear(); // one workgroup per bin
        auto it = timed.find(tab);
        if (it != timed.end() && !again) {
            *ms = it->second;
            return DAMAS_OK;
        }
        int r = DAMAS_OK;
        int64_t n = 0;
        for (int rep = 0; rep < 2 && r == DAMAS_OK; ++rep) {
            double t = 0.0;
            (void)damas_ctx_phase_time(ctx, DAMAS_PHASE_SWEEPS, &t, &n);
            r = damas_solve_dev(ctx, g, n_bins, freq, csm, &tp, nullptr, xm, nullptr, nullptr,
                                nullptr, s);
            if (r == DAMAS_OK)
                r = damas_check(ctx, s);
            if (r == DAMAS_OK)
                r = damas_ctx_phase_time(ctx, DAMAS_PHASE_SWEEPS, ms, &n);
        }
        if (r == DAMAS_OK) {
            if (it != timed.end())
                *ms = std::min(*ms, it->second); // a schedule keeps its lowest time
            timed[tab] = *ms;
            if (!again)
                ++ran;
        }
        return r;
    };
    double best = 1e300, dflt = 0.0;
    size_t bi = 0;
    std::vector<std::pair<double, size_t>> scan; // (time, candidate) of the grid
    for (size_t c = 0; c < cands.size() && rc == DAMAS_OK; ++c) {
        double ms = 0.0;
        if ((rc = time_cand(cands[c], &ms)))
            break;
        scan.push_back({ms, c});
        if (c == 1)
            dflt = ms; // the untuned knobs
        if (ms < best) {
            best = ms;
            bi = c;
        }
    }
    // With wide bins, the cost of their elements in the schedule, around
    // the three fastest cooperative grid points (the best wide cost depends
    // on the other knobs: around the single best point the search missed
    // schedules 4 % faster).
    if (rc == DAMAS_OK && any_wide) {
        std::stable_sort(scan.begin(), scan.end());
        std::vector<size_t> bases;
        std::set<std::vector<int32_t>> distinct;
        for (const auto &e : scan) {
            if (!cands[e.second].coop || bases.size() >= 3)
                continue;
            apply(cands[e.second]);
            std::vector<int32_t> tab;
            int gpw = 0;
            if (plan_coop(ctx, P, tab, &gpw, cls.empty() ? nullptr : cls.data()) == 0)
                tab.clear();
            if (distinct.insert(tab).second)
                bases.push_back(e.second);
        }
        for (size_t b : bases) {
            const Cand base = cands[b];
            for (double wcost : {1.0, 1.35, 2.1, 2.6}) {
                Cand c = base;
                c.wide_cost = wcost;
                double ms = 0.0;
                if ((rc = time_cand(c, &ms)))
                    break;
                cands.push_back(c);
                if (ms < best) {
                    best = ms;
                    bi = cands.size() - 1;
                }
            }
            if (rc)
                break;
        }
    }
    // The schedules within 5 % of the best are timed twice more, in turn,
    // each keeping its lowest time: one trial varies by a few percent, and a
    // schedule chosen on a single trial lost up to 4 % on the full solve.
    if (rc == DAMAS_OK) {
        std::vector<std::pair<double, size_t>> near; // (time, candidate), one per schedule
        std::map<std::vector<int32_t>, size_t> seen;
        for (size_t c = 0; c < cands.size(); ++c) {
            apply(cands[c]);
            std::vector<int32_t> tab;
            int gpw = 0;
            if (plan_coop(ctx, P, tab, &gpw, cls.empty() ? nullptr : cls.data()) == 0)
                tab.clear();
            auto it = timed.find(tab);
            if (it != timed.end() && it->second <= 1.05 * best && seen.emplace(tab, c).second)
                near.push_back({it->second, c});
        }
        std::sort(near.begin(), near.end());
        if (near.size() > 4)
            near.resize(4);
        for (int pass = 0; pass < 2 && near.size() > 1 && rc == DAMAS_OK; ++pass)
            for (auto &e : near) {
                if ((rc = time_cand(cands[e.second], &e.first, true)))
                    break;
            }
        if (rc == DAMAS_OK && near.size() > 1) {
            const auto w = std::min_element(near.begin(), near.end());
            best = w->first;
            bi = w->second;
        }
    }
    double t = 0.0;
    int64_t n = 0;
    (void)damas_ctx_phase_time(ctx, DAMAS_PHASE_SYSTEM, &t, &n);
    ctx->timing = saved_timing;
    (void)hipFree(xm);
    if (rc) {
        ctx->tune = saved;
        return rc;
    }
    apply(cands[bi]);
    report(ctx->tune);
    out->best_ms_per_sweep = best / trial_sweeps;
    out->default_ms_per_sweep = dflt / trial_sweeps;
    out->candidates_timed = ran;
    if (!key.empty()) {
        ctx->tune_entries[key] = {ctx->tune, out->best_ms_per_sweep};
        const TuneKnobs &k = ctx->tune;
        bool ok = false;
        if (FILE *fh = fopen(ctx->tune_cache.c_str(), "a")) {
            ok = fprintf(fh, "%s %d %d %.17g %.17g %d %.17g %.17g\n", key.c_str(),
                         k.coop ? 1 : 0, k.min_rows, k.split, k.overhead, k.floor_rows,
                         k.wide_cost, out->best_ms_per_sweep) >= 0;
            ok = fclose(fh) == 0 && ok;
        }
        if (!ok)
            return fail(DAMAS_EINVAL,
                        "the tuned choice is applied, but the autotune cache %s could not be "
                        "written",
                        ctx->tune_cache.c_str());
    }
    return DAMAS_OK;
}

extern "C" int damas_ctx_set_schedule(damas_ctx *ctx, const damas_tune_result *k)
{
    CtxScope scope(ctx);
    if (!ctx || !k)
        return fail(DAMAS_EINVAL, "ctx and knobs must be non-NULL");
    if (!knobs_valid(k->coop, k->coop_min_rows, k->coop_split, k->coop_overhead,
                     k->coop_floor_rows, k->wide_cost))
        return fail(DAMAS_EINVAL, "schedule knobs out of range");
    ctx->tune.coop = k->coop == 1;
    ctx->tune.min_rows = k->coop_min_rows;
    ctx->tune.split = k->coop_split;
    ctx->tune.overhead = k->coop_overhead;
    ctx->tune.floor_rows = k->coop_floor_rows;
    ctx->tune.wide_cost = k->wide_cost;
    return DAMAS_OK;
}

// ---------------------------------------------------------------------------
// graphs: a whole-path solve captured once, replayed on any stream

struct damas_graph {
    damas_ctx *ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t *tab = nullptr; // the cooperative schedule the graph replays (or null)
    int workgroups = 0;     // of its sweep launches
};

// Set the cooperative attribute on the graph's sweep kernel nodes.
static int mark_coop_nodes(hipGraph_t graph)
{
    size_t n = 0;
    if (hipGraphGetNodes(graph, nullptr, &n) != hipSuccess)
        return 1;
    std::vector<hipGraphNode_t> nodes(n);
    if (n && hipGraphGetNodes(graph, nodes.data(), &n) != hipSuccess)
        return 1;
    int marked = 0;
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType t;
        if (hipGraphNodeGetType(nd, &t) != hipSuccess)
            return 1;
        if (t != hipGraphNodeTypeKernel)
            continue;
        hipKernelNodeParams kp{};
        if (hipGraphKernelNodeGetParams(nd, &kp) != hipSuccess)
            return 1;
        if (!gs_is_coop_kernel(kp.func))
            continue;
        hipKernelNodeAttrValue v{};
        v.cooperative = 1;
        if (hipGraphKernelNodeSetAttribute(nd, hipKernelNodeAttributeCooperative, &v) !=
            hipSuccess)
            return 1;
        ++marked;
    }
    return marked > 0 ? 0 : 1;
}

extern "C" int damas_graph_capture(damas_ctx *ctx, const damas_geometry *g, int32_t n_bins,
                                   const double *freq, const double *csm,
                                   const damas_params *p, const void *x_init, void *x_map,
                                   double *b_map, int32_t *idx, int32_t *s_tilde,
                                   damas_graph **out)
{
    CtxScope scope(ctx);
    if (!ctx || !out)
        return fail(DAMAS_EINVAL, "ctx and out must be non-NULL");
    if (ctx->timing)
        return fail(DAMAS_EINVAL, "timing must be off while capturing");
    HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
    // One eager solve sizes every buffer, uploads the keep counts and, for a
    // batched solve of host-known kept counts, chooses the cooperative
    // schedule.  The graph keeps its own copy of that table, so later solves
    // on the context cannot change what it replays.
    int rc = damas_solve_dev(ctx, g, n_bins, freq, csm, p, x_init, x_map, b_map, idx, s_tilde,
                             s);
    if (rc == DAMAS_OK)
        rc = damas_check(ctx, s);
    int32_t *tab = nullptr;
    int nwg = 0, gpw = 0;
    if (rc == DAMAS_OK && ctx->last_coop) {
        const size_t bytes = sizeof(int32_t) * ctx->coop_tab_host.size();
        if (hipMalloc((void **)&tab, bytes) != hipSuccess) {
            (void)hipGetLastError();
            tab = nullptr;
            rc = fail(DAMAS_ENOMEM, "graph schedule table (%zu bytes)", bytes);
        } else if (hipMemcpy(tab, ctx->coop_tab_host.data(), bytes, hipMemcpyHostToDevice) !=
                   hipSuccess) {
            rc = fail(DAMAS_EDEVICE, "graph schedule table upload");
        }
        nwg = ctx->last_workgroups;
        gpw = ctx->last_gpw;
    }
    hipGraph_t graph = nullptr;
    if (rc == DAMAS_OK) {
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = fail(DAMAS_EDEVICE, "hipStreamBeginCapture");
        } else {
            ctx->capturing = ctx->in_capture = true;
            ctx->cap_tab = tab;
            ctx->cap_nwg = nwg;
            ctx->cap_gpw = gpw;
            rc = damas_solve_dev(ctx, g, n_bins, freq, csm, p, x_init, x_map, b_map, idx,
                                 s_tilde, s);
            ctx->capturing = ctx->in_capture = false;
            ctx->cap_tab = nullptr;
            const hipError_t e = hipStreamEndCapture(s, &graph);
            if (rc == DAMAS_OK && e != hipSuccess)
                rc = fail(DAMAS_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        }
    }
    // Capture records a cooperative launch as a plain kernel node; the
    // sweep nodes get the cooperative attribute back, so a replay launches
    // them as the eager solve does (all workgroups resident together).
    if (rc == DAMAS_OK && tab && (rc = mark_coop_nodes(graph)))
        rc = fail(DAMAS_EDEVICE, "marking the cooperative sweep nodes");
    (void)hipStreamDestroy(s);
    auto drop = [&](int code) {
        if (graph)
            (void)hipGraphDestroy(graph);
        if (tab)
            (void)hipFree(tab);
        return code;
    };
    if (rc)
        return drop(rc);
    damas_graph *gr = new (std::nothrow) damas_graph();
    if (!gr)
        return drop(fail(DAMAS_ENOMEM, "graph allocation"));
    if (hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        delete gr;
        return drop(fail(DAMAS_EDEVICE, "hipGraphInstantiate"));
    }
    gr->graph = graph;
    gr->ctx = ctx;
    gr->tab = tab;
    gr->workgroups = tab ? nwg : ctx->last_workgroups;
    ++ctx->graphs;
    *out = gr;
    return DAMAS_OK;
}

extern "C" int32_t damas_graph_workgroups(const damas_graph *gr)
{
    return gr ? gr->workgroups : 0;
}

extern "C" int damas_graph_launch(damas_graph *gr, void *stream)
{
    CtxScope scope(gr ? gr->ctx : nullptr);
    if (!gr)
        return fail(DAMAS_EINVAL, "graph is NULL");
    HIP_TRY(hipSetDevice(gr->ctx->device), "hipSetDevice");
    HIP_TRY(hipGraphLaunch(gr->exec, (hipStream_t)stream), "hipGraphLaunch");
    return DAMAS_OK;
}

extern "C" void damas_graph_destroy(damas_graph *gr)
{
    if (!gr)
        return;
    (void)hipSetDevice(gr->ctx->device);
    (void)hipDeviceSynchronize();
    if (gr->exec)
        (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph)
        (void)hipGraphDestroy(gr->graph);
    if (gr->tab)
        (void)hipFree(gr->tab);
    --gr->ctx->graphs;
    delete gr;
}

// ---------------------------------------------------------------------------
// whole-path solve without allocation: the workspace in a static device
// array

namespace {

// Workspace of damas_solve_static: one array per device, held for the
// process's lifetime.  Host code never passes the array's name to a kernel
// or copy (it is a host-side stand-in there); it uses the device address
// hipGetSymbolAddress returns for the current device, kept per device.
constexpr size_t kStaticScratchBytes = (size_t)96 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
std::unordered_map<int, unsigned char *> g_scratch;

// Device address of the current device's array, looked up once per
// device; *out is null (and DAMAS_OK returned) when `create` is false and
// no static solve has run on this device yet.
int scratch_addr(unsigned char **out, bool create = true)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        *out = it->second;
        return DAMAS_OK;
    }
    *out = nullptr;
    if (!create)
        return DAMAS_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(DAMAS_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch[dev] = (unsigned char *)p;
    *out = (unsigned char *)p;
    return DAMAS_OK;
}

// The static solve's fault word: the first 4 bytes of the array.
int static_fault(int **out)
{
    unsigned char *base = nullptr;
    int rc = scratch_addr(&base, false);
    *out = base ? (int *)base : nullptr;
    return rc;
}

// Clears n words (a kernel, not a memset node, so a captured graph replays
// it faithfully).
__global__ void static_fill_zero(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Sets n words to v.
__global__ void static_fill_value(uint32_t *p, int64_t n, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Bump allocation of 256-byte aligned regions from the array.
struct Carve {
    unsigned char *base;
    size_t used = 256; // bytes 0..255: the fault word
    void *take(size_t bytes)
    {
        void *p = base + used;
        used += (bytes + 255) & ~(size_t)255;
        return p;
    }
};

} // namespace

extern "C" int64_t damas_static_scratch_bytes(void) { return (int64_t)kStaticScratchBytes; }

extern "C" int damas_solve_static(const damas_geometry *g, int32_t n_bins, const double *freq,
                                  const double *csm, const damas_params *p,
                                  const int32_t *keep_count, const void *x_init, void *x_map,
                                  double *b_map, int32_t *idx, int32_t *s_tilde, void *stream)
{
    int rc = check_geometry(g);
    if (rc)
        return rc;
    if (!p)
        return fail(DAMAS_EINVAL, "params are NULL");
    // KEEP_FRAC: the host knows the count, so it also bounds max_kept; the
    // counts go to the device from the array.
    const bool frac = p->select_mode == DAMAS_SEL_KEEP_FRAC;
    damas_params pn;
    if ((rc = resolve_frac(p, g->N, pn, &p)))
        return rc;
    if (p->precision != DAMAS_PREC_FP64 && p->precision != DAMAS_PREC_FP32)
        return fail(DAMAS_EINVAL, "damas_solve_static solves at FP64 or FP32 (precision %d)",
                    p->precision);
    if ((rc = check_mode(p->select_mode, p->eps)))
        return rc;
    if (p->predictor != DAMAS_PRED_HAAR && p->predictor != DAMAS_PRED_LINEAR)
        return fail(DAMAS_EINVAL, "predictor = %d is not a DAMAS_PRED_* value", p->predictor);
    if (p->policy != DAMAS_POLICY_AUTO && p->policy != DAMAS_POLICY_FIXED)
        return fail(DAMAS_EINVAL, "policy = %d is not a DAMAS_POLICY_* value", p->policy);
    if (!(p->rho_wide >= 0.0))
        return fail(DAMAS_EINVAL, "rho_wide must be >= 0 (0: default)");
    if ((rc = check_form(p->steering, p->diag_removal, p->precision)))
        return rc;
    if (n_bins < 0 || p->iterations < 0)
        return fail(DAMAS_EINVAL, "n_bins and iterations must be >= 0");
    if (n_bins == 0)
        return DAMAS_OK;
    if (!freq || !csm || !x_map)
        return fail(DAMAS_EINVAL, "freq, csm and x_map must be non-NULL");
    if (p->select_mode == DAMAS_SEL_KEEP_COUNT && !keep_count && !frac)
        return fail(DAMAS_EINVAL, "KEEP_COUNT needs keep_count (device, n_bins int32)");
    const int32_t S = g->N * g->N, M = g->M;
    const int32_t frac_kept =
        frac ? std::min(std::max(p->keep_count_all, coarse_count(g->N)), S) : 0;
    const int32_t max_kept = p->select_mode == DAMAS_SEL_KEEP_ALL ? S
                             : frac ? frac_kept
                                    : (p->max_kept > 0 ? std::min(p->max_kept, S) : S);
    if ((rc = check_kept(max_kept, S, p->precision)))
        return rc;

    // Sizes of the workspace, all in the array.
    const bool classes = p->policy == DAMAS_POLICY_AUTO && p->precision == DAMAS_PREC_FP32;
    const size_t nb = (size_t)n_bins, es = elem_size(p->precision);
    const int64_t ldm = ld_of(max_kept);
    const int64_t e_stride = ldm * 2 * M * (p->steering == DAMAS_STEER_PAPER ? 2 : 1);
    const int64_t a_elems = (int64_t)n_bins * ldm * ldm;
    const int64_t tiles = psf_tiles(max_kept, p->steering);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t need = 256;
    need += b_map ? 0 : al(sizeof(double) * nb * S);
    need += idx ? 0 : al(sizeof(int32_t) * nb * S);
    need += s_tilde ? 0 : al(sizeof(int32_t) * nb);
    need += al(sizeof(int64_t) * (nb + 1)) + al(sizeof(double) * nb * e_stride) +
            al(es * (size_t)a_elems);
    if (frac)
        need += al(sizeof(int32_t) * nb);
    if (classes)
        need += al(sizeof(uint16_t) * (size_t)a_elems) + al(sizeof(double) * nb * tiles) +
                al(nb);
    if (need > kStaticScratchBytes)
        return fail(DAMAS_EINVAL,
                    "this solve needs %zu bytes of workspace; damas_solve_static holds %zu "
                    "(fewer bins, a smaller max_kept, or caller-supplied b_map/idx/s_tilde)",
                    need, kStaticScratchBytes);

    unsigned char *base = nullptr;
    if ((rc = scratch_addr(&base)))
        return rc;
    Carve c{base};
    int *fault = (int *)base;
    double *bm = b_map ? b_map : (double *)c.take(sizeof(double) * nb * S);
    int32_t *ix = idx ? idx : (int32_t *)c.take(sizeof(int32_t) * nb * S);
    int32_t *st = s_tilde ? s_tilde : (int32_t *)c.take(sizeof(int32_t) * nb);
    int64_t *off = (int64_t *)c.take(sizeof(int64_t) * (nb + 1));
    double *E = (double *)c.take(sizeof(double) * nb * e_stride);
    void *A = c.take(es * (size_t)a_elems);
    int32_t *kc = frac ? (int32_t *)c.take(sizeof(int32_t) * nb) : nullptr;
    PsfClassArgs pc;
    GsClassArgs gca;
    if (classes) {
        pc.lo = (uint16_t *)c.take(sizeof(uint16_t) * (size_t)a_elems);
        pc.tsum = (double *)c.take(sizeof(double) * nb * tiles);
        pc.cls = (uint8_t *)c.take(nb);
        pc.rho_wide = p->rho_wide > 0.0 ? p->rho_wide : DAMAS_RHO_WIDE_DEFAULT;
        pc.rho_f32 = HUGE_VAL;
        pc.wide_cap = gs_wide_capacity();
        gca.cls = pc.cls;
        gca.lo = pc.lo;
        gca.iters_cls = p->iterations;
    }
    gca.power = p->power;

    hipStream_t s = (hipStream_t)stream;
    const Geom kg = make_geom(*g);
    hipLaunchKernelGGL(static_fill_zero, dim3(1), dim3(64), 0, s, (uint32_t *)fault, (int64_t)1);
    HIP_TRY(hipGetLastError(), "fault word clear");
    if (frac) {
        hipLaunchKernelGGL(static_fill_value, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s,
                           (uint32_t *)kc, (int64_t)nb, (uint32_t)frac_kept);
        HIP_TRY(hipGetLastError(), "keep counts fill");
        keep_count = kc;
    }
    HIP_TRY(launch_das(kg, n_bins, freq, csm, bm, s, p->steering, p->diag_removal),
            "das launch");
    HIP_TRY(launch_select(g->N, n_bins, bm, p->select_mode, p->eps, p->predictor,
                          p->select_mode == DAMAS_SEL_KEEP_COUNT ? keep_count : nullptr, ix, st,
                          s),
            "select launch");
    HIP_TRY(launch_layout(n_bins, st, max_kept, a_elems, off, fault, s), "layout launch");
    HIP_TRY(launch_steer(kg, n_bins, freq, ix, st, max_kept, E, e_stride, fault, s,
                         p->steering),
            "steer launch");
    HIP_TRY(launch_psf(M, n_bins, st, max_kept, p->precision, E, e_stride, off, A, fault, s, pc,
                       p->steering, p->diag_removal),
            "psf launch");
    HIP_TRY(launch_gs(g->N, n_bins, st, max_kept, ix, off, p->precision, 1, A, bm,
                      p->iterations, x_init, x_map, fault, s, gca),
            "gs launch");
    return DAMAS_OK;
}
