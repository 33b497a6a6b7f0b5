"""Thin ctypes binding of ``libdamas_hip.so`` (C ABI in ``include/damas.h``).

Argument marshalling only: torch tensors supply device memory and torch's
current HIP stream; every step of the path runs in the library's kernels.
There is no fallback: if the library is missing, importing this module
fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdamas_hip.so")

OK = 0
EINVAL = -1
ENOMEM = -2
EDEVICE = -3
EADMIT = -4
EBUSY = -5
ETIMEDOUT = -6
ECAPACITY = -7

SEL_KEEP_ALL = 0
SEL_EPS_REL = 1
SEL_KEEP_COUNT = 2
SEL_KEEP_FRAC = 3
PRED_HAAR = 0
PRED_LINEAR = 1

PREC_FP64 = 0
PREC_FP32 = 1
PREC_BF16 = 2

STEER_UNIT = 0
STEER_PAPER = 1

POLICY_AUTO = 0
POLICY_FIXED = 1
CLASS_NARROW = 0
CLASS_FP32 = 1
CLASS_WIDE = 2

# Element type of A by precision, and of the x maps.
_DTYPE = {PREC_FP64: torch.float64, PREC_FP32: torch.float32, PREC_BF16: torch.bfloat16}
_XTYPE = {PREC_FP64: torch.float64, PREC_FP32: torch.float32, PREC_BF16: torch.float32}

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
        " (or python paper_1608_05179_amd/build.py)")

_lib = ctypes.CDLL(LIB_PATH)

c_i32, c_i64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class Geometry(ctypes.Structure):
    """damas_geometry: M mics (device M x 3 doubles), N x N scan grid on the
    plane z = z0 spanning [x0, x1] x [y0, y1], speed of sound c."""
    _fields_ = [("M", c_i32), ("mic", c_vp), ("N", c_i32), ("x0", c_dbl),
                ("x1", c_dbl), ("y0", c_dbl), ("y1", c_dbl), ("z0", c_dbl),
                ("c", c_dbl)]


class Params(ctypes.Structure):
    _fields_ = [("select_mode", c_i32), ("eps", c_dbl),
                ("keep_count", ctypes.POINTER(c_i32)), ("keep_count_all", c_i32),
                ("iterations", c_i32), ("precision", c_i32), ("batched", c_i32),
                ("max_kept", c_i32), ("refine_sweeps", c_i32), ("predictor", c_i32),
                ("policy", c_i32), ("rho_wide", c_dbl), ("rho_f32", c_dbl),
                ("steering", c_i32), ("diag_removal", c_i32), ("power", c_vp),
                ("keep_frac", c_dbl)]


def _sig(name, res, *args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = list(args)
    return fn


_sig("damas_strerror", ctypes.c_char_p, ctypes.c_int)
_sig("damas_last_error", ctypes.c_char_p)
_sig("damas_ld", c_i64, c_i32)
_sig("damas_coarse_count", c_i32, c_i32)
_sig("damas_mp", c_i32, c_i32)
_sig("damas_gs_capacity", c_i32, c_i32)
_sig("damas_wide_capacity", c_i32)
_G = ctypes.POINTER(Geometry)
_sig("damas_csm", ctypes.c_int, c_i32, c_i32, c_i32, c_vp, c_vp, c_vp)
_sig("damas_das_map", ctypes.c_int, _G, c_i32, c_vp, c_vp, c_vp, c_vp)
_sig("damas_select", ctypes.c_int, c_i32, c_i32, c_vp, c_i32, c_dbl, c_vp, c_vp, c_vp, c_vp)
_sig("damas_select_pred", ctypes.c_int, c_i32, c_i32, c_vp, c_i32, c_dbl, c_i32, c_vp, c_vp,
     c_vp, c_vp)
_sig("damas_layout", ctypes.c_int, c_i32, c_vp, c_i32, c_i64, c_vp, c_vp)
_sig("damas_steer", ctypes.c_int, _G, c_i32, c_vp, c_vp, c_vp, c_i32, c_vp, c_i64, c_vp)
_sig("damas_psf", ctypes.c_int, c_i32, c_i32, c_vp, c_i32, c_i32, c_vp, c_i64, c_vp, c_vp, c_vp)
_sig("damas_steer_bf16", ctypes.c_int, _G, c_i32, c_vp, c_vp, c_vp, c_i32, c_vp, c_i64, c_vp)
_sig("damas_das_map_ex", ctypes.c_int, _G, c_i32, c_vp, c_vp, c_i32, c_i32, c_vp, c_vp)
_sig("damas_steer_ex", ctypes.c_int, _G, c_i32, c_vp, c_vp, c_vp, c_i32, c_i32, c_vp, c_i64, c_vp)
_sig("damas_psf_ex", ctypes.c_int, c_i32, c_i32, c_vp, c_i32, c_i32, c_i32, c_i32, c_vp, c_i64,
     c_vp, c_vp, c_vp)
_sig("damas_psf_bf16", ctypes.c_int, c_i32, c_i32, c_vp, c_i32, c_vp, c_i64, c_vp, c_vp, c_vp)
_sig("damas_gs", ctypes.c_int, c_i32, c_i32, c_vp, c_i32, c_vp, c_vp, c_i32, c_i32, c_vp,
     c_vp, c_i32, c_vp, c_vp, c_vp)
_sig("damas_ctx_create", ctypes.c_int, c_i32, ctypes.POINTER(c_vp))


class CtxOpts(ctypes.Structure):
    _fields_ = [("device", c_i32), ("hbm_budget", ctypes.c_uint64),
                ("tune_cache", ctypes.c_char_p), ("deterministic", c_i32)]


_sig("damas_ctx_create_ex", ctypes.c_int, ctypes.POINTER(CtxOpts), ctypes.POINTER(c_vp))
_sig("damas_ctx_last_error", ctypes.c_char_p, c_vp)
_sig("damas_ctx_destroy", None, c_vp)
_sig("damas_ctx_set_timing", ctypes.c_int, c_vp, c_i32)
_sig("damas_ctx_classes", ctypes.c_int, c_vp, c_i32, c_vp)
_sig("damas_ctx_set_coop", ctypes.c_int, c_vp, c_i32)
_sig("damas_ctx_last_workgroups", ctypes.c_int, c_vp, ctypes.POINTER(c_i32))
_sig("damas_ctx_gs_time", ctypes.c_int, c_vp, ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64))
_sig("damas_ctx_phase_time", ctypes.c_int, c_vp, c_i32, ctypes.POINTER(c_dbl),
     ctypes.POINTER(c_i64))
PHASE_SWEEPS = 0
PHASE_SYSTEM = 1
_sig("damas_solve_dev", ctypes.c_int, c_vp, _G, c_i32, c_vp, c_vp, ctypes.POINTER(Params),
     c_vp, c_vp, c_vp, c_vp, c_vp, c_vp)
_sig("damas_check", ctypes.c_int, c_vp, c_vp)
_sig("damas_solve_static", ctypes.c_int, _G, c_i32, c_vp, c_vp, ctypes.POINTER(Params), c_vp,
     c_vp, c_vp, c_vp, c_vp, c_vp, c_vp)
_sig("damas_static_scratch_bytes", c_i64)
_sig("damas_query_footprint", ctypes.c_int, c_i32, c_i32, c_i32, ctypes.POINTER(Params),
     ctypes.POINTER(ctypes.c_uint64))


class TuneResult(ctypes.Structure):
    _fields_ = [("coop", c_i32), ("coop_min_rows", c_i32), ("coop_split", c_dbl),
                ("coop_overhead", c_dbl), ("best_ms_per_sweep", c_dbl),
                ("default_ms_per_sweep", c_dbl), ("candidates_timed", c_i32),
                ("coop_floor_rows", c_i32), ("wide_cost", c_dbl)]


_sig("damas_ctx_autotune", ctypes.c_int, c_vp, _G, c_i32, c_vp, c_vp, ctypes.POINTER(Params),
     c_i32, c_vp, ctypes.POINTER(TuneResult))
_sig("damas_ctx_set_schedule", ctypes.c_int, c_vp, ctypes.POINTER(TuneResult))
_sig("damas_graph_capture", ctypes.c_int, c_vp, _G, c_i32, c_vp, c_vp, ctypes.POINTER(Params),
     c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(c_vp))
_sig("damas_graph_launch", ctypes.c_int, c_vp, c_vp)
_sig("damas_graph_workgroups", c_i32, c_vp)
_sig("damas_graph_destroy", None, c_vp)


class ServerOpts(ctypes.Structure):
    _fields_ = [("device", c_i32), ("hbm_budget", ctypes.c_uint64),
                ("cache_budget", ctypes.c_uint64), ("slots", c_i32), ("max_queue", c_i32),
                ("max_batch", c_i32)]


class Request(ctypes.Structure):
    _fields_ = [("M", c_i32), ("mic", c_vp), ("N", c_i32), ("x0", c_dbl), ("x1", c_dbl),
                ("y0", c_dbl), ("y1", c_dbl), ("z0", c_dbl), ("c", c_dbl), ("n_bins", c_i32),
                ("freq", c_vp), ("csm", c_vp), ("params", Params), ("x_map", c_vp),
                ("s_tilde", c_vp)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", c_i32), ("cache_hit", c_i32), ("queue_ms", c_dbl),
                ("run_ms", c_dbl), ("total_ms", c_dbl)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("cache_hits", ctypes.c_uint64),
                ("cache_misses", ctypes.c_uint64), ("held_bytes", ctypes.c_uint64),
                ("cache_bytes", ctypes.c_uint64), ("queued", c_i32), ("running", c_i32),
                ("batches", ctypes.c_uint64), ("merged", ctypes.c_uint64)]


_sig("damas_server_create", ctypes.c_int, ctypes.POINTER(ServerOpts), ctypes.POINTER(c_vp))
_sig("damas_server_destroy", None, c_vp)
_sig("damas_submit", ctypes.c_int, c_vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64))
_sig("damas_wait", ctypes.c_int, c_vp, ctypes.c_uint64, c_i32, ctypes.POINTER(RequestInfo))
_sig("damas_poll", ctypes.c_int, c_vp, ctypes.c_uint64)
_sig("damas_server_get_stats", ctypes.c_int, c_vp, ctypes.POINTER(ServerStats))


class DamasError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_lib.damas_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise DamasError(rc, _lib.damas_last_error().decode())


def strerror(code: int) -> str:
    return _lib.damas_strerror(code).decode()


def last_error() -> str:
    return _lib.damas_last_error().decode()


def ld(s_tilde: int) -> int:
    """Row stride of a compressed system with s_tilde unknowns."""
    return int(_lib.damas_ld(int(s_tilde)))


def coarse_count(N: int) -> int:
    """Points of the coarsest grid G^0, always kept."""
    return int(_lib.damas_coarse_count(int(N)))


def mp(M: int) -> int:
    """Half-width of a bf16 steering row (M rounded up to 16)."""
    return int(_lib.damas_mp(int(M)))


def gs_capacity(precision: int) -> int:
    """Largest max_kept the sweeps accept at this precision (0 if unknown)."""
    return int(_lib.damas_gs_capacity(int(precision)))


def wide_capacity() -> int:
    """Largest kept count of a wide bin (float hi + bf16 lo sweeps)."""
    return int(_lib.damas_wide_capacity())


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return t.data_ptr()


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def geometry(mic: torch.Tensor, N: int, x0: float, x1: float, y0: float,
             y1: float, z0: float, c: float = 343.0) -> Geometry:
    """Build a damas_geometry; ``mic`` is a device tensor (M, 3) float64 that
    the caller keeps alive while the geometry is in use."""
    if mic.dim() != 2 or mic.shape[1] != 3:
        raise ValueError("mic must have shape (M, 3)")
    return Geometry(mic.shape[0], _ptr(mic, torch.float64, "mic"), int(N), float(x0),
                    float(x1), float(y0), float(y1), float(z0), float(c))


# ---- step-level calls ------------------------------------------------------

def csm(snap, out=None, stream=None):
    """Eq. (1): per bin the average of p p^H over its snapshots.
    snap: complex128 (n_bins, n_snap, M) or float64 (n_bins, n_snap, M, 2);
    returns complex128 (n_bins, M, M)."""
    s = _as_interleaved(snap)
    nb, K, M = s.shape[0], s.shape[1], s.shape[2]
    if out is None:
        out = torch.empty(nb, M, M, dtype=torch.complex128, device=s.device)
    o = torch.view_as_real(out)
    _check(_lib.damas_csm(M, K, nb, _ptr(s, torch.float64, "snap"),
                          _ptr(o, torch.float64, "csm"), _stream(stream)))
    return out


def das_map(g: Geometry, freq, csm, b=None, stream=None):
    """b[f, n] = Re(e_n^H C_f e_n) / M^2 (float64, n_bins x N*N).
    csm: complex128 (n_bins, M, M) or float64 (n_bins, M, M, 2)."""
    csm = _as_interleaved(csm)
    nb = freq.numel()
    if b is None:
        b = torch.empty(nb, g.N * g.N, dtype=torch.float64, device=freq.device)
    _check(_lib.damas_das_map(ctypes.byref(g), nb, _ptr(freq, torch.float64, "freq"),
                              _ptr(csm, torch.float64, "csm"),
                              _ptr(b, torch.float64, "b"), _stream(stream)))
    return b


def das_map_ex(g: Geometry, freq, csm, steering=STEER_UNIT, diag_removal=False, b=None,
               stream=None):
    """das_map with a steering form and optional CSM diagonal removal."""
    csm = _as_interleaved(csm)
    nb = freq.numel()
    if b is None:
        b = torch.empty(nb, g.N * g.N, dtype=torch.float64, device=freq.device)
    _check(_lib.damas_das_map_ex(ctypes.byref(g), nb, _ptr(freq, torch.float64, "freq"),
                                 _ptr(csm, torch.float64, "csm"), int(steering),
                                 1 if diag_removal else 0, _ptr(b, torch.float64, "b"),
                                 _stream(stream)))
    return b


def steer_ex(g: Geometry, freq, idx, s_tilde, max_kept: int, steering=STEER_UNIT,
             stream=None):
    """Steering rows (n_bins, rows, 2M) double; the paper's pair has 2 ld rows
    per bin (beamformer rows first, then propagation rows)."""
    nb = freq.numel()
    L = ld(max_kept) * (2 if steering == STEER_PAPER else 1)
    E = torch.zeros(nb, L, 2 * g.M, dtype=torch.float64, device=freq.device)
    _check(_lib.damas_steer_ex(ctypes.byref(g), nb, _ptr(freq, torch.float64, "freq"),
                               _ptr(idx, torch.int32, "idx"),
                               _ptr(s_tilde, torch.int32, "s_tilde"), int(max_kept),
                               int(steering), _ptr(E, torch.float64, "E"), L * 2 * g.M,
                               _stream(stream)))
    return E


def psf_ex(M: int, s_tilde, max_kept: int, precision: int, E, off, steering=STEER_UNIT,
           diag_removal=False, A=None, stream=None):
    """Packed A arena (flat) with a steering form and diagonal removal; the
    paper's pair stores A transposed (row = source point)."""
    nb = s_tilde.numel()
    if A is None:
        total = int(off[-1].item())
        A = torch.full((max(total, 1),), float("nan"), dtype=_DTYPE[precision],
                       device=off.device)
    _check(_lib.damas_psf_ex(int(M), nb, _ptr(s_tilde, torch.int32, "s_tilde"), int(max_kept),
                             int(precision), int(steering), 1 if diag_removal else 0,
                             _ptr(E, torch.float64, "E"), E.shape[1] * E.shape[2],
                             _ptr(off, torch.int64, "off"), _ptr(A, _DTYPE[precision], "A"),
                             _stream(stream)))
    return A


def select(N: int, b, mode: int, eps: float = 0.0, keep_count=None, predictor=0,
           stream=None):
    """Algorithm 1 with predictor PRED_HAAR or PRED_LINEAR: returns
    (idx int32 (n_bins, N*N), s_tilde int32 (n_bins))."""
    nb = b.shape[0]
    idx = torch.zeros(nb, N * N, dtype=torch.int32, device=b.device)
    st = torch.zeros(nb, dtype=torch.int32, device=b.device)
    _check(_lib.damas_select_pred(int(N), nb, _ptr(b, torch.float64, "b"), int(mode),
                                  float(eps), int(predictor),
                                  _ptr(keep_count, torch.int32, "keep_count"),
                                  _ptr(idx, torch.int32, "idx"),
                                  _ptr(st, torch.int32, "s_tilde"), _stream(stream)))
    return idx, st


def layout(s_tilde, max_kept: int, capacity: int = 2 ** 62, stream=None):
    """Offsets (int64, n_bins + 1) of the packed per-bin systems; bins over
    max_kept or past `capacity` elements get s_tilde = 0 (in place)."""
    nb = s_tilde.numel()
    off = torch.zeros(nb + 1, dtype=torch.int64, device=s_tilde.device)
    _check(_lib.damas_layout(nb, _ptr(s_tilde, torch.int32, "s_tilde"), int(max_kept),
                             int(capacity), _ptr(off, torch.int64, "off"), _stream(stream)))
    return off


def steer(g: Geometry, freq, idx, s_tilde, max_kept: int, stream=None):
    """Steering rows of the kept points, double: (n_bins, ld(max_kept), 2M)."""
    nb = freq.numel()
    L = ld(max_kept)
    E = torch.zeros(nb, L, 2 * g.M, dtype=torch.float64, device=freq.device)
    _check(_lib.damas_steer(ctypes.byref(g), nb, _ptr(freq, torch.float64, "freq"),
                            _ptr(idx, torch.int32, "idx"), _ptr(s_tilde, torch.int32, "s_tilde"),
                            int(max_kept), _ptr(E, torch.float64, "E"), L * 2 * g.M,
                            _stream(stream)))
    return E


def psf(M: int, s_tilde, max_kept: int, precision: int, E, off, A=None, stream=None):
    """Packed A arena of all bins (flat tensor, off[-1] elements)."""
    nb = s_tilde.numel()
    if A is None:
        total = int(off[-1].item())
        A = torch.full((max(total, 1),), float("nan"), dtype=_DTYPE[precision],
                       device=off.device)
    _check(_lib.damas_psf(int(M), nb, _ptr(s_tilde, torch.int32, "s_tilde"), int(max_kept),
                          int(precision), _ptr(E, torch.float64, "E"),
                          E.shape[1] * E.shape[2], _ptr(off, torch.int64, "off"),
                          _ptr(A, _DTYPE[precision], "A"), _stream(stream)))
    return A


def steer_bf16(g: Geometry, freq, idx, s_tilde, max_kept: int, stream=None):
    """bf16 steering rows of the kept points: (n_bins, ld(max_kept), 2 mp(M))
    torch.bfloat16, [cos | -sin] each padded to mp(M) mics."""
    nb = freq.numel()
    L = ld(max_kept)
    K = 2 * mp(g.M)
    E = torch.zeros(nb, L, K, dtype=torch.bfloat16, device=freq.device)
    _check(_lib.damas_steer_bf16(ctypes.byref(g), nb, _ptr(freq, torch.float64, "freq"),
                                 _ptr(idx, torch.int32, "idx"),
                                 _ptr(s_tilde, torch.int32, "s_tilde"), int(max_kept),
                                 _ptr(E, torch.bfloat16, "E16"), L * K, _stream(stream)))
    return E


def psf_bf16(M: int, s_tilde, max_kept: int, E16, off, A=None, stream=None):
    """Packed bf16 A arena of all bins (flat torch.bfloat16, off[-1] elements),
    built on the bf16 matrix cores."""
    nb = s_tilde.numel()
    if A is None:
        total = int(off[-1].item())
        A = torch.full((max(total, 1),), float("nan"), dtype=torch.bfloat16, device=off.device)
    _check(_lib.damas_psf_bf16(int(M), nb, _ptr(s_tilde, torch.int32, "s_tilde"), int(max_kept),
                               _ptr(E16, torch.bfloat16, "E16"), E16.shape[1] * E16.shape[2],
                               _ptr(off, torch.int64, "off"), _ptr(A, torch.bfloat16, "A16"),
                               _stream(stream)))
    return A


def gs(N: int, s_tilde, max_kept: int, idx, off, precision: int, A, b, iterations: int,
       x_init=None, x_map=None, unit_diagonal=False, stream=None):
    """Non-negative Gauss-Seidel sweeps; returns x_map (n_bins, N*N).
    unit_diagonal: A_ii = 1 for every row (true of psf()'s output)."""
    nb = s_tilde.numel()
    dt, xt = _DTYPE[precision], _XTYPE[precision]
    if x_map is None:
        x_map = torch.empty(nb, N * N, dtype=xt, device=b.device)
    _check(_lib.damas_gs(int(N), nb, _ptr(s_tilde, torch.int32, "s_tilde"), int(max_kept),
                         _ptr(idx, torch.int32, "idx"), _ptr(off, torch.int64, "off"),
                         int(precision), 1 if unit_diagonal else 0, _ptr(A, dt, "A"),
                         _ptr(b, torch.float64, "b"),
                         int(iterations), _ptr(x_init, xt, "x_init"),
                         _ptr(x_map, xt, "x_map"), _stream(stream)))
    return x_map


def check(ctx=None, stream=None):
    """Synchronise and report device-side capacity failures."""
    _check(_lib.damas_check(ctx._h if ctx is not None else None, _stream(stream)))


# ---- the whole path ----------------------------------------------------------

def static_scratch_bytes() -> int:
    """Bytes of the static device workspace of solve_static."""
    return int(_lib.damas_static_scratch_bytes())


def solve_static(g: Geometry, freq, csm, *, select_mode=SEL_KEEP_ALL, eps=0.0,
                 keep_count=None, iterations=1000, precision=PREC_FP32, max_kept=0,
                 x_init=None, x_map=None, b_map=None, idx=None, s_tilde=None, predictor=0,
                 policy=POLICY_AUTO, rho_wide=0.0, steering=STEER_UNIT, diag_removal=False,
                 keep_frac=0.0, stream=None):
    """The whole-path solve with no allocation by the library (damas_solve_static):
    keep_count is a device int32 tensor of n_bins (KEEP_COUNT; KEEP_FRAC takes
    keep_frac instead).  Faults are
    reported by check(None)."""
    csm = _as_interleaved(csm)
    nb = freq.numel()
    if x_map is None:
        x_map = torch.empty(nb, g.N * g.N, dtype=_XTYPE[precision], device=freq.device)
    p, _kc = _params(nb, select_mode, eps, None, iterations, precision, True, max_kept, 0,
                     predictor, policy, rho_wide, 0.0, steering, diag_removal, keep_frac)
    dt = _XTYPE[precision]
    _check(_lib.damas_solve_static(ctypes.byref(g), nb, _ptr(freq, torch.float64, "freq"),
                                   _ptr(csm, torch.float64, "csm"), ctypes.byref(p),
                                   _ptr(keep_count, torch.int32, "keep_count"),
                                   _ptr(x_init, dt, "x_init"), _ptr(x_map, dt, "x_map"),
                                   _ptr(b_map, torch.float64, "b_map"),
                                   _ptr(idx, torch.int32, "idx"),
                                   _ptr(s_tilde, torch.int32, "s_tilde"), _stream(stream)))
    return x_map

class Context:
    """damas_ctx: the device workspace of whole-path solves."""

    def __init__(self, device: int = 0, *, hbm_budget: int = 0, tune_cache=None,
                 deterministic: bool = False):
        """hbm_budget: bytes the workspace may hold (0: no limit);
        tune_cache: path of the autotune cache file; deterministic: one
        workgroup per bin, results independent of tuning."""
        o = CtxOpts(int(device), int(hbm_budget),
                    None if tune_cache is None else str(tune_cache).encode(),
                    1 if deterministic else 0)
        h = c_vp()
        _check(_lib.damas_ctx_create_ex(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.device = device

    def last_error(self) -> str:
        """The last failure of a call made on this context, from any thread."""
        return _lib.damas_ctx_last_error(self._h).decode()

    def close(self):
        if getattr(self, "_h", None):
            _lib.damas_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_coop(self, max_workgroups: int):
        """Workgroup budget of cooperative sweeps: -1 what fits the device,
        0 never, n at most n."""
        _check(_lib.damas_ctx_set_coop(self._h, int(max_workgroups)))

    def last_workgroups(self) -> int:
        """Workgroups of the last sweep launch (bins when none cooperated)."""
        v = c_i32()
        _check(_lib.damas_ctx_last_workgroups(self._h, ctypes.byref(v)))
        return v.value

    def set_timing(self, enabled: bool):
        _check(_lib.damas_ctx_set_timing(self._h, 1 if enabled else 0))

    def classes(self, n_bins: int) -> np.ndarray:
        """Storage class per bin of the last batched solve (CLASS_*)."""
        out = np.zeros(n_bins, np.uint8)
        _check(_lib.damas_ctx_classes(self._h, int(n_bins), out.ctypes.data))
        return out

    def gs_time(self):
        """(milliseconds, launches) of the timed sweep launches since the
        last call."""
        return self.phase_time(PHASE_SWEEPS)

    def phase_time(self, phase: int):
        """(milliseconds, intervals) of a timed phase (PHASE_SWEEPS or
        PHASE_SYSTEM) since its last read."""
        ms, n = c_dbl(), c_i64()
        _check(_lib.damas_ctx_phase_time(self._h, int(phase), ctypes.byref(ms),
                                         ctypes.byref(n)))
        return ms.value, n.value

    def solve(self, g: Geometry, freq, csm, *, select_mode=SEL_KEEP_ALL, eps=0.0,
              keep_count=None, iterations=1000, precision=PREC_FP32, batched=True,
              max_kept=0, refine_sweeps=0, x_init=None, x_map=None, b_map=None, idx=None,
              s_tilde=None, predictor=0, policy=POLICY_AUTO, rho_wide=0.0, rho_f32=0.0,
              steering=STEER_UNIT, diag_removal=False, power=None, keep_frac=0.0,
              stream=None):
        """Every step for every bin on the device; returns x_map.  power (a
        device float64 tensor of n_bins, optional) receives each bin's
        integrated power.

        keep_count: an int, or a sequence of per-bin ints (host values)."""
        csm = _as_interleaved(csm)
        nb = freq.numel()
        S = g.N * g.N
        if x_map is None:
            x_map = torch.empty(nb, S, dtype=_XTYPE[precision], device=freq.device)
        p, kc_arr = _params(nb, select_mode, eps, keep_count, iterations, precision, batched,
                            max_kept, refine_sweeps, predictor, policy, rho_wide, rho_f32,
                            steering, diag_removal, keep_frac)
        p.power = _ptr(power, torch.float64, "power")
        dt = _XTYPE[precision]
        _check(_lib.damas_solve_dev(self._h, ctypes.byref(g), nb,
                                    _ptr(freq, torch.float64, "freq"),
                                    _ptr(csm, torch.float64, "csm"), ctypes.byref(p),
                                    _ptr(x_init, dt, "x_init"), _ptr(x_map, dt, "x_map"),
                                    _ptr(b_map, torch.float64, "b_map"),
                                    _ptr(idx, torch.int32, "idx"),
                                    _ptr(s_tilde, torch.int32, "s_tilde"), _stream(stream)))
        return x_map

    def check(self, stream=None):
        check(self, stream)

    def set_schedule(self, **knobs):
        """Apply schedule knobs (keys of autotune()'s result: coop,
        coop_min_rows, coop_split, coop_overhead, coop_floor_rows, wide_cost;
        defaults for the others) without trial solves."""
        r = TuneResult()
        base = {"coop": 1, "coop_min_rows": 320, "coop_split": 1.25, "coop_overhead": 1.3,
                "coop_floor_rows": 0, "wide_cost": 1.7}
        base.update(knobs)
        for k, v in base.items():
            setattr(r, k, v)
        _check(_lib.damas_ctx_set_schedule(self._h, ctypes.byref(r)))

    def autotune(self, g: Geometry, freq, csm, *, select_mode=SEL_KEEP_ALL, eps=0.0,
                 keep_count=None, precision=PREC_FP32, max_kept=0, trial_sweeps=30,
                 policy=POLICY_AUTO, rho_wide=0.0, rho_f32=0.0, keep_frac=0.0,
                 stream=None) -> dict:
        """Tune the cooperative sweep schedule on this problem (trial solves
        of trial_sweeps sweeps); the choice stays on the context."""
        csm = _as_interleaved(csm)
        nb = freq.numel()
        p, _kc = _params(nb, select_mode, eps, keep_count, trial_sweeps, precision, True,
                         max_kept, 0, 0, policy, rho_wide, rho_f32, keep_frac=keep_frac)
        r = TuneResult()
        _check(_lib.damas_ctx_autotune(self._h, ctypes.byref(g), nb,
                                       _ptr(freq, torch.float64, "freq"),
                                       _ptr(csm, torch.float64, "csm"), ctypes.byref(p),
                                       int(trial_sweeps), _stream(stream), ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in TuneResult._fields_}

    def capture(self, g: Geometry, freq, csm, *, select_mode=SEL_KEEP_ALL, eps=0.0,
                keep_count=None, iterations=1000, precision=PREC_FP32, max_kept=0,
                refine_sweeps=0, x_init=None, x_map=None, b_map=None, idx=None,
                s_tilde=None, predictor=0, policy=POLICY_AUTO, rho_wide=0.0, rho_f32=0.0,
                steering=STEER_UNIT, diag_removal=False, power=None, keep_frac=0.0):
        """Capture this batched solve into a Graph (csm must be float64
        interleaved (n_bins, M, M, 2) so that in-place updates reach the
        graph)."""
        if csm.dtype != torch.float64:
            raise ValueError("capture needs csm as float64 (n_bins, M, M, 2)")
        nb = freq.numel()
        if x_map is None:
            x_map = torch.empty(nb, g.N * g.N, dtype=_XTYPE[precision], device=freq.device)
        p, kc = _params(nb, select_mode, eps, keep_count, iterations, precision, True,
                        max_kept, refine_sweeps, predictor, policy, rho_wide, rho_f32,
                        steering, diag_removal, keep_frac)
        p.power = _ptr(power, torch.float64, "power")
        dt = _XTYPE[precision]
        h = c_vp()
        _check(_lib.damas_graph_capture(self._h, ctypes.byref(g), nb,
                                        _ptr(freq, torch.float64, "freq"),
                                        _ptr(csm, torch.float64, "csm"), ctypes.byref(p),
                                        _ptr(x_init, dt, "x_init"), _ptr(x_map, dt, "x_map"),
                                        _ptr(b_map, torch.float64, "b_map"),
                                        _ptr(idx, torch.int32, "idx"),
                                        _ptr(s_tilde, torch.int32, "s_tilde"), ctypes.byref(h)))
        return Graph(h, self, x_map)


class Graph:
    """A captured whole-path solve (damas_graph); launch() replays it."""

    def __init__(self, h, ctx, x_map):
        self._h = h
        self._ctx = ctx  # the context must outlive the graph
        self.x_map = x_map

    def launch(self, stream=None):
        _check(_lib.damas_graph_launch(self._h, _stream(stream)))
        return self.x_map

    def workgroups(self) -> int:
        """Workgroups of the captured sweep launches (n_bins: one per bin)."""
        return int(_lib.damas_graph_workgroups(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.damas_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _params(nb, select_mode, eps, keep_count, iterations, precision, batched, max_kept,
            refine_sweeps, predictor=0, policy=POLICY_AUTO, rho_wide=0.0, rho_f32=0.0,
            steering=STEER_UNIT, diag_removal=False, keep_frac=0.0):
    """Params struct and the ctypes array that keeps per-bin counts alive."""
    kc_arr = None
    kc_all = 0
    if keep_count is not None:
        if isinstance(keep_count, (int, np.integer)):
            kc_all = int(keep_count)
        else:
            vals = [int(v) for v in keep_count]
            if len(vals) != nb:
                raise ValueError("keep_count needs one value per bin")
            kc_arr = (c_i32 * nb)(*vals)
    p = Params(int(select_mode), float(eps),
               ctypes.cast(kc_arr, ctypes.POINTER(c_i32)) if kc_arr is not None else None,
               int(kc_all), int(iterations), int(precision), 1 if batched else 0,
               int(max_kept), int(refine_sweeps), int(predictor), int(policy),
               float(rho_wide), float(rho_f32), int(steering), 1 if diag_removal else 0,
               None, float(keep_frac))
    return p, kc_arr


def query_footprint(M: int, N: int, n_bins: int, *, select_mode=SEL_KEEP_ALL, eps=0.0,
                    keep_count=None, iterations=1000, precision=PREC_FP32, max_kept=0,
                    refine_sweeps=0, policy=POLICY_AUTO, keep_frac=0.0) -> int:
    """Device bytes of a whole-path solve of this shape (no device work)."""
    p, _kc = _params(n_bins, select_mode, eps, keep_count, iterations, precision, True,
                     max_kept, refine_sweeps, 0, policy, keep_frac=keep_frac)
    out = ctypes.c_uint64()
    _check(_lib.damas_query_footprint(int(M), int(N), int(n_bins), ctypes.byref(p),
                                      ctypes.byref(out)))
    return int(out.value)


class Server:
    """damas_server: whole-path solves from host arrays, run by worker
    threads on stream slots, admitted by device footprint, with a PSF cache.
    Inputs are numpy arrays (copied at submission); results come back as
    numpy arrays from wait()."""

    def __init__(self, device=0, hbm_budget=64 << 30, cache_budget=8 << 30, slots=2,
                 max_queue=256, max_batch=1):
        """max_batch > 1: compatible queued requests (any grid) run as one
        batch, their sweeps in one launch."""
        o = ServerOpts(int(device), int(hbm_budget), int(cache_budget), int(slots),
                       int(max_queue), int(max_batch))
        h = c_vp()
        _check(_lib.damas_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._out = {}

    def close(self):
        if getattr(self, "_h", None):
            _lib.damas_server_destroy(self._h)
            self._h = None
            self._out.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, mic, N, extent, z0, freqs, csm, *, select_mode=SEL_KEEP_COUNT, eps=0.0,
               keep_count=None, iterations=1000, precision=PREC_FP32, refine_sweeps=0,
               max_kept=0, c=343.0, policy=POLICY_AUTO, keep_frac=0.0) -> int:
        """Queue one solve; returns its ticket.  csm: complex (n_bins, M, M)."""
        mic = np.ascontiguousarray(mic, dtype=np.float64)
        freqs = np.ascontiguousarray(freqs, dtype=np.float64)
        nb = freqs.size
        csm = np.ascontiguousarray(np.asarray(csm, dtype=np.complex128).view(np.float64))
        p, kc = _params(nb, select_mode, eps, keep_count, iterations, precision, True,
                        max_kept, refine_sweeps, 0, policy, keep_frac=keep_frac)
        x = np.zeros((nb, N * N), np.float64 if precision == PREC_FP64 else np.float32)
        st = np.zeros(nb, np.int32)
        x0, x1, y0, y1 = extent
        r = Request(mic.shape[0], mic.ctypes.data, int(N), float(x0), float(x1), float(y0),
                    float(y1), float(z0), float(c), nb, freqs.ctypes.data, csm.ctypes.data, p,
                    x.ctypes.data, st.ctypes.data)
        t = ctypes.c_uint64()
        _check(_lib.damas_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._out[t.value] = (x, st)
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        """(x_map, s_tilde, info dict) of a finished request; raises
        DamasError (code ETIMEDOUT while it is still running)."""
        info = RequestInfo()
        rc = _lib.damas_wait(self._h, ctypes.c_uint64(ticket), int(timeout_ms),
                             ctypes.byref(info))
        if rc == ETIMEDOUT:
            _check(rc)
        x, st = self._out.pop(ticket, (None, None))
        _check(rc)
        return x, st, {"status": info.status, "cache_hit": bool(info.cache_hit),
                       "queue_ms": info.queue_ms, "run_ms": info.run_ms,
                       "total_ms": info.total_ms}

    def poll(self, ticket: int) -> bool:
        rc = _lib.damas_poll(self._h, ctypes.c_uint64(ticket))
        if rc < 0:
            _check(rc)
        return rc == 1

    def stats(self) -> dict:
        s = ServerStats()
        _check(_lib.damas_server_get_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}


def _as_interleaved(csm):
    if csm.dtype == torch.complex128:
        return torch.view_as_real(csm.contiguous()).contiguous()
    return csm
