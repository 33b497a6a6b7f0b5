"""FP64 CPU oracle of DAMAS on a wavelet-compressed grid (Ma & Liu).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  It shares
no code with the GPU library and never calls it; the GPU product path must
never route through it.

The arithmetic lives in ``damas_oracle.c`` (plain C99, double precision,
compiled with ``-ffp-contract=off``); this module only compiles it with gcc
and marshals numpy arrays through ctypes.  Each wrapper names the passage of
the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "damas_oracle.c")
_HDR = os.path.join(_HERE, "damas_oracle.h")
_LIB = os.path.join(_HERE, "libdamas_oracle.so")

STEER_UNIT = 0
STEER_PAPER = 1

SEL_KEEP_ALL = 0
SEL_EPS_REL = 1
SEL_KEEP_COUNT = 2

PRED_HAAR = 0
PRED_LINEAR = 1

CFLAGS = ["-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/libdamas_oracle.so``."""
    stale = (not os.path.exists(_LIB)
             or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                             os.path.getmtime(_HDR)))
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.POINTER
        d, i = ctypes.c_double, ctypes.c_int
        pd, pi = P(d), P(i)
        lib.orc_grid_point.argtypes = [P(_Geom), i, pd]
        lib.orc_steering.argtypes = [P(_Geom), d, i, pi, pd]
        lib.orc_das_map.argtypes = [P(_Geom), d, pd, pd]
        lib.orc_csm.argtypes = [i, i, pd, pd]
        lib.orc_level.argtypes = [i, i, i, pi, pi]
        lib.orc_level.restype = i
        lib.orc_select.argtypes = [i, pd, i, d, i, pi, pd, pd]
        lib.orc_select.restype = i
        lib.orc_select_pred.argtypes = [i, pd, i, d, i, i, pi, pd, pd]
        lib.orc_select_pred.restype = i
        lib.orc_psf.argtypes = [i, i, pd, pd]
        lib.orc_gs.argtypes = [i, pd, pd, i, pd]
        lib.orc_solve_bin.argtypes = [P(_Geom), d, pd, i, d, i, i, pd, pd, pi,
                                      pd, pd]
        lib.orc_solve_bin.restype = i
        lib.orc_steering_form.argtypes = [P(_Geom), d, i, i, pi, pd, pd]
        lib.orc_das_map_ex.argtypes = [P(_Geom), d, pd, i, i, pd]
        lib.orc_psf_ex.argtypes = [i, i, pd, pd, i, pd]
        lib.orc_solve_bin_ex.argtypes = [P(_Geom), d, pd, i, i, i, d, i, i, pd, pd, pi,
                                         pd, pd]
        lib.orc_solve_bin_ex.restype = i
        _lib = lib
    return _lib


class _Geom(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("mic", ctypes.POINTER(ctypes.c_double)),
                ("N", ctypes.c_int), ("x0", ctypes.c_double),
                ("x1", ctypes.c_double), ("y0", ctypes.c_double),
                ("y1", ctypes.c_double), ("z0", ctypes.c_double),
                ("c", ctypes.c_double)]


@dataclass
class Geometry:
    """Microphone positions (M x 3, plane z = 0) and the N x N scan grid on
    the plane z = z0 spanning [x0, x1] x [y0, y1] (section "Beamforming")."""
    mic: np.ndarray
    N: int
    x0: float
    x1: float
    y0: float
    y1: float
    z0: float
    c: float = 343.0

    def _c(self):
        mic = np.ascontiguousarray(self.mic, dtype=np.float64)
        g = _Geom(mic.shape[0], _pd(mic), self.N, self.x0, self.x1, self.y0,
                  self.y1, self.z0, self.c)
        return g, mic  # keep mic alive alongside the struct


def _pd(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pi(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def grid_point(geom: Geometry, n: int) -> np.ndarray:
    """Position of grid point n = iy*N + ix."""
    g, keep = geom._c()
    r = np.zeros(3)
    _load().orc_grid_point(ctypes.byref(g), int(n), _pd(r))
    return r


def steering(geom: Geometry, freq: float, pts) -> np.ndarray:
    """e_nm = exp(-i k |r_n - r_m|), k = 2 pi f / c, for the listed points
    (unit-magnitude reading of the steering component in "Beamforming").
    Returns complex128 of shape (len(pts), M)."""
    g, keep = geom._c()
    pts = np.ascontiguousarray(pts, dtype=np.int32)
    e = np.zeros((len(pts), geom.mic.shape[0], 2))
    _load().orc_steering(ctypes.byref(g), float(freq), len(pts), _pi(pts), _pd(e))
    return e[..., 0] + 1j * e[..., 1]


def csm(snap: np.ndarray) -> np.ndarray:
    """Eq. (1): the cross-spectral matrix averaged over snapshots.

    snap: n_snap x M complex (one row per snapshot); returns M x M complex,
    C[m, q] = mean_k snap[k, m] conj(snap[k, q])."""
    snap = np.asarray(snap)
    K, M = snap.shape
    s = np.ascontiguousarray(np.stack([snap.real, snap.imag], axis=-1), dtype=np.float64)
    out = np.zeros((M, M, 2))
    _load().orc_csm(int(M), int(K), _pd(s), _pd(out))
    return out[..., 0] + 1j * out[..., 1]


def das_map(geom: Geometry, freq: float, csm: np.ndarray) -> np.ndarray:
    """Delay-and-sum map, Eq. (2): b_n = e_n^H C e_n / M^2, all N*N points."""
    g, keep = geom._c()
    c = _interleave(csm)
    b = np.zeros(geom.N * geom.N)
    _load().orc_das_map(ctypes.byref(g), float(freq), _pd(c), _pd(b))
    return b


def level(N: int, ix: int, iy: int):
    """(level, parent_ix, parent_iy) of a grid point in Algorithm 1's
    nested grids."""
    px, py = ctypes.c_int(), ctypes.c_int()
    lv = _load().orc_level(int(N), int(ix), int(iy), ctypes.byref(px),
                           ctypes.byref(py))
    return lv, px.value, py.value


def select(N: int, b: np.ndarray, mode: int, eps: float = 0.0,
           keep_count: int = 0, predictor: int = PRED_HAAR):
    """Algorithm 1 (wavelet compression computational grid), with the
    order-0 (HAAR) or the linear interpolating (LINEAR) predictor.

    Returns (idx int32 ascending, detail |d| per point, margin)."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    assert b.size == N * N
    idx = np.zeros(N * N, dtype=np.int32)
    det = np.zeros(N * N)
    mg = ctypes.c_double()
    st = _load().orc_select_pred(int(N), _pd(b), int(mode), float(eps),
                                 int(keep_count), int(predictor), _pi(idx), _pd(det),
                                 ctypes.byref(mg))
    return idx[:st].copy(), det, mg.value


def psf(e: np.ndarray) -> np.ndarray:
    """A_ij = |e_i^H e_j|^2 / M^2 from steering rows e (St x M complex)."""
    e = np.ascontiguousarray(e, dtype=np.complex128)
    st, M = e.shape
    ei = np.ascontiguousarray(np.stack([e.real, e.imag], axis=-1))
    A = np.zeros((st, st))
    _load().orc_psf(int(M), int(st), _pd(ei), _pd(A))
    return A


def gs(A: np.ndarray, b: np.ndarray, iters: int, x0=None) -> np.ndarray:
    """DAMAS non-negative Gauss-Seidel, ``iters`` sweeps from x0 (or 0)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    st = b.size
    x = np.zeros(st) if x0 is None else np.array(x0, dtype=np.float64)
    _load().orc_gs(int(st), _pd(A), _pd(b), int(iters), _pd(x))
    return x


def solve_bin(geom: Geometry, freq: float, csm: np.ndarray, mode: int,
              eps: float = 0.0, keep_count: int = 0, iters: int = 1000,
              x_init=None):
    """One bin end to end.  Returns dict(b, idx, x, margin)."""
    g, keep = geom._c()
    S = geom.N * geom.N
    c = _interleave(csm)
    b = np.zeros(S)
    idx = np.zeros(S, dtype=np.int32)
    x = np.zeros(S)
    xi = None if x_init is None else np.ascontiguousarray(x_init, dtype=np.float64)
    mg = ctypes.c_double()
    st = _load().orc_solve_bin(ctypes.byref(g), float(freq), _pd(c), int(mode),
                               float(eps), int(keep_count), int(iters),
                               None if xi is None else _pd(xi), _pd(b),
                               _pi(idx), _pd(x), ctypes.byref(mg))
    if st < 0:
        raise MemoryError("oracle allocation failed")
    return {"b": b, "idx": idx[:st].copy(), "x": x, "margin": mg.value}


def _interleave(csm):
    csm = np.asarray(csm)
    if np.iscomplexobj(csm):
        return np.ascontiguousarray(np.stack([csm.real, csm.imag], axis=-1),
                                    dtype=np.float64)
    return np.ascontiguousarray(csm, dtype=np.float64)


# --------------------------------------------------------------------------
# Options beside the default readings: the paper's steering pair and CSM
# diagonal removal.

def steering_form(geom: Geometry, freq: float, pts, form: int = STEER_UNIT):
    """(v, w): beamformer vectors v_m(r) and propagation vectors (the paper's
    g_m(r)) of the listed points, complex128 (len(pts), M) each.  The unit
    form gives v = w = exp(-i k |r - r_m|) ("Beamforming"); the paper's pair
    weights them by |r - r_m| / |r| and |r| / |r - r_m| ("Beamforming",
    "DAMAS")."""
    g, keep = geom._c()
    pts = np.ascontiguousarray(pts, dtype=np.int32)
    M = geom.mic.shape[0]
    v = np.zeros((len(pts), M, 2))
    w = np.zeros((len(pts), M, 2))
    _load().orc_steering_form(ctypes.byref(g), float(freq), int(form), len(pts), _pi(pts),
                              _pd(v), _pd(w))
    return v[..., 0] + 1j * v[..., 1], w[..., 0] + 1j * w[..., 1]


def das_map_ex(geom: Geometry, freq: float, csm: np.ndarray, form: int = STEER_UNIT,
               diag_removal: bool = False) -> np.ndarray:
    """Delay-and-sum map with a steering form and optional CSM diagonal
    removal: b = (v^H C v - diag sum_m |v_m|^2 C_mm) / (M^2 - diag M)."""
    g, keep = geom._c()
    c = _interleave(csm)
    b = np.zeros(geom.N * geom.N)
    _load().orc_das_map_ex(ctypes.byref(g), float(freq), _pd(c), int(form),
                           1 if diag_removal else 0, _pd(b))
    return b


def psf_ex(v: np.ndarray, w: np.ndarray, diag_removal: bool = False) -> np.ndarray:
    """A[i][j] = (|v_i^H w_j|^2 - diag sum_m |v_im|^2 |w_jm|^2) / (M^2 - diag M):
    row i the beamformer point, column j the source point."""
    v = np.ascontiguousarray(v, dtype=np.complex128)
    w = np.ascontiguousarray(w, dtype=np.complex128)
    st, M = v.shape
    vi = np.ascontiguousarray(np.stack([v.real, v.imag], axis=-1))
    wi = np.ascontiguousarray(np.stack([w.real, w.imag], axis=-1))
    A = np.zeros((st, st))
    _load().orc_psf_ex(int(M), int(st), _pd(vi), _pd(wi), 1 if diag_removal else 0, _pd(A))
    return A


def solve_bin_ex(geom: Geometry, freq: float, csm: np.ndarray, mode: int,
                 form: int = STEER_UNIT, diag_removal: bool = False, eps: float = 0.0,
                 keep_count: int = 0, iters: int = 1000, x_init=None):
    """One bin end to end with a steering form and diagonal removal."""
    g, keep = geom._c()
    S = geom.N * geom.N
    c = _interleave(csm)
    b = np.zeros(S)
    idx = np.zeros(S, dtype=np.int32)
    x = np.zeros(S)
    xi = None if x_init is None else np.ascontiguousarray(x_init, dtype=np.float64)
    mg = ctypes.c_double()
    st = _load().orc_solve_bin_ex(ctypes.byref(g), float(freq), _pd(c), int(form),
                                  1 if diag_removal else 0, int(mode), float(eps),
                                  int(keep_count), int(iters),
                                  None if xi is None else _pd(xi), _pd(b), _pi(idx), _pd(x),
                                  ctypes.byref(mg))
    if st < 0:
        raise MemoryError("oracle allocation failed")
    return {"b": b, "idx": idx[:st].copy(), "x": x, "margin": mg.value}
