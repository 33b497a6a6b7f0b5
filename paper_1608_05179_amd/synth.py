"""Seeded synthetic workloads: microphone arrays, scan grids and measured
cross-spectral matrices.

This module simulates the acoustic world the method images.  It holds none
of the method's steps (no beamforming, no grid compression, no point-spread
matrix, no deconvolution) and serves the GPU path and the oracle alike.

Physics of the simulated world (the paper's source model, section "DAMAS"):
uncorrelated monopoles at scan-grid points radiate into free field; the
pressure at microphone m due to a unit source at r_s is the unit-magnitude
transfer exp(-i k |r_s - r_m|), k = 2 pi f / c (the amplitude-normalised
reading under which the beamformer and the source model share one vector).
Snapshot model: p_i = sum_k sqrt(q_k) s_ki g_k + n_i with s_ki ~ CN(0, 1)
and n_i ~ CN(0, sigma^2 I), sigma^2 = sum_k q_k / 10^(SNR/10) (per-mic SNR);
the CSM is the snapshot average of p_i p_i^H, Eq. (1).

Random streams: numpy PCG64 seeded by SeedSequence([config id, purpose, bin]),
so every bin and every config is reproducible on its own.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SPEED_OF_SOUND = 343.0

# Purpose codes of the random streams.
_ARRAY, _SOURCES, _SNAPSHOTS, _KEEP = 0, 1, 2, 3

SEL_KEEP_ALL = 0
SEL_EPS_REL = 1
SEL_KEEP_COUNT = 2


def _rng(*key):
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


# --------------------------------------------------------------------------
# Arrays


def disc_array(M: int, radius: float, seed_key) -> np.ndarray:
    """M microphones uniformly distributed in a disc (plane z = 0)."""
    rng = _rng(*seed_key, _ARRAY)
    rho = radius * np.sqrt(rng.random(M))
    th = 2.0 * np.pi * rng.random(M)
    return np.stack([rho * np.cos(th), rho * np.sin(th), np.zeros(M)], axis=1)


def spiral_array(M: int = 64, radius: float = 0.6, arms: int = 5,
                 rho0: float = 0.05, spiral_deg: float = 70.0) -> np.ndarray:
    """Multi-arm logarithmic spiral: mic m on arm m % arms, step m // arms,
    radius rho0 * (R / rho0)^(t / (n_arm - 1)), angle
    2 pi a / arms + ln(rho / rho0) / tan(spiral angle)."""
    pos = np.zeros((M, 3))
    per_arm = [len(range(a, M, arms)) for a in range(arms)]
    cot = 1.0 / math.tan(math.radians(spiral_deg))
    for m in range(M):
        a, t = m % arms, m // arms
        n_a = per_arm[a]
        rho = rho0 * (radius / rho0) ** (t / max(n_a - 1, 1))
        th = 2.0 * math.pi * a / arms + math.log(rho / rho0) * cot
        pos[m] = (rho * math.cos(th), rho * math.sin(th), 0.0)
    return pos


# --------------------------------------------------------------------------
# Simulated acoustic field


def grid_xyz(N: int, x0: float, x1: float, y0: float, y1: float, z0: float,
             pts) -> np.ndarray:
    """World coordinates of scan-grid points n = iy*N + ix (end points
    included)."""
    pts = np.asarray(pts)
    xs = np.linspace(x0, x1, N)
    ys = np.linspace(y0, y1, N)
    return np.stack([xs[pts % N], ys[pts // N], np.full(pts.shape, z0)], axis=-1)


def monopole_field(mic: np.ndarray, src_xyz: np.ndarray, freq: float,
                   c: float = SPEED_OF_SOUND, model: str = "unit") -> np.ndarray:
    """Free-field pressure at each mic from monopoles: M x K complex.
    model "unit": unit magnitude exp(-i k d) at every mic; model "spherical":
    the 1/d spreading of a monopole normalised to the pressure at the array
    centre, (|r_s| / d) exp(-i k d), d = |r_s - r_m|."""
    dist = np.linalg.norm(mic[:, None, :] - src_xyz[None, :, :], axis=-1)
    p = np.exp(-1j * (2.0 * np.pi * freq / c) * dist)
    if model == "spherical":
        p = p * (np.linalg.norm(src_xyz, axis=-1)[None, :] / dist)
    elif model != "unit":
        raise ValueError(f"unknown source model {model!r}")
    return p


def exact_csm(mic, src_xyz, powers, freq, c=SPEED_OF_SOUND, model="unit") -> np.ndarray:
    """C = sum_k q_k g_k g_k^H: the expectation of Eq. (1) for uncorrelated
    sources without noise."""
    g = monopole_field(mic, src_xyz, freq, c, model)
    C = (g * powers[None, :]) @ g.conj().T
    return 0.5 * (C + C.conj().T)


def snapshot_csm(mic, src_xyz, powers, freq, n_snap, snr_db, seed_key,
                 c=SPEED_OF_SOUND, model="unit") -> np.ndarray:
    """Eq. (1): average of p_i p_i^H over n_snap complex-Gaussian snapshots
    with white noise at the given per-microphone SNR."""
    rng = _rng(*seed_key, _SNAPSHOTS)
    g = monopole_field(mic, src_xyz, freq, c, model)
    K = len(powers)
    M = mic.shape[0]
    s = (rng.standard_normal((K, n_snap)) + 1j * rng.standard_normal((K, n_snap)))
    s *= np.sqrt(0.5 * np.asarray(powers))[:, None]
    sigma2 = float(np.sum(powers)) / 10.0 ** (snr_db / 10.0)
    noise = (rng.standard_normal((M, n_snap)) + 1j * rng.standard_normal((M, n_snap)))
    noise *= math.sqrt(0.5 * sigma2)
    P = g @ s + noise
    C = (P @ P.conj().T) / n_snap
    return 0.5 * (C + C.conj().T)


# --------------------------------------------------------------------------
# Workloads


@dataclass
class Workload:
    """One batch of synthetic input: geometry, grid, bins, CSMs and the
    compression / deconvolution parameters."""
    name: str
    mic: np.ndarray          # M x 3
    N: int
    x0: float
    x1: float
    y0: float
    y1: float
    z0: float
    freqs: np.ndarray        # n_bins, Hz
    csm: np.ndarray          # n_bins x M x M complex128
    select_mode: int
    eps: float = 0.0
    keep_count: int = 0
    keep_counts: np.ndarray | None = None  # per-bin K (int32) or None
    iterations: int = 1000
    precision: str = "fp32"  # fp64 | fp32 | bf16
    refine_sweeps: int = 0
    c: float = SPEED_OF_SOUND
    sources: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))
    powers: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def M(self):
        return self.mic.shape[0]

    @property
    def S(self):
        return self.N * self.N

    @property
    def n_bins(self):
        return len(self.freqs)

    def keep_count_of(self, f):
        if self.keep_counts is not None:
            return int(self.keep_counts[f])
        return int(self.keep_count)

    def max_kept(self):
        if self.select_mode == SEL_KEEP_COUNT:
            k = (int(np.max(self.keep_counts)) if self.keep_counts is not None
                 else int(self.keep_count))
            return max(1, min(k, self.S))
        return self.S


def _sources(cfg, S, K, rng_key):
    rng = _rng(cfg, *rng_key, _SOURCES)
    pts = np.sort(rng.choice(S, size=K, replace=False))
    return pts, rng


def plain_fp64(n_bins: int = 1) -> Workload:
    """Plain DAMAS, FP64: 16 mics uniform in a 0.5 m disc, 21 x 21 grid on a
    1 x 1 m plane at 1 m, one bin at 4 kHz, 3 sources of power U(0.5, 1),
    exact CSM, no compression, 500 sweeps."""
    cfg = 1
    mic = disc_array(16, 0.5, (cfg,))
    N, z0 = 21, 1.0
    pts, rng = _sources(cfg, N * N, 3, ())
    q = rng.uniform(0.5, 1.0, size=3)
    freqs = np.array([4000.0] if n_bins == 1 else np.linspace(3000.0, 5000.0, n_bins))
    xyz = grid_xyz(N, -0.5, 0.5, -0.5, 0.5, z0, pts)
    csm = np.stack([exact_csm(mic, xyz, q, f) for f in freqs])
    return Workload("plain-fp64 M16 N21 1bin", mic, N, -0.5, 0.5, -0.5, 0.5, z0,
                    freqs, csm, SEL_KEEP_ALL, iterations=500, precision="fp64",
                    sources=pts, powers=q)


def compressed_fp32(keep_frac: float = 0.2, n_bins: int = 64,
                    N: int = 41, iterations: int = 1000) -> Workload:
    """Wavelet-compressed DAMAS, FP32: 64-mic 5-arm log spiral of radius
    0.6 m, 41 x 41 grid on a 2 x 2 m plane at 1.5 m, 64 bins over 1-8 kHz,
    5 sources of power U(0.5, 1), 1024 snapshots at 20 dB SNR; the grid keeps
    the top ``keep_frac`` of points by wavelet detail; 1000 sweeps."""
    cfg = 2
    mic = spiral_array(64, 0.6)
    z0 = 1.5
    S = N * N
    pts, rng = _sources(cfg, S, 5, ())
    q = rng.uniform(0.5, 1.0, size=5)
    all_freqs = np.linspace(1000.0, 8000.0, 64)
    freqs = all_freqs[:n_bins] if n_bins <= 64 else np.linspace(1000.0, 8000.0, n_bins)
    xyz = grid_xyz(N, -1.0, 1.0, -1.0, 1.0, z0, pts)
    csm = np.stack([snapshot_csm(mic, xyz, q, f, 1024, 20.0, (cfg, b))
                    for b, f in enumerate(freqs)])
    K = int(math.ceil(keep_frac * S - 1e-9))
    return Workload(f"compressed-fp32 M64 N{N} {len(freqs)}bins keep{keep_frac:g}",
                    mic, N, -1.0, 1.0, -1.0, 1.0, z0, freqs, csm, SEL_KEEP_COUNT,
                    keep_count=K, iterations=iterations, precision="fp32",
                    sources=pts, powers=q)


def precision_bf16(n_bins: int = 32, N: int = 81, iterations: int = 1000,
                   refine_sweeps: int = 10) -> Workload:
    """Precision variant: 64-mic spiral, 81 x 81 grid, 32 bins over 2-10 kHz,
    8 sources over a 10-15 dB dynamic range, 1024 snapshots at 20 dB SNR,
    no compression, BF16 bulk sweeps with FP32 refinement sweeps."""
    cfg = 3
    mic = spiral_array(64, 0.6)
    z0 = 1.5
    S = N * N
    pts, rng = _sources(cfg, S, 8, ())
    D = rng.uniform(10.0, 15.0)
    q = np.empty(8)
    q[0], q[1] = 1.0, 10.0 ** (-D / 10.0)
    q[2:] = 10.0 ** (-rng.uniform(0.0, D, size=6) / 10.0)
    freqs = np.linspace(2000.0, 10000.0, 32)[:n_bins]
    xyz = grid_xyz(N, -1.0, 1.0, -1.0, 1.0, z0, pts)
    csm = np.stack([snapshot_csm(mic, xyz, q, f, 1024, 20.0, (cfg, b))
                    for b, f in enumerate(freqs)])
    return Workload(f"precision-bf16 M64 N{N} {len(freqs)}bins", mic, N,
                    -1.0, 1.0, -1.0, 1.0, z0, freqs, csm, SEL_KEEP_ALL,
                    iterations=iterations, precision="bf16",
                    refine_sweeps=refine_sweeps, sources=pts, powers=q)


def batched_fp32(n_bins: int = 256, N: int = 101, iterations: int = 2000,
                 kmin: int = 300, kmax: int = 4000) -> Workload:
    """Batched variant: 128 mics uniform in a 0.6 m disc, 101 x 101 grid on a
    2 x 2 m plane at 1.5 m, 256 bins over 0.5-12 kHz, 10 sources, 2048
    snapshots at 10 dB SNR, 2000 sweeps; per-bin compressed sizes drawn
    uniformly from [kmin, kmax] points."""
    cfg = 4
    mic = disc_array(128, 0.6, (cfg,))
    z0 = 1.5
    S = N * N
    pts, rng = _sources(cfg, S, 10, ())
    q = rng.uniform(0.5, 1.0, size=10)
    freqs = np.linspace(500.0, 12000.0, 256)[:n_bins]
    xyz = grid_xyz(N, -1.0, 1.0, -1.0, 1.0, z0, pts)
    csm = np.stack([snapshot_csm(mic, xyz, q, f, 2048, 10.0, (cfg, b))
                    for b, f in enumerate(freqs)])
    krng = _rng(cfg, _KEEP)
    kc = krng.integers(kmin, kmax + 1, size=len(freqs)).astype(np.int32)
    kc = np.minimum(kc, S).astype(np.int32)
    return Workload(f"batched-fp32 M128 N{N} {len(freqs)}bins", mic, N,
                    -1.0, 1.0, -1.0, 1.0, z0, freqs, csm, SEL_KEEP_COUNT,
                    keep_counts=kc, iterations=iterations, precision="fp32",
                    sources=pts, powers=q)


def served_request(seed: int, table_bins: int = 64) -> Workload:
    """One request of the served workload: the 64-mic spiral, a grid of
    N in {41, 61, 81, 101} on the 2 x 2 m plane at 1.5 m, 1-64 bins drawn
    without replacement from the compressed workload's 64-bin table over
    1-8 kHz, 3-10 sources of power U(0.5, 1), 1024 snapshots at an SNR of
    U(10, 30) dB, and a keep count K ~ U{200 .. min(6000, N^2)}; 1000
    sweeps, FP32."""
    cfg = 5
    rng = _rng(cfg, seed, _SOURCES)
    mic = spiral_array(64, 0.6)
    N = int(rng.choice([41, 61, 81, 101]))
    S = N * N
    nb = int(rng.integers(1, table_bins + 1))
    table = np.linspace(1000.0, 8000.0, table_bins)
    freqs = np.sort(rng.choice(table, size=nb, replace=False))
    n_src = int(rng.integers(3, 11))
    pts = np.sort(rng.choice(S, size=n_src, replace=False))
    q = rng.uniform(0.5, 1.0, size=n_src)
    snr = float(rng.uniform(10.0, 30.0))
    K = int(rng.integers(200, min(6000, S) + 1))
    xyz = grid_xyz(N, -1.0, 1.0, -1.0, 1.0, 1.5, pts)
    csm = np.stack([snapshot_csm(mic, xyz, q, f, 1024, snr, (cfg, seed, b))
                    for b, f in enumerate(freqs)])
    return Workload(f"served M64 N{N} {nb}bins K{K}", mic, N, -1.0, 1.0, -1.0, 1.0, 1.5,
                    freqs, csm, SEL_KEEP_COUNT, keep_count=K, iterations=1000,
                    precision="fp32", sources=pts, powers=q)


def custom(mic, N, extent, z0, freqs, src_pts, powers, *, snapshots=None,
           snr_db=None, seed=99, select_mode=SEL_KEEP_ALL, eps=0.0,
           keep_count=0, iterations=100, precision="fp32", model="unit") -> Workload:
    """A small workload for tests: exact CSM when ``snapshots`` is None."""
    x0, x1, y0, y1 = extent
    src_pts = np.asarray(src_pts)
    powers = np.asarray(powers, dtype=np.float64)
    xyz = grid_xyz(N, x0, x1, y0, y1, z0, src_pts)
    freqs = np.asarray(freqs, dtype=np.float64)
    if snapshots is None:
        csm = np.stack([exact_csm(mic, xyz, powers, f, model=model) for f in freqs])
    else:
        csm = np.stack([snapshot_csm(mic, xyz, powers, f, snapshots, snr_db,
                                     (seed, b), model=model) for b, f in enumerate(freqs)])
    return Workload("custom", np.asarray(mic, dtype=np.float64), N, x0, x1, y0,
                    y1, z0, freqs, csm, select_mode, eps=eps,
                    keep_count=keep_count, iterations=iterations,
                    precision=precision, sources=src_pts, powers=powers)
