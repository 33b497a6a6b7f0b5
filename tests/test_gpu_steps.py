"""Parity of each step of the HIP path with the FP64 oracle, through the
C ABI, on seeded synthetic inputs.

Bars: selection bit-exact (same b in, same indices out); DAS map within
1e-12 of max|b| (double on both sides, different summation order); steering
within 1e-12; A within 1e-12 (double storage) / 6e-8 (float storage: one
rounding of a value in [0, 1]), bitwise symmetric, unit diagonal, zero
padding; sweeps within 1e-10 (double A) / 1e-4 relative L2 (float A) of the
oracle's iterate.
"""
import json
import os

import numpy as np
import pytest

from paper_1608_05179_amd import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _t(a, dtype, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype)


def _geoms(orc, dm, w, dev):
    import torch
    mic = _t(w.mic, torch.float64, dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    og = orc.Geometry(w.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    return g, og, mic


WORKLOADS = {
    "plain_fp64": lambda: synth.plain_fp64(),
    "spiral_N41_4bins": lambda: synth.compressed_fp32(n_bins=4),
    "disc128_N23_2bins": lambda: synth.custom(
        synth.disc_array(128, 0.6, (31,)), 23, (-1.0, 1.0, -1.0, 1.0), 1.5,
        [700.0, 11500.0], [5, 200, 333], [1.0, 0.7, 0.5], snapshots=256, snr_db=10.0),
    "M5_N7": lambda: synth.custom(
        synth.disc_array(5, 0.3, (3,)), 7, (-0.4, 0.6, -0.5, 0.5), 0.8,
        [2500.0], [10], [1.0]),
}


@pytest.mark.parametrize("name", sorted(WORKLOADS))
def test_das_map(orc, dm, dev, name):
    import torch
    w = WORKLOADS[name]()
    g, og, mic = _geoms(orc, dm, w, dev)
    freq = _t(w.freqs, torch.float64, dev)
    csm = _t(w.csm, torch.complex128, dev)
    b = dm.das_map(g, freq, csm).cpu().numpy()
    for f in range(w.n_bins):
        ref = orc.das_map(og, w.freqs[f], w.csm[f])
        err = np.abs(b[f] - ref).max() / np.abs(ref).max()
        assert err < 1e-12, (f, err)


def _select_cases():
    rng = np.random.default_rng(2024)
    cases = []
    for N in (1, 2, 3, 5, 9, 16, 17, 21, 33, 41, 64, 101):
        S = N * N
        maps = [rng.random(S) ** 3, np.round(rng.random(S) * 4) / 4,
                np.full(S, 0.5)]
        cases.append((N, np.stack(maps)))
    return cases


@pytest.mark.parametrize("N,maps", _select_cases(), ids=lambda v: str(v) if isinstance(v, int) else "")
def test_select_bit_exact(orc, dm, dev, N, maps):
    import torch
    S = N * N
    b = _t(maps, torch.float64, dev)
    for eps in (0.0, 0.01, 0.1, 0.3, 1.0):
        idx, st = dm.select(N, b, dm.SEL_EPS_REL, eps)
        idx, st = idx.cpu().numpy(), st.cpu().numpy()
        for f in range(maps.shape[0]):
            ref, _, _ = orc.select(N, maps[f], orc.SEL_EPS_REL, eps)
            assert st[f] == len(ref), (eps, f)
            assert np.array_equal(idx[f, :st[f]], ref), (eps, f)
    n0 = dm.coarse_count(N)
    for K in sorted({0, 1, n0, n0 + 1, S // 10, S // 5, S // 3, S - 1, S, S + 5}):
        kc = _t(np.full(maps.shape[0], K), torch.int32, dev)
        idx, st = dm.select(N, b, dm.SEL_KEEP_COUNT, keep_count=kc)
        idx, st = idx.cpu().numpy(), st.cpu().numpy()
        for f in range(maps.shape[0]):
            ref, _, _ = orc.select(N, maps[f], orc.SEL_KEEP_COUNT, keep_count=K)
            assert st[f] == len(ref), (K, f)
            assert np.array_equal(idx[f, :st[f]], ref), (K, f)
    idx, st = dm.select(N, b, dm.SEL_KEEP_ALL)
    assert (st.cpu().numpy() == S).all()
    assert (idx.cpu().numpy() == np.arange(S)).all()


def test_select_per_bin_counts_and_delta_fixture(orc, dm, dev):
    import torch
    with open(os.path.join(GOLDEN, "select_delta_N9.json")) as fh:
        fx = json.load(fh)
    maps = []
    for case in fx["delta_maps"]:
        m = np.zeros(81)
        ix, iy = case["spike"]
        m[iy * 9 + ix] = 1.0
        maps.append(m)
    b = _t(np.stack(maps), torch.float64, dev)
    idx, st = dm.select(9, b, dm.SEL_EPS_REL, 0.5)
    idx, st = idx.cpu().numpy(), st.cpu().numpy()
    for f, case in enumerate(fx["delta_maps"]):
        assert idx[f, :st[f]].tolist() == case["kept"]
    # different K per bin in one launch
    rng = np.random.default_rng(5)
    maps = rng.random((6, 41 * 41))
    Ks = np.array([4, 5, 100, 337, 1000, 1681], dtype=np.int32)
    idx, st = dm.select(41, _t(maps, torch.float64, dev), dm.SEL_KEEP_COUNT,
                        keep_count=_t(Ks, torch.int32, dev))
    idx, st = idx.cpu().numpy(), st.cpu().numpy()
    for f in range(6):
        ref, _, _ = orc.select(41, maps[f], orc.SEL_KEEP_COUNT, keep_count=int(Ks[f]))
        assert np.array_equal(idx[f, :st[f]], ref)


def _kept_sets(orc, w, og, mode, K):
    out = []
    for f in range(w.n_bins):
        b = orc.das_map(og, w.freqs[f], w.csm[f])
        idx, _, _ = orc.select(w.N, b, mode, keep_count=K)
        out.append((b, idx))
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_steer_and_psf(orc, dm, dev, prec):
    import torch
    P = dm.PREC_FP64 if prec == "fp64" else dm.PREC_FP32
    for w, K in ((synth.compressed_fp32(n_bins=3), 337),
                 (WORKLOADS["disc128_N23_2bins"](), 130),
                 (WORKLOADS["M5_N7"](), 1)):
        g, og, mic = _geoms(orc, dm, w, dev)
        kept = _kept_sets(orc, w, og, orc.SEL_KEEP_COUNT, K)
        S = w.S
        idx = np.zeros((w.n_bins, S), np.int32)
        st = np.zeros(w.n_bins, np.int32)
        for f, (_, ix) in enumerate(kept):
            idx[f, :len(ix)] = ix
            st[f] = len(ix)
        mk = int(st.max())
        freq = _t(w.freqs, torch.float64, dev)
        idx_d = _t(idx, torch.int32, dev)
        st_d = _t(st, torch.int32, dev)
        E = dm.steer(g, freq, idx_d, st_d, mk)
        off = dm.layout(st_d, mk)
        A = dm.psf(w.M, st_d, mk, P, E, off).double().cpu().numpy()
        E = E.double().cpu().numpy()
        offh = off.cpu().numpy()
        M = w.M
        for f in range(w.n_bins):
            ix = kept[f][1]
            n = len(ix)
            L = dm.ld(n)
            e_ref = orc.steering(og, w.freqs[f], ix)
            e_gpu = E[f, :n, :M] + 1j * E[f, :n, M:]
            assert np.abs(e_gpu - e_ref).max() < 1e-12
            assert (E[f, n:L] == 0).all()
            assert offh[f + 1] - offh[f] == L * L
            Af = A[offh[f]:offh[f + 1]].reshape(L, L)
            A_ref = orc.psf(e_ref)
            # float storage: one rounding of a value in [0, 1]
            tol_a = 1e-12 if P == dm.PREC_FP64 else 6e-8
            assert np.abs(Af[:n, :n] - A_ref).max() < tol_a, f
            assert np.array_equal(Af, Af.T)
            assert (np.diag(Af)[:n] == 1.0).all()
            assert (Af[n:, :] == 0).all() and (Af[:, n:] == 0).all()


def _pack_system(dm, A, bt, N=None):
    """One-bin layout of an explicit system: idx = 0..n-1 on an N x N grid."""
    n = len(bt)
    if N is None:
        N = max(1, int(np.ceil(np.sqrt(n))))
    L = dm.ld(n)
    Ap = np.zeros((L, L))
    Ap[:n, :n] = A
    b = np.zeros(N * N)
    b[:n] = bt
    idx = np.zeros(N * N, np.int32)
    idx[:n] = np.arange(n)
    return N, Ap.ravel(), b[None], idx[None], np.array([n], np.int32), np.array([0, L * L])


def _gpu_gs(dm, dev, A, bt, iters, prec, x0=None, unit=False):
    import torch
    N, Ap, b, idx, st, off = _pack_system(dm, A, bt)
    dt = torch.float64 if prec == dm.PREC_FP64 else torch.float32
    xi = None
    if x0 is not None:
        xm = np.zeros(N * N)
        xm[:len(bt)] = x0
        xi = _t(xm[None], dt, dev)
    x = dm.gs(N, _t(st, torch.int32, dev), int(st[0]), _t(idx, torch.int32, dev),
              _t(off, torch.int64, dev), prec, _t(Ap, dt, dev), _t(b, torch.float64, dev),
              iters, x_init=xi, unit_diagonal=unit)
    x = x.double().cpu().numpy()[0]
    assert (x[len(bt):] == 0).all()
    return x[:len(bt)]


def test_gs_hand_cases(dm, dev):
    with open(os.path.join(GOLDEN, "gs_2x2.json")) as fh:
        fx = json.load(fh)
    for case in fx["cases"]:
        x = _gpu_gs(dm, dev, np.array(case["A"], float), np.array(case["b"], float),
                    case["sweeps"], dm.PREC_FP64)
        assert x.tolist() == case["x"], case


# Sizes span one and several 64-row tiles, S~ a multiple of 8 with a partial
# last tile (72, 136), and strips longer than the part of a strip the stream
# waves hold in their head (448 rows for double A, 360 for float A), whose
# tails end on one batch or two depending on the wave (385 .. 1100).
@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 72, 130, 136, 257, 337, 385, 441, 1000, 1100])
def test_gs_matches_oracle(orc, dm, dev, n):
    rng = np.random.default_rng(n)
    M = 24
    e = np.exp(1j * rng.uniform(0, 2 * np.pi, size=(n, M)))
    A = orc.psf(e)
    bt = np.abs(rng.standard_normal(n)) * 0.5
    for it in (0, 1, 3, 40):
        ref = orc.gs(A, bt, it)
        scale = max(np.linalg.norm(ref), 1e-300)
        for unit in (False, True):  # A_ii = 1 here, so both variants apply
            x64 = _gpu_gs(dm, dev, A, bt, it, dm.PREC_FP64, unit=unit)
            assert np.linalg.norm(x64 - ref) / scale < 1e-10, (n, it, unit)
            x32 = _gpu_gs(dm, dev, A, bt, it, dm.PREC_FP32, unit=unit)
            if it:
                assert np.linalg.norm(x32 - ref) / scale < 1e-4, (n, it, unit)
    # warm start equals a longer run
    x1 = orc.gs(A, bt, 5)
    x2 = _gpu_gs(dm, dev, A, bt, 7, dm.PREC_FP64, x0=x1)
    assert np.linalg.norm(x2 - orc.gs(A, bt, 12)) <= 1e-10 * np.linalg.norm(x2)


@pytest.mark.parametrize("n", [3, 64, 65, 72, 200, 264, 392])
def test_gs_general_diagonal(orc, dm, dev, n):
    # Symmetric positive definite A with a non-unit diagonal: the sweeps
    # divide by A_ii (scaling variant).
    rng = np.random.default_rng(300 + n)
    Bm = rng.standard_normal((n, n)) / np.sqrt(n)
    A = Bm @ Bm.T + np.diag(rng.uniform(0.5, 3.0, n))
    bt = rng.standard_normal(n)
    for it in (1, 2, 25):
        ref = orc.gs(A, bt, it)
        x = _gpu_gs(dm, dev, A, bt, it, dm.PREC_FP64)
        assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref), (n, it)
        x32 = _gpu_gs(dm, dev, A, bt, it, dm.PREC_FP32)
        assert np.linalg.norm(x32 - ref) <= 1e-5 * np.linalg.norm(ref), (n, it)


def _bf16_round(a32):
    """bf16 bit patterns of float32 values (round to nearest even; finite)."""
    u = a32.view(np.uint32)
    return ((u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) >> np.uint32(16)).astype(np.uint16)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_gs_at_capacity(orc, dm, dev, prec):
    """A bin of exactly damas_gs_capacity unknowns (x~ filling the LDS left
    beside the sums and blocks): the sweeps match the oracle run on the very
    values of A the GPU reads.  A: symmetric, unit diagonal, small
    non-negative off-diagonal entries (PSF-like); two sweeps."""
    import torch
    p = {"fp64": dm.PREC_FP64, "fp32": dm.PREC_FP32, "bf16": dm.PREC_BF16}[prec]
    n = dm.gs_capacity(p)
    assert n > 0 and dm.ld(n) == n
    N = int(np.ceil(np.sqrt(n)))
    rng = np.random.default_rng(n + p)
    R = np.abs(rng.standard_normal((n, n), dtype=np.float32)) * np.float32(0.5 / np.sqrt(n))
    A32 = R + R.T
    del R
    np.fill_diagonal(A32, 1.0)
    if p == dm.PREC_FP64:
        A_host = A32.astype(np.float64)
        A_d = torch.from_numpy(A_host.ravel()).to(dev)
    elif p == dm.PREC_FP32:
        A_host = A32
        A_d = torch.from_numpy(A32.ravel()).to(dev)
    else:
        bits = _bf16_round(A32)
        A_host = (bits.astype(np.uint32) << np.uint32(16)).view(np.float32)
        A_d = torch.from_numpy(bits.ravel().view(np.int16)).to(dev).view(torch.bfloat16)
    del A32
    bt = np.abs(rng.standard_normal(n)) * 0.5
    b = np.zeros((1, N * N))
    b[0, :n] = bt
    idx = np.zeros((1, N * N), np.int32)
    idx[0, :n] = np.arange(n)
    st = _t(np.array([n], np.int32), torch.int32, dev)
    off = _t(np.array([0, n * n]), torch.int64, dev)
    A64 = np.asarray(A_host, dtype=np.float64)
    for it in (1, 2):
        x = dm.gs(N, st, n, _t(idx, torch.int32, dev), off, p, A_d, _t(b, torch.float64, dev),
                  it, unit_diagonal=True)
        x = x.double().cpu().numpy()[0]
        assert (x[n:] == 0).all()
        ref = orc.gs(A64, bt, it)
        err = np.linalg.norm(x[:n] - ref) / np.linalg.norm(ref)
        # double A: summation order only; float and bf16 A: FP32 partial sums
        # (each of a few hundred terms) and float x maps
        assert err <= (1e-10 if p == dm.PREC_FP64 else 1e-5), (prec, it, err)


@pytest.mark.parametrize("n", [64, 200, 337])
def test_gs_sparse_tiles(orc, dm, dev, n):
    """Tiles with few moving rows visit only those (the rest stay at zero
    with a positive residual): b~ negative on about 85 % of the rows keeps
    those rows at 0 from the first sweep, so almost every tile takes that
    path; the iterate must still be the row-by-row one."""
    rng = np.random.default_rng(900 + n)
    e = np.exp(1j * rng.uniform(0, 2 * np.pi, size=(n, 24)))
    A = orc.psf(e)
    bt = np.abs(rng.standard_normal(n)) * 0.5
    bt[rng.uniform(size=n) < 0.85] *= -1.0
    for it in (1, 4, 30):
        ref = orc.gs(A, bt, it)
        scale = max(np.linalg.norm(ref), 1e-300)
        x64 = _gpu_gs(dm, dev, A, bt, it, dm.PREC_FP64, unit=True)
        assert np.linalg.norm(x64 - ref) / scale < 1e-10, (n, it)
        x32 = _gpu_gs(dm, dev, A, bt, it, dm.PREC_FP32, unit=True)
        assert np.linalg.norm(x32 - ref) / scale < 1e-4, (n, it)
    # a general diagonal scales each row by 1 / A_ii on the same path
    D = np.diag(rng.uniform(0.5, 2.0, n))
    A2 = np.sqrt(D) @ A @ np.sqrt(D)
    ref = orc.gs(A2, bt, 12)
    x = _gpu_gs(dm, dev, A2, bt, 12, dm.PREC_FP64)
    assert np.linalg.norm(x - ref) <= 1e-10 * max(np.linalg.norm(ref), 1e-300), n


def test_gs_identity_one_sweep(dm, dev):
    bt = np.random.default_rng(0).standard_normal(200)
    x = _gpu_gs(dm, dev, np.eye(200), bt, 1, dm.PREC_FP64)
    assert np.array_equal(x, np.maximum(bt, 0.0))


def test_gs_deterministic(orc, dm, dev):
    rng = np.random.default_rng(77)
    n = 500
    A = orc.psf(np.exp(1j * rng.uniform(0, 2 * np.pi, size=(n, 32))))
    bt = np.abs(rng.standard_normal(n))
    a = _gpu_gs(dm, dev, A, bt, 50, dm.PREC_FP32)
    b = _gpu_gs(dm, dev, A, bt, 50, dm.PREC_FP32)
    assert np.array_equal(a, b)
