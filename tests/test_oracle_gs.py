"""Pins of the oracle's DAMAS Gauss-Seidel sweeps and its end-to-end path.

Hand-computed sweeps, the identity-matrix special case, the descent and
complementarity properties of projected Gauss-Seidel on a symmetric PSD
system, a brute-force solution of the linear complementarity problem, scipy's
NNLS on consistent data, exact recovery of on-grid sources and bitwise
resume.
"""
import itertools
import json
import os

import numpy as np
import pytest
from scipy.optimize import nnls

from paper_1608_05179_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _geom(orc, w):
    return orc.Geometry(w.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)


def test_hand_computed_sweeps(orc):
    with open(os.path.join(GOLDEN, "gs_2x2.json")) as f:
        fx = json.load(f)
    for case in fx["cases"]:
        x = orc.gs(np.array(case["A"], float), np.array(case["b"], float),
                   case["sweeps"])
        assert x.tolist() == case["x"]


def test_identity_matrix_one_sweep(orc):
    b = np.random.default_rng(0).standard_normal(50)
    x = orc.gs(np.eye(50), b, 1)
    assert np.array_equal(x, np.maximum(b, 0.0))


def _pd_system(rng, n, M=None):
    if M is None:
        M = 3 * n
    e = np.exp(1j * rng.uniform(0, 2 * np.pi, size=(n, M)))
    return e


def test_objective_never_increases(orc):
    # For symmetric PSD A each row step minimises f(x) = x'Ax/2 - b'x along
    # coordinate i subject to x_i >= 0, so f is non-increasing per sweep.
    w = synth.compressed_fp32(n_bins=4)
    g = _geom(orc, w)
    f = 3
    b = orc.das_map(g, w.freqs[f], w.csm[f])
    idx, _, _ = orc.select(w.N, b, orc.SEL_KEEP_COUNT, keep_count=200)
    A = orc.psf(orc.steering(g, w.freqs[f], idx))
    bt = b[idx]
    x = np.zeros(len(idx))
    fprev = 0.0
    for it in range(30):
        x = orc.gs(A, bt, 1, x)
        fx = 0.5 * x @ A @ x - bt @ x
        assert fx <= fprev + 1e-12 * abs(fprev)
        fprev = fx
    assert x.min() >= 0.0


def test_kkt_at_convergence(orc):
    # Converged projected GS solves LCP(A, -b): x >= 0, w = Ax - b >= 0 where
    # x = 0 and w = 0 where x > 0.
    rng = np.random.default_rng(5)
    e = _pd_system(rng, 30, 60)
    A = orc.psf(e)
    b = rng.standard_normal(30) * 0.3 + 0.2
    x = orc.gs(A, b, 3000)
    w = A @ x - b
    assert x.min() >= 0.0
    act = x > 1e-12
    assert np.abs(w[act]).max() < 1e-9
    assert w[~act].min() > -1e-9


def _lcp_bruteforce(A, b):
    """All supports P: x_P = A_PP^-1 b_P, keep the KKT-feasible one."""
    n = len(b)
    best = None
    for k in range(n + 1):
        for P in itertools.combinations(range(n), k):
            x = np.zeros(n)
            if k:
                P = list(P)
                x[P] = np.linalg.solve(A[np.ix_(P, P)], b[P])
                if x[P].min() < -1e-12:
                    continue
            w = A @ x - b
            mask = np.ones(n, bool)
            mask[list(P)] = False
            if mask.any() and w[mask].min() < -1e-10:
                continue
            best = x
    return best


@pytest.mark.parametrize("n", [1, 2, 4, 7, 9])
def test_matches_bruteforce_lcp(orc, n):
    rng = np.random.default_rng(100 + n)
    for trial in range(3):
        A = orc.psf(_pd_system(rng, n, 2 * n + 2))
        b = rng.standard_normal(n)
        x_bf = _lcp_bruteforce(A, b)
        x = orc.gs(A, b, 5000)
        assert np.abs(x - x_bf).max() < 1e-9


def test_matches_nnls_on_consistent_data(orc):
    # With b = A x*, x* >= 0 and A positive definite the LCP solution is x*,
    # which is also the NNLS solution.
    rng = np.random.default_rng(9)
    A = orc.psf(_pd_system(rng, 12, 40))
    xs = np.maximum(rng.standard_normal(12), 0)
    b = A @ xs
    x = orc.gs(A, b, 20000)
    x_nnls, _ = nnls(A, b)
    assert np.abs(x - x_nnls).max() < 1e-9
    assert np.abs(x - xs).max() < 1e-9


def test_exact_recovery_on_well_conditioned_grid(orc):
    # 5 x 5 grid, 16 mics, spacing about one beamwidth: A is positive
    # definite; exact CSM of on-grid sources is recovered from x = 0.
    mic = synth.disc_array(16, 0.5, (42,))
    pts = [3, 12, 21]
    q = [1.0, 0.6, 0.3]
    w = synth.custom(mic, 5, (-1.2, 1.2, -1.2, 1.2), 1.0, [6000.0], pts, q)
    g = _geom(orc, w)
    A = orc.psf(orc.steering(g, 6000.0, np.arange(25)))
    np.linalg.cholesky(A)  # positive definite
    r = orc.solve_bin(g, 6000.0, w.csm[0], orc.SEL_KEEP_ALL, iters=4000)
    xt = np.zeros(25)
    xt[pts] = q
    assert np.abs(r["x"] - xt).max() < 1e-10


def test_resume_is_bitwise(orc):
    w = synth.plain_fp64()
    g = _geom(orc, w)
    b = orc.das_map(g, w.freqs[0], w.csm[0])
    A = orc.psf(orc.steering(g, w.freqs[0], np.arange(w.S)))
    x1 = orc.gs(A, b, 7)
    x2 = orc.gs(A, b, 5, x1)
    assert np.array_equal(x2, orc.gs(A, b, 12))


def test_solve_bin_composes_the_steps(orc):
    # Keep-all compressed DAMAS is plain DAMAS, bitwise, and solve_bin is
    # exactly DAS -> selection -> PSF -> sweeps -> scatter.
    w = synth.compressed_fp32(n_bins=2, N=21)
    g = _geom(orc, w)
    f = 1
    for mode, K in ((orc.SEL_KEEP_ALL, 0), (orc.SEL_KEEP_COUNT, 80)):
        r = orc.solve_bin(g, w.freqs[f], w.csm[f], mode, keep_count=K, iters=40)
        b = orc.das_map(g, w.freqs[f], w.csm[f])
        idx, _, _ = orc.select(w.N, b, mode, keep_count=K)
        A = orc.psf(orc.steering(g, w.freqs[f], idx))
        x = orc.gs(A, b[idx], 40)
        xm = np.zeros(w.S)
        xm[idx] = x
        assert np.array_equal(r["b"], b)
        assert np.array_equal(r["idx"], idx)
        assert np.array_equal(r["x"], xm)
    # x_init restarts from the kept entries of a full map
    r1 = orc.solve_bin(g, w.freqs[f], w.csm[f], orc.SEL_KEEP_COUNT, keep_count=80, iters=15)
    r2 = orc.solve_bin(g, w.freqs[f], w.csm[f], orc.SEL_KEEP_COUNT, keep_count=80, iters=25,
                       x_init=r1["x"])
    r3 = orc.solve_bin(g, w.freqs[f], w.csm[f], orc.SEL_KEEP_COUNT, keep_count=80, iters=40)
    assert np.array_equal(r2["x"], r3["x"])
