"""Pins of the oracle's geometry, steering, DAS map and point-spread matrix.

Each test checks the oracle against something other than itself: a closed
form, an exact identity of the paper's source model, or an invariant that a
plausible slip (a dropped conjugate, a transposed CSM, a wrong normalisation,
a wrong sign in the phase) would break.
"""
import json
import os

import numpy as np
import pytest

from paper_1608_05179_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _geom(orc, w):
    return orc.Geometry(w.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)


def test_grid_points_closed_form(orc):
    # Scan plane of N x N equidistant points, end points included
    # (section "Beamforming"); n = iy*N + ix.
    g = orc.Geometry(np.zeros((1, 3)), 3, -1.0, 1.0, -2.0, 2.0, 1.5)
    assert np.array_equal(orc.grid_point(g, 0), [-1.0, -2.0, 1.5])
    assert np.array_equal(orc.grid_point(g, 4), [0.0, 0.0, 1.5])
    assert np.array_equal(orc.grid_point(g, 5), [1.0, 0.0, 1.5])
    assert np.array_equal(orc.grid_point(g, 8), [1.0, 2.0, 1.5])
    # matches the generator's independent linspace placement
    w = synth.plain_fp64()
    gw = _geom(orc, w)
    xyz = synth.grid_xyz(w.N, w.x0, w.x1, w.y0, w.y1, w.z0, np.arange(w.S))
    ours = np.array([orc.grid_point(gw, n) for n in range(w.S)])
    assert np.abs(ours - xyz).max() < 1e-15


def test_steering_345_triangle(orc):
    # Two mics at (0,0,0) and (3,0,0), focus (0,0,4): distances 4 and 5
    # (3-4-5 triangle).  With k = 1 the phases are 4 and 5 rad and the
    # component is exp(-i k d).
    mic = np.array([[0.0, 0.0, 0.0], [3.0, 0.0, 0.0]])
    c = 343.0
    g = orc.Geometry(mic, 2, 0.0, 3.0, 0.0, 3.0, 4.0, c)
    f = c / (2.0 * np.pi)  # k = 2 pi f / c = 1
    e = orc.steering(g, f, [0])[0]
    assert abs(e[0] - (np.cos(4.0) - 1j * np.sin(4.0))) < 1e-14
    assert abs(e[1] - (np.cos(5.0) - 1j * np.sin(5.0))) < 1e-14
    # focus (3,0,4): distances 5 and 4
    e = orc.steering(g, f, [1])[0]
    assert abs(np.angle(e[0]) - np.angle(np.exp(-5j))) < 1e-13
    assert abs(np.angle(e[1]) - np.angle(np.exp(-4j))) < 1e-13


def test_steering_unit_magnitude(orc):
    w = synth.compressed_fp32(n_bins=1)
    g = _geom(orc, w)
    e = orc.steering(g, 8000.0, np.arange(0, w.S, 7))
    assert np.abs(np.abs(e) - 1.0).max() < 1e-14


def test_das_exact_csm_equals_psf_times_powers(orc):
    # Incoherent on-grid sources: C = sum_s x_s g_s g_s^H gives
    # b = A x (Eq. dirty_map_3 and Eq. Axb) exactly up to rounding.
    w = synth.plain_fp64()
    g = _geom(orc, w)
    b = orc.das_map(g, w.freqs[0], w.csm[0])
    A = orc.psf(orc.steering(g, w.freqs[0], np.arange(w.S)))
    x = np.zeros(w.S)
    x[w.sources] = w.powers
    assert np.abs(A @ x - b).max() < 1e-12 * b.max()


def test_das_single_source_is_psf_column(orc):
    mic = synth.disc_array(24, 0.5, (77,))
    n0 = 5 * 13 + 7
    w = synth.custom(mic, 13, (-0.6, 0.6, -0.6, 0.6), 1.2, [5000.0], [n0], [1.0])
    g = _geom(orc, w)
    b = orc.das_map(g, w.freqs[0], w.csm[0])
    A = orc.psf(orc.steering(g, w.freqs[0], np.arange(w.S)))
    assert abs(b[n0] - 1.0) < 1e-13          # unit source seen at its own point
    assert int(np.argmax(b)) == n0
    assert np.abs(b - A[:, n0]).max() < 1e-13
    assert b.min() > -1e-15


def test_das_white_noise_closed_form(orc):
    # C = s2 * I gives e^H C e / M^2 = s2 * M / M^2 at every point.
    mic = synth.disc_array(20, 0.5, (5,))
    g = orc.Geometry(mic, 7, -1.0, 1.0, -1.0, 1.0, 1.0)
    s2 = 0.37
    b = orc.das_map(g, 3000.0, s2 * np.eye(20, dtype=complex))
    assert np.abs(b - s2 / 20).max() < 1e-15


def test_das_noisy_csm_bounds(orc):
    # C Hermitian PSD: 0 <= b_n <= lambda_max(C) / M.
    w = synth.compressed_fp32(n_bins=3)
    g = _geom(orc, w)
    for f in range(3):
        b = orc.das_map(g, w.freqs[f], w.csm[f])
        lmax = np.linalg.eigvalsh(w.csm[f]).max()
        assert b.min() >= -1e-12
        assert b.max() <= lmax / w.M * (1 + 1e-12)


def test_psf_invariants(orc):
    w = synth.plain_fp64()
    g = _geom(orc, w)
    A = orc.psf(orc.steering(g, w.freqs[0], np.arange(w.S)))
    M = w.M
    assert np.array_equal(A, A.T)                          # mirrored: exact
    assert np.abs(np.diag(A) - 1.0).max() < 1e-13           # |e| = 1
    assert A.min() >= 0.0 and A.max() <= 1.0 + 1e-13        # Cauchy-Schwarz
    assert np.linalg.eigvalsh(A).min() > -1e-10            # Schur product of PSD
    # A_nn' = |u_n^H u_n'|/M^2 with u_n = e_n (x) conj(e_n): the M diagonal
    # coordinates of u_n are all 1, so rank(A) <= M^2 - M + 1.
    assert np.linalg.matrix_rank(A, tol=1e-9) <= M * M - M + 1


def test_psf_dft_steering_is_identity(orc):
    # Columns of an M-point DFT are orthogonal: A = I exactly in exact
    # arithmetic.  A dropped conjugate would give |sum w^{(a+b)m}|^2 != 0.
    M = 8
    m = np.arange(M)
    e = np.exp(-2j * np.pi * np.outer(m, m) / M)
    A = orc.psf(e)
    assert np.abs(A - np.eye(M)).max() < 1e-14


def test_psf_conjugation_hand_case(orc):
    # e_1 = e_2 = [1, i]: e_1^H e_2 = 1 + 1 = 2 so A_12 = 4 / 4 = 1;
    # without the conjugate it would be 1 + i*i = 0.
    e = np.array([[1.0, 1j], [1.0, 1j], [1.0, -1.0]])
    A = orc.psf(e)
    assert A[0, 1] == 1.0
    # e_1^H e_3 = 1 + (-i)(-1) = 1 + i, |.|^2 = 2 -> 0.5
    assert abs(A[0, 2] - 0.5) < 1e-15
