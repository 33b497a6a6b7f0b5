"""Pins of the oracle's two options beside the default readings: removal of
the CSM diagonal (section "Beamforming") with its matching point-spread
matrix, and the paper's amplitude-weighted steering pair v_m = (d_m/|r|)
e_m for the beamformer and g_m = (|r|/d_m) e_m for the source model
(sections "Beamforming" and "DAMAS").  Each pin is a closed form written
out in the test, a special case that reduces to the default path bitwise,
or an identity between the map and the matrix that a dropped or misplaced
term breaks.
"""
import numpy as np
import pytest

from paper_1608_05179_amd import synth


def _geom(orc, M=12, N=9, z0=1.2, seed=4, ext=0.8):
    rng = np.random.default_rng(seed)
    mic = np.zeros((M, 3))
    mic[:, 0] = rng.uniform(-0.4, 0.4, M)
    mic[:, 1] = rng.uniform(-0.4, 0.4, M)
    return orc.Geometry(mic, N, -ext, ext, -ext * 0.7, ext * 1.1, z0)


@pytest.mark.parametrize("form", [0, 1])
def test_diagonal_removal_rejects_white_noise(orc, form):
    g = _geom(orc)
    M = g.mic.shape[0]
    sigma2 = 0.37
    C = sigma2 * np.eye(M, dtype=np.complex128)
    b = orc.das_map_ex(g, 2500.0, C, form=form, diag_removal=True)
    assert np.abs(b).max() <= 1e-15 * sigma2
    # without removal: sigma^2 sum_m |v_m|^2 / M^2 (sigma^2 / M for the unit form)
    b0 = orc.das_map_ex(g, 2500.0, C, form=form, diag_removal=False)
    v, _ = orc.steering_form(g, 2500.0, np.arange(g.N * g.N), form)
    want = sigma2 * (np.abs(v) ** 2).sum(axis=1) / M ** 2
    assert np.allclose(b0, want, rtol=1e-13, atol=0)
    if form == 0:
        assert np.allclose(b0, sigma2 / M, rtol=1e-13)


def test_psf_with_orthogonal_steering(orc):
    # DFT rows are orthogonal: |v_i^H v_j|^2 = M^2 delta_ij, so with the
    # diagonal removed the off-diagonal entries are -M / (M^2 - M) exactly.
    M, S = 8, 8
    v = np.exp(-2j * np.pi * np.outer(np.arange(S), np.arange(M)) / M)
    A = orc.psf_ex(v, v, diag_removal=True)
    want = np.full((S, S), -1.0 / (M - 1))
    np.fill_diagonal(want, 1.0)
    assert np.allclose(A, want, rtol=1e-13, atol=1e-14)
    assert np.allclose(orc.psf_ex(v, v, diag_removal=False), np.eye(S), atol=1e-14)


def test_psf_hand_computed_two_mics(orc):
    # M = 2, entries worked by hand:
    #   v = [1, 1], w = [1, i]:  |v^H w|^2 = |1 + i|^2 = 2, sum |v|^2|w|^2 = 2
    #   v = [2, 1], w = [1, 1]:  |v^H w|^2 = 9, sum |v|^2|w|^2 = 5
    v = np.array([[1, 1], [2, 1]], dtype=np.complex128)
    w = np.array([[1, 1j], [1, 1]], dtype=np.complex128)
    A = orc.psf_ex(v, w, diag_removal=True)    # (|.|^2 - dd) / (4 - 2)
    A0 = orc.psf_ex(v, w, diag_removal=False)  # |.|^2 / 4
    # rows: beamformer point i; columns: source point j
    assert A[0, 0] == (2 - 2) / 2 and A0[0, 0] == 2 / 4
    assert A[1, 1] == (9 - 5) / 2 and A0[1, 1] == 9 / 4
    # v_0 = [1, 1] with w_1 = [1, 1]: 4 and 2;  v_1 = [2, 1] with w_0 = [1, i]:
    # |2 + i|^2 = 5 and 4 + 1 = 5
    assert A[0, 1] == (4 - 2) / 2 and A[1, 0] == (5 - 5) / 2
    assert A0[0, 1] == 1.0 and A0[1, 0] == 5 / 4


def test_unit_form_options_off_are_the_default_path(orc):
    g = _geom(orc)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((g.mic.shape[0], 20)) + 1j * rng.standard_normal((g.mic.shape[0], 20))
    C = X @ X.conj().T / 20
    assert np.array_equal(orc.das_map_ex(g, 3100.0, C), orc.das_map(g, 3100.0, C))
    pts = np.arange(0, g.N * g.N, 3)
    v, w = orc.steering_form(g, 3100.0, pts)
    e = orc.steering(g, 3100.0, pts)
    assert np.array_equal(v, e) and np.array_equal(w, e)
    assert np.array_equal(orc.psf_ex(v, w), orc.psf(e))


def test_paper_pair_single_mic_closed_form(orc):
    # One microphone at (xm, ym, 0): v^H g = (d_i/|r_i|)(|r_j|/d_j) exp(...),
    # so A[i][j] = ((d_i |r_j|) / (|r_i| d_j))^2 with d the distance to the
    # mic and |r| the distance to the origin.
    mic = np.array([[0.31, -0.12, 0.0]])
    g = orc.Geometry(mic, 5, -0.5, 0.5, -0.5, 0.5, 0.9)
    S = 25
    v, w = orc.steering_form(g, 1800.0, np.arange(S), orc.STEER_PAPER)
    A = orc.psf_ex(v, w)
    xs = np.linspace(-0.5, 0.5, 5)
    r = np.array([[xs[n % 5], xs[n // 5], 0.9] for n in range(S)])
    d = np.linalg.norm(r - mic[0], axis=1)
    rn = np.linalg.norm(r, axis=1)
    want = ((d[:, None] * rn[None, :]) / (rn[:, None] * d[None, :])) ** 2
    assert np.allclose(A, want, rtol=1e-12)


@pytest.mark.parametrize("diag", [False, True])
def test_paper_pair_unit_diagonal_and_asymmetry(orc, diag):
    g = _geom(orc, M=16)
    v, w = orc.steering_form(g, 2200.0, np.arange(g.N * g.N), orc.STEER_PAPER)
    A = orc.psf_ex(v, w, diag_removal=diag)
    assert np.allclose(np.diag(A), 1.0, atol=1e-13)
    assert np.abs(A - A.T).max() > 1e-3  # not symmetric off the array axis


@pytest.mark.parametrize("form,model", [(0, "unit"), (1, "spherical")])
@pytest.mark.parametrize("diag", [False, True])
def test_map_is_psf_times_powers_for_on_grid_sources(orc, form, model, diag):
    # An exact CSM of uncorrelated on-grid sources (the source model that
    # matches the steering form): the map at every grid point is the PSF
    # matrix times the source powers, diagonal removed or not.
    g = _geom(orc, M=14, N=11)
    src = np.array([7, 40, 88, 113])
    q = np.array([1.0, 0.4, 0.75, 0.2])
    xyz = synth.grid_xyz(g.N, g.x0, g.x1, g.y0, g.y1, g.z0, src)
    C = synth.exact_csm(g.mic, xyz, q, 2700.0, model=model)
    b = orc.das_map_ex(g, 2700.0, C, form=form, diag_removal=diag)
    v, w = orc.steering_form(g, 2700.0, np.arange(g.N * g.N), form)
    A = orc.psf_ex(v, w, diag_removal=diag)
    assert np.allclose(b, A[:, src] @ q, rtol=1e-11, atol=1e-13)


def test_diagonal_removal_maps_can_go_negative(orc):
    g = _geom(orc, M=10, N=15)
    w = synth.custom(g.mic, g.N, (g.x0, g.x1, g.y0, g.y1), g.z0, [3000.0], [50, 170],
                     [1.0, 0.5], snapshots=64, snr_db=0.0, seed=5)
    b = orc.das_map_ex(g, 3000.0, w.csm[0], diag_removal=True)
    assert b.min() < 0.0 < b.max()


def test_solve_bin_ex_composes_the_steps(orc):
    g = _geom(orc, M=16, N=13)
    w = synth.custom(g.mic, g.N, (g.x0, g.x1, g.y0, g.y1), g.z0, [2600.0], [30, 100],
                     [1.0, 0.6], snapshots=256, snr_db=15.0, seed=7, model="spherical")
    for form in (0, 1):
        for diag in (False, True):
            r = orc.solve_bin_ex(g, 2600.0, w.csm[0], orc.SEL_KEEP_COUNT, form=form,
                                 diag_removal=diag, keep_count=60, iters=50)
            b = orc.das_map_ex(g, 2600.0, w.csm[0], form, diag)
            kept, _, _ = orc.select(g.N, b, orc.SEL_KEEP_COUNT, keep_count=60)
            assert np.array_equal(r["idx"], kept)
            v, wv = orc.steering_form(g, 2600.0, kept, form)
            x = orc.gs(orc.psf_ex(v, wv, diag), b[kept], 50)
            assert np.array_equal(r["x"][kept], x)
