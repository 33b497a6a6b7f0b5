"""Pins of the oracle's cross-spectral matrix (Eq. (1): the average of
p p^H over snapshots) against facts that do not come from its own formula.
"""
import numpy as np

from paper_1608_05179_amd import synth


def _field(M, freq, seed):
    rng = np.random.default_rng(seed)
    mic = synth.disc_array(M, 0.5, (seed,))
    src = np.array([[rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), 1.2]])
    return mic, synth.monopole_field(mic, src, freq)[:, 0]


def test_csm_exactly_hermitian_and_psd(orc):
    rng = np.random.default_rng(1)
    P = rng.standard_normal((37, 11)) + 1j * rng.standard_normal((37, 11))
    C = orc.csm(P)
    assert np.array_equal(C, C.conj().T)
    assert (C.diagonal().imag == 0).all() and (C.diagonal().real > 0).all()
    w = np.linalg.eigvalsh(C)
    assert w.min() >= -1e-13 * w.max()
    # 11 microphones and 37 snapshots: full rank; 4 snapshots: rank 4
    assert (w > 1e-8 * w.max()).sum() == 11
    w4 = np.linalg.eigvalsh(orc.csm(P[:4]))
    assert (w4 > 1e-8 * w4.max()).sum() == 4


def test_csm_of_one_source_with_unit_amplitudes(orc):
    # p_k = g s_k with |s_k| = 1: C = g g^H whatever the phases.  Pins the
    # conjugate's side, the operand order and the 1/K.
    M, K = 16, 9
    _, g = _field(M, 3000.0, 2)
    s = np.exp(1j * np.random.default_rng(3).uniform(0, 2 * np.pi, K))
    C = orc.csm(s[:, None] * g[None, :])
    assert np.abs(C - np.outer(g, g.conj())).max() < 1e-14


def test_csm_of_orthogonal_sources_is_the_exact_csm(orc):
    # Source j sends sqrt(q_j) exp(2 pi i j k / K) in snapshot k; over K
    # snapshots the sequences are exactly orthogonal, so the average of
    # p p^H is sum_j q_j g_j g_j^H: the generator's exact CSM, formed there
    # by a matrix product of its own.
    M, K, J = 24, 12, 3
    mic = synth.disc_array(M, 0.5, (4,))
    rng = np.random.default_rng(5)
    src = np.column_stack([rng.uniform(-0.6, 0.6, J), rng.uniform(-0.6, 0.6, J),
                           np.full(J, 1.4)])
    q = np.array([1.0, 0.4, 0.15])
    f = 4500.0
    g = synth.monopole_field(mic, src, f)                 # M x J
    k = np.arange(K)
    s = np.sqrt(q)[:, None] * np.exp(2j * np.pi * np.arange(J)[:, None] * k[None, :] / K)
    P = (g @ s).T                                          # K x M
    C = orc.csm(P)
    ref = synth.exact_csm(mic, src, q, f)
    assert np.abs(C - ref).max() < 1e-14 * max(1.0, np.abs(ref).max()) * M


def test_csm_scales_with_amplitude_squared(orc):
    rng = np.random.default_rng(6)
    P = rng.standard_normal((5, 7)) + 1j * rng.standard_normal((5, 7))
    a = 0.5 - 2.0j  # |a|^2 = 4.25; powers of two keep the products exact
    C1, C2 = orc.csm(P), orc.csm(a * P)
    assert np.abs(C2 - 4.25 * C1).max() < 1e-13 * np.abs(C1).max()
