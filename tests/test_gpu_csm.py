"""Parity of the cross-spectral-matrix step (damas_csm, Eq. (1)) with the
oracle: within 1e-12 of max |C| (both sum in double, in different orders;
the bound is far above K ulps of the largest entry for K <= 2048), exactly
Hermitian with a real diagonal.  Shapes cover microphone counts that are
not multiples of the 32-wide block, snapshot counts that are not multiples
of the MFMA's 4, a single snapshot, and the batched workload's full size.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _snap(rng, nb, K, M):
    return (rng.standard_normal((nb, K, M)) + 1j * rng.standard_normal((nb, K, M))) * 0.7


def _check(orc, C, snap, bins):
    for f in bins:
        ref = orc.csm(snap[f])
        assert np.array_equal(C[f], C[f].conj().T), f
        assert (C[f].diagonal().imag == 0).all(), f
        err = np.abs(C[f] - ref).max()
        assert err <= 1e-12 * np.abs(ref).max(), (f, err)


@pytest.mark.parametrize("nb,K,M", [(2, 1, 5), (1, 3, 16), (2, 7, 33), (1, 9, 100),
                                    (3, 1024, 64), (2, 2048, 128), (1, 5, 1), (1, 130, 257)])
def test_csm_matches_oracle(orc, dm, dev, nb, K, M):
    import torch
    rng = np.random.default_rng(1000 + 7 * K + M)
    snap = _snap(rng, nb, K, M)
    C = dm.csm(torch.from_numpy(snap).to(dev)).cpu().numpy()
    _check(orc, C, snap, range(nb))


def test_csm_full_batched_size(orc, dm, dev):
    # 256 bins x 2048 snapshots x 128 microphones (1 GB of snapshots), the
    # batched workload's array and snapshot count; bins 0, 97 and 255 checked.
    import torch
    rng = np.random.default_rng(77)
    nb, K, M = 256, 2048, 128
    s = torch.empty(nb, K, M, dtype=torch.complex128, device=dev)
    host = {}
    for f in range(nb):  # generated per bin to bound host memory
        x = _snap(rng, 1, K, M)[0]
        s[f] = torch.from_numpy(x).to(dev)
        if f in (0, 97, 255):
            host[f] = x
    C = dm.csm(s)
    del s
    Ch = {f: C[f].cpu().numpy() for f in host}
    for f, x in host.items():
        ref = orc.csm(x)
        assert np.array_equal(Ch[f], Ch[f].conj().T), f
        assert np.abs(Ch[f] - ref).max() <= 1e-12 * np.abs(ref).max(), f


def test_csm_empty_and_reuse(orc, dm, dev):
    import torch
    rng = np.random.default_rng(3)
    out = torch.full((2, 40, 40), complex(7.0, 7.0), dtype=torch.complex128, device=dev)
    empty = torch.empty(0, 4, 40, dtype=torch.complex128, device=dev)
    dm.csm(empty, out=out[:0])
    assert (out.cpu().numpy() == complex(7.0, 7.0)).all()  # nothing written
    snap = _snap(rng, 2, 11, 40)
    dm.csm(torch.from_numpy(snap).to(dev), out=out)  # every entry overwritten
    _check(orc, out.cpu().numpy(), snap, range(2))
