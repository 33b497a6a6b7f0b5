"""Algorithm 1 with the linear interpolating predictor on the GPU: the kept
set is bit-exact against the oracle (both form 0.5 (a + b) and
0.25 ((a + b) + (c + d)) in double with no fused operation), on grids whose
stencils fit (N = 2^J + 1), grids with mirrored neighbours at the far edges,
and powers of two; and the whole path with this predictor agrees with the
oracle's composition of the same steps within 1e-4 relative L2 (FP32 A).
"""
import numpy as np
import pytest

from paper_1608_05179_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N", [9, 16, 17, 21, 41, 101])
@pytest.mark.parametrize("mode", ["eps", "count"])
def test_select_linear_bit_exact(orc, dm, dev, N, mode):
    import torch
    rng = np.random.default_rng(40 + N)
    nb = 3
    b = rng.standard_normal((nb, N * N)) ** 2
    b[1] = np.linspace(0.0, 1.0, N * N) ** 3  # smooth map: many small details
    b_d = torch.from_numpy(b).to(dev)
    if mode == "eps":
        idx, st = dm.select(N, b_d, dm.SEL_EPS_REL, eps=0.05, predictor=dm.PRED_LINEAR)
    else:
        K = max(4, N * N // 5)
        kc = torch.full((nb,), K, dtype=torch.int32, device=dev)
        idx, st = dm.select(N, b_d, dm.SEL_KEEP_COUNT, keep_count=kc, predictor=dm.PRED_LINEAR)
    idx, st = idx.cpu().numpy(), st.cpu().numpy()
    for f in range(nb):
        if mode == "eps":
            ref, _, margin = orc.select(N, b[f], orc.SEL_EPS_REL, eps=0.05,
                                        predictor=orc.PRED_LINEAR)
        else:
            ref, _, margin = orc.select(N, b[f], orc.SEL_KEEP_COUNT, keep_count=K,
                                        predictor=orc.PRED_LINEAR)
        assert st[f] == len(ref), (f, st[f], len(ref))
        assert np.array_equal(idx[f, :st[f]], ref), f


def test_select_linear_differs_from_haar(orc, dm, dev):
    import torch
    N = 41
    b = (np.arange(N * N, dtype=np.float64) % N) * 0.01 + 1.0  # linear in x
    b_d = torch.from_numpy(b[None]).to(dev)
    _, st_lin = dm.select(N, b_d, dm.SEL_EPS_REL, eps=1e-9, predictor=dm.PRED_LINEAR)
    _, st_haar = dm.select(N, b_d, dm.SEL_EPS_REL, eps=1e-9)
    # a linear ramp is predicted exactly except where the stencil is mirrored
    ref_lin, _, _ = orc.select(N, b, orc.SEL_EPS_REL, eps=1e-9, predictor=orc.PRED_LINEAR)
    assert int(st_lin[0]) == len(ref_lin) < int(st_haar[0])


def test_solve_with_linear_predictor(orc, dm, dev):
    import torch
    w = synth.compressed_fp32(n_bins=3, N=41, iterations=200)
    K = w.keep_count
    mic = torch.tensor(w.mic, dtype=torch.float64, device=dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    freq = torch.tensor(w.freqs, dtype=torch.float64, device=dev)
    csm = torch.tensor(w.csm, dtype=torch.complex128, device=dev)
    st = torch.zeros(w.n_bins, dtype=torch.int32, device=dev)
    idx = torch.zeros(w.n_bins, w.S, dtype=torch.int32, device=dev)
    ctx = dm.Context(0)
    x = ctx.solve(g, freq, csm, select_mode=dm.SEL_KEEP_COUNT, keep_count=K,
                  iterations=w.iterations, precision=dm.PREC_FP32, idx=idx, s_tilde=st,
                  predictor=dm.PRED_LINEAR)
    ctx.check()
    ctx.close()
    x, st, idx = x.double().cpu().numpy(), st.cpu().numpy(), idx.cpu().numpy()
    og = orc.Geometry(w.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    for f in range(w.n_bins):
        b = orc.das_map(og, w.freqs[f], w.csm[f])
        kept, _, margin = orc.select(w.N, b, orc.SEL_KEEP_COUNT, keep_count=K,
                                     predictor=orc.PRED_LINEAR)
        assert margin > 1e-12, (f, margin)
        assert np.array_equal(idx[f, :st[f]], kept), f
        A = orc.psf(orc.steering(og, w.freqs[f], kept))
        ref = np.zeros(w.S)
        ref[kept] = orc.gs(A, b[kept], w.iterations)
        err = np.linalg.norm(x[f] - ref) / np.linalg.norm(ref)
        assert err <= 1e-4, (f, err)


def test_select_linear_mirror_fixture(orc, dm, dev):
    # The hand-derived spike fixture: the mirrored point (20, 0) has detail
    # exactly 1.0, so eps = 1 keeps it (with the 4 coarse points) and
    # eps = 0.75 keeps it alone of the fine points; a clamp reading keeps
    # neither.
    import json
    import os
    import torch
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "select_linear_mirror_N21.json")) as fh:
        g = json.load(fh)
    N = g["N"]
    b = np.zeros(N * N)
    b[g["spike"][1] * N + g["spike"][0]] = 1.0
    b_d = torch.from_numpy(b[None]).to(dev)
    coarse = [0, 16, 16 * N, 16 * N + 16]
    for eps, want in ((1.0, sorted(coarse + [20])), (0.75, sorted(coarse + [20])),
                      (0.5, None)):
        idx, st = dm.select(N, b_d, dm.SEL_EPS_REL, eps=eps, predictor=dm.PRED_LINEAR)
        got = idx[0, :int(st[0])].cpu().numpy()
        ref, _, _ = orc.select(N, b, orc.SEL_EPS_REL, eps=eps, predictor=orc.PRED_LINEAR)
        assert np.array_equal(got, ref), eps
        if want is not None:
            assert got.tolist() == want, (eps, got.tolist())
