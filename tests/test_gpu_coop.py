"""Cooperative sweeps (several workgroups per bin) against the oracle and
against the one-workgroup kernel.  The iteration is the same; only the
summation order of each residual changes, so FP64 agrees with the oracle to
1e-9 and with the one-workgroup result to 1e-11, and FP32 storage within
1e-4 of the oracle."""
import numpy as np
import pytest

from paper_1608_05179_amd import synth

pytestmark = pytest.mark.gpu


def _t(a, dtype, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype)


def _solve(dm, dev, w, mode, K, prec, coop, refine=0):
    import torch
    mic = _t(w.mic, torch.float64, dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    ctx = dm.Context(0)
    ctx.set_coop(coop)
    st = torch.zeros(w.n_bins, dtype=torch.int32, device=dev)
    idx = torch.zeros(w.n_bins, w.S, dtype=torch.int32, device=dev)
    x = ctx.solve(g, _t(w.freqs, torch.float64, dev), _t(w.csm, torch.complex128, dev),
                  select_mode=mode, keep_count=K, iterations=w.iterations, precision=prec,
                  refine_sweeps=refine, idx=idx, s_tilde=st)
    ctx.check()
    wg = ctx.last_workgroups()
    if coop == 0:
        assert wg == w.n_bins
    elif coop > 0:
        assert wg <= coop  # the budget holds (bins pack when it is small)
    else:
        assert wg > w.n_bins  # some bin had helpers
    out = x.double().cpu().numpy(), st.cpu().numpy(), idx.cpu().numpy()
    ctx.close()
    return out


def _oracle(orc, w, f, mode, K):
    og = orc.Geometry(w.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    return orc.solve_bin(og, w.freqs[f], w.csm[f], mode, keep_count=K, iters=w.iterations)


def test_coop_fp64_keep_all(orc, dm, dev):
    # 41 x 41 grid kept whole (1681 unknowns, 27 tiles), 2 bins, 60 sweeps
    w = synth.precision_bf16(n_bins=2, N=41, iterations=60)
    x1, _, _ = _solve(dm, dev, w, dm.SEL_KEEP_ALL, None, dm.PREC_FP64, 0)
    xc, _, _ = _solve(dm, dev, w, dm.SEL_KEEP_ALL, None, dm.PREC_FP64, -1)
    for f in range(w.n_bins):
        ref = _oracle(orc, w, f, orc.SEL_KEEP_ALL, 0)["x"]
        assert np.linalg.norm(xc[f] - ref) <= 1e-9 * np.linalg.norm(ref), f
        assert np.linalg.norm(xc[f] - x1[f]) <= 1e-11 * np.linalg.norm(x1[f]), f


@pytest.mark.parametrize("budget", [-1, 6, 37])
def test_coop_fp32_uneven_bins(orc, dm, dev, budget):
    # uneven kept counts: the big bins get helpers, the small ones none;
    # budgets that leave one or several helpers per bin
    w = synth.compressed_fp32(n_bins=4, N=61, iterations=200)
    Ks = [2400, 700, 3600, 150]
    xc, st, idx = _solve(dm, dev, w, dm.SEL_KEEP_COUNT, Ks, dm.PREC_FP32, budget)
    for f in range(w.n_bins):
        ref = _oracle(orc, w, f, orc.SEL_KEEP_COUNT, Ks[f])
        if ref["margin"] > 1e-12:
            assert np.array_equal(idx[f, :st[f]], ref["idx"]), f
        err = np.linalg.norm(xc[f] - ref["x"]) / np.linalg.norm(ref["x"])
        assert err <= 1e-4, (f, err)


def test_coop_bf16_refined_equals_one_workgroup(dm, dev):
    # bf16 bulk + FP32 refinement, 2 bins of 1681 unknowns: cooperative and
    # one-workgroup sweeps read the same A and differ only in summation order
    w = synth.precision_bf16(n_bins=2, N=41, iterations=100)
    w.freqs, w.csm = w.freqs[::-1].copy(), w.csm[::-1].copy()  # the 10 kHz end
    a, _, _ = _solve(dm, dev, w, dm.SEL_KEEP_ALL, None, dm.PREC_BF16, 0, refine=20)
    b, _, _ = _solve(dm, dev, w, dm.SEL_KEEP_ALL, None, dm.PREC_BF16, -1, refine=20)
    for f in range(w.n_bins):
        assert np.linalg.norm(a[f] - b[f]) <= 1e-5 * np.linalg.norm(a[f]), f


def test_coop_off_is_the_one_workgroup_kernel(dm, dev):
    w = synth.compressed_fp32(n_bins=2, N=41, iterations=40)
    Ks = [1200, 1600]
    a, _, _ = _solve(dm, dev, w, dm.SEL_KEEP_COUNT, Ks, dm.PREC_FP32, 0)
    b, _, _ = _solve(dm, dev, w, dm.SEL_KEEP_COUNT, Ks, dm.PREC_FP32, 0)
    assert np.array_equal(a, b)
    c, _, _ = _solve(dm, dev, w, dm.SEL_KEEP_COUNT, Ks, dm.PREC_FP32, -1)
    assert np.linalg.norm(a - c) <= 1e-5 * np.linalg.norm(a)


@pytest.mark.parametrize("budget", [5, -1])
def test_coop_packs_bins_onto_workgroups(orc, dm, dev, budget):
    # 12 uneven bins; a budget of 5 workgroups packs several bins alone onto
    # each workgroup after the ranks of the largest
    w = synth.compressed_fp32(n_bins=12, N=61, iterations=80)
    rng = np.random.default_rng(9)
    Ks = [int(k) for k in rng.integers(150, 3000, size=12)]
    Ks[3] = 3600
    x, st, idx = _solve(dm, dev, w, dm.SEL_KEEP_COUNT, Ks, dm.PREC_FP32, budget)
    for f in (3, 0, 7, 11):
        ref = _oracle(orc, w, f, orc.SEL_KEEP_COUNT, Ks[f])
        if ref["margin"] > 1e-12:
            assert np.array_equal(idx[f, :st[f]], ref["idx"]), f
        err = np.linalg.norm(x[f] - ref["x"]) / np.linalg.norm(ref["x"])
        assert err <= 1e-4, (f, err)
    # every bin was solved: the map is zero exactly off each kept set
    for f in range(w.n_bins):
        offk = np.ones(w.S, bool)
        offk[idx[f, :st[f]]] = False
        assert (x[f, offk] == 0).all() and x[f, ~offk].max() > 0


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_coop_run_to_run_bitwise(dm, dev, prec):
    # The cooperative kernel's sums are added in a fixed order (the owner's
    # stream waves as a tree, then the helpers in rank order), so repeated
    # solves give the same bits; a race in the owner-helper exchange (a sum
    # read before it is published, an x tile read mid-update) would not.
    if prec == "fp32":
        w = synth.compressed_fp32(n_bins=4, N=61, iterations=120)
        Ks = [2400, 700, 3600, 150]
        args = (dm.SEL_KEEP_COUNT, Ks, dm.PREC_FP32, -1)
        kw = {}
    else:
        w = synth.precision_bf16(n_bins=3, N=61, iterations=120)
        args = (dm.SEL_KEEP_ALL, None, dm.PREC_BF16, -1)
        kw = {"refine": 30}
    runs = [_solve(dm, dev, w, *args, **kw)[0] for _ in range(3)]
    assert np.isfinite(runs[0]).all() and runs[0].max() > 0
    for r in runs[1:]:
        assert np.array_equal(r, runs[0])
