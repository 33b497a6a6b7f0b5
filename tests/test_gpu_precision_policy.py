"""Per-bin precision classes (DAMAS_POLICY_AUTO).

A bin's class comes from its mean PSF row sum over the kept points,
rho = (1/S~) sum_ij A_ij, computed on the device from the tile sums of the
float PSF: in a float solve, a bin with rho above rho_wide is wide (A as
float hi + bf16 lo, FP64 strip sums); in a bf16 solve, a bin above rho_f32
runs every sweep on the float system.  Checked here: the classes match the
oracle's rho, a forced-wide solve stays within 2e-6 of the FP64 iterate on
the one-workgroup and the cooperative kernels (float storage alone moves
these iterates by up to 1e-5), the policy changes nothing where no bin is
widened, and a bf16 solve meets 1e-4 on every bin under the policy.
"""
import numpy as np
import pytest

from paper_1608_05179_amd import synth

pytestmark = pytest.mark.gpu


def _t(a, dtype, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype)


def _solve(dm, dev, w, K, prec=None, coop=-1, refine=0, **kw):
    import torch
    prec = dm.PREC_FP32 if prec is None else prec
    mic = _t(w.mic, torch.float64, dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    ctx = dm.Context(0)
    ctx.set_coop(coop)
    st = torch.zeros(w.n_bins, dtype=torch.int32, device=dev)
    idx = torch.zeros(w.n_bins, w.S, dtype=torch.int32, device=dev)
    mode = dm.SEL_KEEP_COUNT if K is not None else dm.SEL_KEEP_ALL
    x = ctx.solve(g, _t(w.freqs, torch.float64, dev), _t(w.csm, torch.complex128, dev),
                  select_mode=mode, keep_count=K, iterations=w.iterations, precision=prec,
                  refine_sweeps=refine, idx=idx, s_tilde=st, **kw)
    ctx.check()
    cls = ctx.classes(w.n_bins) if kw.get("policy", dm.POLICY_AUTO) == dm.POLICY_AUTO \
        and prec != dm.PREC_FP64 else None
    wg = ctx.last_workgroups()
    out = x.double().cpu().numpy(), st.cpu().numpy(), idx.cpu().numpy(), cls, wg
    ctx.close()
    return out


def _oracle_bin(orc, w, f, K):
    og = orc.Geometry(w.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    b = orc.das_map(og, w.freqs[f], w.csm[f])
    mode = orc.SEL_KEEP_COUNT if K is not None else orc.SEL_KEEP_ALL
    kept, _, _ = orc.select(w.N, b, mode, keep_count=0 if K is None else K[f])
    A = orc.psf(orc.steering(og, w.freqs[f], kept))
    return kept, A, b[kept]


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("coop", [0, -1])
def test_forced_wide_is_near_the_fp64_iterate(orc, dm, dev, coop):
    # Every bin wide (rho_wide below any rho): uneven bins on the 61 x 61
    # grid, the large ones on several cooperating workgroups when coop = -1.
    w = synth.compressed_fp32(n_bins=4, N=61, iterations=300)
    w.freqs = np.array([1000.0, 1250.0, 3000.0, 6000.0])
    w.csm = np.stack([synth.snapshot_csm(w.mic, synth.grid_xyz(w.N, w.x0, w.x1, w.y0, w.y1,
                                                                w.z0, w.sources),
                                         w.powers, f, 1024, 20.0, (9, k))
                      for k, f in enumerate(w.freqs)])
    K = [2400, 700, 3600, 150]
    x, st, idx, cls, wg = _solve(dm, dev, w, K, coop=coop, rho_wide=1e-9)
    assert (cls == dm.CLASS_WIDE).all()
    if coop == -1:
        assert wg > w.n_bins
    for f in range(w.n_bins):
        kept, A, bt = _oracle_bin(orc, w, f, K)
        assert np.array_equal(idx[f, :st[f]], kept)
        ref = orc.gs(A, bt, w.iterations)
        e = _rel(x[f, kept], ref)
        print(f"bin {f} ({w.freqs[f]:.0f} Hz, {st[f]} kept): wide vs FP64 {e:.2e}")
        assert e <= 2e-6, (f, e)


def test_classes_follow_rho(orc, dm, dev):
    # The batched workload's first 24 bins (0.5-1.5 kHz, 101 x 101 grid,
    # 300-4000 kept) straddle the default threshold rho = 100.
    w = synth.batched_fp32(n_bins=24, iterations=4)
    K = [int(k) for k in w.keep_counts]
    _, st, _, cls, _ = _solve(dm, dev, w, K)
    cap = dm.wide_capacity()
    n_wide = 0
    for f in range(w.n_bins):
        kept, A, _ = _oracle_bin(orc, w, f, K)
        rho = A.sum() / len(kept)
        if abs(rho - 100.0) < 1e-6 * 100.0:
            continue
        want = dm.CLASS_WIDE if rho > 100.0 and len(kept) <= cap else dm.CLASS_NARROW
        assert cls[f] == want, (f, rho, cls[f])
        n_wide += want == dm.CLASS_WIDE
    assert 0 < n_wide < w.n_bins


def test_auto_without_wide_bins_equals_fixed(dm, dev):
    # High, well-separated bins: no bin is widened, and the policy's extra
    # outputs leave the sweeps untouched.
    w = synth.compressed_fp32(n_bins=6, N=41, iterations=150)
    w.freqs, w.csm = w.freqs[::-1].copy(), w.csm[::-1].copy()
    a, _, _, cls, _ = _solve(dm, dev, w, w.keep_count)
    b, _, _, _, _ = _solve(dm, dev, w, w.keep_count, policy=dm.POLICY_FIXED)
    assert (cls == dm.CLASS_NARROW).all()
    assert np.array_equal(a, b)


def test_bf16_policy_meets_the_bar(orc, dm, dev):
    # A bf16 solve of 8 bins over 1-8 kHz with 60 refinement sweeps: bins
    # with rho above 12 run every sweep on float A (and would miss 1e-4 on
    # bf16), the sparse high bins keep the bf16 bulk.
    w = synth.compressed_fp32(n_bins=64, N=41, iterations=400)
    sel = [0, 9, 21, 33, 45, 51, 57, 63]
    w.freqs, w.csm = w.freqs[sel].copy(), w.csm[sel].copy()
    x, st, idx, cls, _ = _solve(dm, dev, w, w.keep_count, prec=dm.PREC_BF16, refine=60)
    n16 = 0
    for f in range(w.n_bins):
        kept, A, bt = _oracle_bin(orc, w, f, [w.keep_count] * w.n_bins)
        rho = A.sum() / len(kept)
        if abs(rho - 12.0) > 1e-6 * 12.0:
            want = dm.CLASS_NARROW if rho <= 12.0 else (
                dm.CLASS_WIDE if rho > 100.0 else dm.CLASS_FP32)
            assert cls[f] == want, (f, rho, cls[f])
        n16 += cls[f] == dm.CLASS_NARROW
        e = _rel(x[f, kept], orc.gs(A, bt, w.iterations))
        print(f"bin {f} ({w.freqs[f]:.0f} Hz) rho {rho:.1f} class {cls[f]}: {e:.2e}")
        assert e <= 1e-4, (f, e)
    assert 0 < n16 < w.n_bins


def test_bf16_policy_refine_all_equals_fp32(dm, dev):
    # With every sweep on the float system (R = I) a bf16 solve is the
    # float solve bitwise, whatever each bin's class.
    w = synth.compressed_fp32(n_bins=4, N=41, iterations=100)
    a, _, _, ca, _ = _solve(dm, dev, w, w.keep_count, prec=dm.PREC_BF16, refine=100)
    b, _, _, cb, _ = _solve(dm, dev, w, w.keep_count, prec=dm.PREC_FP32)
    assert np.array_equal(a, b)
