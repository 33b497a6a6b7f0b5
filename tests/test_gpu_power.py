"""Integrated power per bin (the paper's Table 1 quantity P = sum_n x_n),
an optional output of the solves: against the oracle's sum of its iterate
(1e-12 in FP64, 1e-4 in FP32), equal to the sum of the returned map up to
the map's float rounding, the same from the one-workgroup, cooperative and
plain launches, and through the host-pointer solve."""
import numpy as np
import pytest

from paper_1608_05179_amd import synth

pytestmark = pytest.mark.gpu


def _t(a, dtype, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype)


def _solve(dm, dev, w, K, prec, coop=-1, batched=True):
    import torch
    mic = _t(w.mic, torch.float64, dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    ctx = dm.Context(0)
    ctx.set_coop(coop)
    pw = torch.full((w.n_bins,), float("nan"), dtype=torch.float64, device=dev)
    x = ctx.solve(g, _t(w.freqs, torch.float64, dev), _t(w.csm, torch.complex128, dev),
                  select_mode=dm.SEL_KEEP_COUNT, keep_count=K, iterations=w.iterations,
                  precision=prec, batched=batched, power=pw)
    ctx.check()
    wg = ctx.last_workgroups()
    out = x.double().cpu().numpy(), pw.cpu().numpy(), wg
    ctx.close()
    return out


def _oracle_power(orc, w, K):
    og = orc.Geometry(w.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    return np.array([orc.solve_bin(og, w.freqs[f], w.csm[f], orc.SEL_KEEP_COUNT,
                                   keep_count=K[f], iters=w.iterations)["x"].sum()
                     for f in range(w.n_bins)])


def test_power_fp64(orc, dm, dev):
    w = synth.compressed_fp32(n_bins=3, N=21, iterations=200)
    K = [120, 200, 441]
    x, pw, _ = _solve(dm, dev, w, K, dm.PREC_FP64)
    ref = _oracle_power(orc, w, K)
    assert np.allclose(pw, ref, rtol=1e-12, atol=0)
    assert np.allclose(pw, x.sum(axis=1), rtol=1e-13, atol=0)


@pytest.mark.parametrize("coop", [0, -1])
def test_power_fp32(orc, dm, dev, coop):
    w = synth.compressed_fp32(n_bins=3, N=61, iterations=150)
    K = [2600, 400, 1700]
    x, pw, wg = _solve(dm, dev, w, K, dm.PREC_FP32, coop=coop)
    if coop == -1:
        assert wg > w.n_bins
    ref = _oracle_power(orc, w, K)
    assert np.allclose(pw, ref, rtol=1e-4, atol=0)
    # the map is float: its sum moves by its rounding
    assert np.allclose(pw, x.sum(axis=1), rtol=1e-6, atol=0)


def test_power_plain_equals_batched(dm, dev):
    w = synth.compressed_fp32(n_bins=4, N=41, iterations=100)
    K = [300, 337, 120, 600]
    _, pb, _ = _solve(dm, dev, w, K, dm.PREC_FP32, coop=0)
    _, pp, _ = _solve(dm, dev, w, K, dm.PREC_FP32, batched=False)
    assert np.array_equal(pb, pp)


def test_power_through_the_host_solve(dm, dev):
    import ctypes
    w = synth.compressed_fp32(n_bins=2, N=21, iterations=60)
    ctx = dm.Context(0)
    ctx.set_coop(0)
    mic = np.ascontiguousarray(w.mic)
    g = dm.Geometry(w.M, mic.ctypes.data, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    freq = np.ascontiguousarray(w.freqs)
    csm = np.ascontiguousarray(w.csm.view(np.float64))
    p, _ = dm._params(w.n_bins, dm.SEL_KEEP_COUNT, 0.0, 200, 60, dm.PREC_FP32, True, 0, 0)
    pw = np.full(w.n_bins, np.nan)
    p.power = pw.ctypes.data
    x = np.zeros((w.n_bins, w.S), np.float32)
    fn = dm._lib.damas_solve
    fn.argtypes = [ctypes.c_void_p, ctypes.POINTER(dm.Geometry), ctypes.c_int32,
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(dm.Params),
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                   ctypes.c_void_p]
    fn.restype = ctypes.c_int
    rc = fn(ctx._h, ctypes.byref(g), w.n_bins, freq.ctypes.data, csm.ctypes.data,
            ctypes.byref(p), None, x.ctypes.data, None, None, None)
    assert rc == dm.OK, dm.last_error()
    assert np.isfinite(pw).all()
    assert np.allclose(pw, x.astype(np.float64).sum(axis=1), rtol=1e-6)
    ctx.close()
