"""damas_solve_static, the whole-path solve that allocates nothing (its
workspace is a static device array per GPU), called through the C ABI: it
equals damas_solve_dev's batched one-workgroup-per-bin solve bitwise on two
calls in a row, the second smaller than the first, and a workspace beyond
the array is refused on the host."""
import ctypes

import numpy as np
import pytest

from paper_1608_05179_amd import synth

pytestmark = pytest.mark.gpu


def _inputs(dm, dev, w):
    import torch
    mic = torch.as_tensor(w.mic, dtype=torch.float64).to(dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    freq = torch.as_tensor(w.freqs, dtype=torch.float64).to(dev)
    csm = torch.as_tensor(w.csm, dtype=torch.complex128).to(dev)
    return mic, g, freq, csm


def _ctx_solve(dm, dev, w, K, iters, policy):
    import torch
    mic, g, freq, csm = _inputs(dm, dev, w)
    ctx = dm.Context(0)
    ctx.set_coop(0)  # one workgroup per bin, as the static solve
    st = torch.zeros(w.n_bins, dtype=torch.int32, device=dev)
    idx = torch.zeros(w.n_bins, w.S, dtype=torch.int32, device=dev)
    x = ctx.solve(g, freq, csm, select_mode=dm.SEL_KEEP_COUNT, keep_count=K,
                  iterations=iters, precision=dm.PREC_FP32, idx=idx, s_tilde=st,
                  policy=policy)
    ctx.check()
    out = x.cpu().numpy(), st.cpu().numpy(), idx.cpu().numpy()
    ctx.close()
    return out


def _static_solve(dm, dev, w, K, iters, policy):
    import torch
    mic, g, freq, csm = _inputs(dm, dev, w)
    kc = torch.as_tensor(np.asarray(K, dtype=np.int32)).to(dev)
    st = torch.zeros(w.n_bins, dtype=torch.int32, device=dev)
    idx = torch.zeros(w.n_bins, w.S, dtype=torch.int32, device=dev)
    x = torch.full((w.n_bins, w.S), float("nan"), dtype=torch.float32, device=dev)
    # the C ABI directly, with the device keep counts
    p, _ = dm._params(w.n_bins, dm.SEL_KEEP_COUNT, 0.0, None, iters, dm.PREC_FP32, True,
                      int(max(K)), 0, 0, policy)
    rc = dm._lib.damas_solve_static(ctypes.byref(g), w.n_bins, freq.data_ptr(),
                                    torch.view_as_real(csm).contiguous().data_ptr(),
                                    ctypes.byref(p), kc.data_ptr(), None, x.data_ptr(), None,
                                    idx.data_ptr(), st.data_ptr(),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == dm.OK, dm.last_error()
    dm.check(None)
    return x.cpu().numpy(), st.cpu().numpy(), idx.cpu().numpy()


@pytest.mark.parametrize("policy", ["auto", "fixed"])
def test_static_solve_equals_context_solve_twice(dm, dev, policy):
    pol = dm.POLICY_AUTO if policy == "auto" else dm.POLICY_FIXED
    # first call: 4 bins of the 61 x 61 grid (1 to 8 kHz) with uneven kept
    # counts, about 70 MB of workspace (the 1 kHz bin is widened under the
    # policy); second: 3 bins of the 21 x 21 grid
    big = synth.compressed_fp32(n_bins=4, N=61, iterations=150)
    Kb = [1600, 900, 1500, 120]
    small = synth.compressed_fp32(n_bins=3, N=21, iterations=80)
    Ks = [60, 100, 441]
    for w, K, it in ((big, Kb, 150), (small, Ks, 80)):
        xs, sts, ixs = _static_solve(dm, dev, w, K, it, pol)
        xc, stc, ixc = _ctx_solve(dm, dev, w, K, it, pol)
        assert np.array_equal(sts, stc) and np.array_equal(ixs, ixc)
        assert np.isfinite(xs).all()
        assert np.array_equal(xs, xc), (w.name, float(np.abs(xs - xc).max()))


def test_static_solve_refuses_a_workspace_beyond_the_array(dm, dev):
    import torch
    w = synth.batched_fp32(n_bins=8, iterations=2)
    mic, g, freq, csm = _inputs(dm, dev, w)
    kc = torch.full((w.n_bins,), 4000, dtype=torch.int32, device=dev)
    x = torch.zeros(w.n_bins, w.S, dtype=torch.float32, device=dev)
    with pytest.raises(dm.DamasError) as ei:
        dm.solve_static(g, freq, csm, select_mode=dm.SEL_KEEP_COUNT, keep_count=kc,
                        max_kept=4000, iterations=2, x_map=x)
    assert ei.value.code == dm.EINVAL and "workspace" in str(ei.value)
    assert dm.static_scratch_bytes() == 96 << 20
