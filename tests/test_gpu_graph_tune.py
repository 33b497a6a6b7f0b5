"""Graph capture and the schedule autotuner.

A captured solve replays bitwise like the eager solve it captured (one
workgroup per bin, or the cooperative schedule of a batched band), on every
replay, with eager work and synchronisations
in between; a CSM changed in place gives the eager solve of the new CSM.
The autotuner's choice stays on the context and its solves still match the
oracle."""
import numpy as np
import pytest

from paper_1608_05179_amd import synth

pytestmark = pytest.mark.gpu


def _t(a, dtype, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype)


def _setup(dm, dev, w):
    import torch
    mic = _t(w.mic, torch.float64, dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    freq = _t(w.freqs, torch.float64, dev)
    csm = torch.view_as_real(torch.tensor(w.csm, dtype=torch.complex128)).contiguous().to(dev)
    return mic, g, freq, csm


def test_graph_replays_match_eager(dm, dev):
    import torch
    w = synth.compressed_fp32(n_bins=6, N=41, iterations=150)
    mic, g, freq, csm = _setup(dm, dev, w)
    eager_ctx = dm.Context(0)
    eager_ctx.set_coop(0)
    ref = eager_ctx.solve(g, freq, csm, select_mode=dm.SEL_KEEP_COUNT,
                          keep_count=w.keep_count, iterations=w.iterations).clone()
    ctx = dm.Context(0)
    graph = ctx.capture(g, freq, csm, select_mode=dm.SEL_KEEP_COUNT, keep_count=w.keep_count,
                        iterations=w.iterations)
    for _ in range(4):
        graph.x_map.fill_(-1.0)
        out = graph.launch()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        # eager work between replays
        eager_ctx.solve(g, freq, csm, select_mode=dm.SEL_KEEP_COUNT, keep_count=w.keep_count,
                        iterations=20)
        torch.cuda.synchronize()
    # a new CSM in place: the replay is the eager solve of the new CSM
    w2 = synth.compressed_fp32(n_bins=6, N=41, iterations=150)
    w2.csm = w2.csm[::-1].copy()
    csm.copy_(torch.view_as_real(torch.tensor(w2.csm, dtype=torch.complex128)))
    ref2 = eager_ctx.solve(g, freq, csm, select_mode=dm.SEL_KEEP_COUNT,
                           keep_count=w.keep_count, iterations=w.iterations).clone()
    out = graph.launch()
    torch.cuda.synchronize()
    assert torch.equal(out, ref2) and not torch.equal(ref, ref2)
    # the workspace is pinned while the graph exists
    with pytest.raises(dm.DamasError) as ei:
        big = synth.compressed_fp32(n_bins=6, N=61, iterations=5)
        m2, g2, f2, c2 = _setup(dm, dev, big)
        ctx.solve(g2, f2, c2, select_mode=dm.SEL_KEEP_COUNT, keep_count=2000, iterations=5)
    assert ei.value.code == dm.EBUSY
    graph.close()
    ctx.close()
    eager_ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_graph_cooperative_replays_match_eager(dm, dev, prec):
    # Uneven kept counts: the long bins get helper workgroups, so the graph
    # holds the cooperative sweep launches (one for FP32; bf16 bulk and FP32
    # refinement for BF16).  Every replay equals, bitwise, the eager solve
    # of a context that plans the same schedule, with eager work and
    # synchronisations between replays; the power output is captured too.
    import torch
    if prec == "fp32":
        w = synth.compressed_fp32(n_bins=4, N=61, iterations=120)
        kw = dict(select_mode=dm.SEL_KEEP_COUNT, keep_count=[2400, 700, 3600, 150],
                  iterations=w.iterations, precision=dm.PREC_FP32)
    else:
        w = synth.precision_bf16(n_bins=3, N=61, iterations=120)
        kw = dict(select_mode=dm.SEL_KEEP_ALL, iterations=w.iterations,
                  precision=dm.PREC_BF16, refine_sweeps=30)
    mic, g, freq, csm = _setup(dm, dev, w)
    eager = dm.Context(0)
    p_ref = torch.zeros(w.n_bins, dtype=torch.float64, device=dev)
    ref = eager.solve(g, freq, csm, power=p_ref, **kw).clone()
    eager.check()
    assert eager.last_workgroups() > w.n_bins
    ctx = dm.Context(0)
    p_out = torch.zeros(w.n_bins, dtype=torch.float64, device=dev)
    graph = ctx.capture(g, freq, csm, power=p_out, **kw)
    assert graph.workgroups() == eager.last_workgroups()
    for _ in range(3):
        graph.x_map.fill_(-1.0)
        p_out.fill_(-1.0)
        out = graph.launch()
        torch.cuda.synchronize()
        ctx.check()
        assert torch.equal(out, ref)
        assert torch.equal(p_out, p_ref)
        eager.solve(g, freq, csm, **dict(kw, iterations=40))
        torch.cuda.synchronize()
    graph.close()
    ctx.close()
    eager.close()


def test_autotune_keeps_a_valid_choice(orc, dm, dev):
    w = synth.compressed_fp32(n_bins=4, N=61, iterations=120)
    Ks = [2400, 700, 3600, 150]
    mic, g, freq, csm = _setup(dm, dev, w)
    ctx = dm.Context(0)
    r = ctx.autotune(g, freq, csm, select_mode=dm.SEL_KEEP_COUNT, keep_count=Ks,
                     trial_sweeps=10)
    assert r["candidates_timed"] >= 2
    assert 0 < r["best_ms_per_sweep"] <= r["default_ms_per_sweep"]
    x = ctx.solve(g, freq, csm, select_mode=dm.SEL_KEEP_COUNT, keep_count=Ks,
                  iterations=w.iterations)
    ctx.check()
    x = x.double().cpu().numpy()
    og = orc.Geometry(w.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    for f in (0, 2):
        ref = orc.solve_bin(og, w.freqs[f], w.csm[f], orc.SEL_KEEP_COUNT, keep_count=Ks[f],
                            iters=w.iterations)
        err = np.linalg.norm(x[f] - ref["x"]) / np.linalg.norm(ref["x"])
        assert err <= 1e-4, (f, err)
    ctx.close()


def test_set_schedule_applies_knobs(dm, dev):
    # Knobs applied without trials give the schedule they describe: the
    # defaults reproduce an untuned context bitwise, and knobs that rank no
    # bin give one workgroup per bin (plain sweeps), equal to coop = 0.
    import torch
    w = synth.compressed_fp32(n_bins=4, N=61, iterations=60)
    Ks = [2400, 700, 3600, 150]
    mic, g, freq, csm = _setup(dm, dev, w)
    kw = dict(select_mode=dm.SEL_KEEP_COUNT, keep_count=Ks, iterations=w.iterations)
    a = dm.Context(0)
    xa = a.solve(g, freq, csm, **kw).clone()
    b = dm.Context(0)
    b.set_schedule()
    xb = b.solve(g, freq, csm, **kw).clone()
    assert torch.equal(xa, xb) and a.last_workgroups() == b.last_workgroups()
    b.set_schedule(coop=0)
    xc = b.solve(g, freq, csm, **kw)
    assert b.last_workgroups() == w.n_bins
    c = dm.Context(0)
    c.set_coop(0)
    xd = c.solve(g, freq, csm, **kw)
    a.check(), b.check(), c.check()
    assert torch.equal(xc, xd)
    with pytest.raises(dm.DamasError) as ei:
        b.set_schedule(coop_split=0.0)
    assert ei.value.code == dm.EINVAL
    for ctx in (a, b, c):
        ctx.close()
