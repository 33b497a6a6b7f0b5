"""Sweeps of a streamed launch (A larger than 512 MiB, read with the
non-temporal hint), whose strip loads leave out the rows of the strip's own
tile and of the tile being updated and take their terms from on chip: the
same iterate, up to summation order, as the same bins solved in launches
that stay in cache (which read those rows in the strips as well).  The band
mixes long cooperative bins, wide and narrow, with bins of one, two and
three tiles (the own tile is left out only from three tiles on) and a bin
whose last strip reaches past its row stride; two small bins are checked
against the oracle too."""
import numpy as np
import pytest

from paper_1608_05179_amd import synth

pytestmark = pytest.mark.gpu

SMALL = [1, 2, 64, 65, 128, 129, 130, 257]
ITERS = 30
BIG, N_BIG = 2000, 36  # the FP32 band
# storage type: (precision, kept points of the long bins, their count, bins
# per cache-resident launch, tolerance of the summation order)
CASES = {
    "fp32": ("PREC_FP32", 2000, 36, 30, 1e-5),
    "bf16": ("PREC_BF16", 2000, 68, 34, 1e-5),
    "fp64": ("PREC_FP64", 1800, 21, 20, 1e-11),
}
ELEM = {"fp32": 4, "bf16": 2, "fp64": 8}


def _t(a, dtype, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype)


def _ld(k):
    return (k + 31) // 32 * 32


def _band(case):
    _, big, n_big, chunk, _ = CASES[case]
    w = synth.batched_fp32(n_bins=n_big + len(SMALL), N=61, iterations=ITERS)
    K = np.array([big] * n_big + SMALL, dtype=np.int32)
    es = ELEM[case]
    # A of the whole band: beyond the 512 MiB above which sweeps stream it
    assert sum(_ld(int(k)) ** 2 for k in K) * es > 512 * 1024 * 1024
    # each reference launch: below it
    assert (chunk * _ld(big) ** 2 + sum(_ld(k) ** 2 for k in SMALL)) * es < 512 * 1024 * 1024
    return w, K


@pytest.fixture(scope="module")
def band():
    return _band("fp32")


def _solve(dm, dev, w, K, bins, case="fp32"):
    import torch
    prec = getattr(dm, CASES[case][0])
    mic = _t(w.mic, torch.float64, dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    ctx = dm.Context(0)
    # bf16: every sweep on the bf16 system (no per-bin classes, no refinement)
    extra = ({"policy": dm.POLICY_FIXED, "refine_sweeps": 0} if case == "bf16" else {})
    x = ctx.solve(g, _t(w.freqs[bins], torch.float64, dev),
                  _t(w.csm[bins], torch.complex128, dev), select_mode=dm.SEL_KEEP_COUNT,
                  keep_count=[int(K[b]) for b in bins], iterations=ITERS,
                  precision=prec, batched=True, **extra)
    ctx.check()
    cls = ctx.classes(len(bins)) if case == "fp32" else None  # per-bin classes: FP32 policy
    out = x.double().cpu().numpy(), ctx.last_workgroups(), cls
    ctx.close()
    return out


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("case", list(CASES))
def test_streamed_band_equals_cache_resident_launches(dm, dev, case):
    w, K = _band(case)
    _, _, n_big, chunk, tol = CASES[case]
    allb = list(range(len(K)))
    xs, wg, cls = _solve(dm, dev, w, K, allb, case)
    assert wg > len(K)                      # cooperative job lists
    if case == "fp32":
        assert (cls == 2).any() and (cls == 0).any(), cls  # wide and narrow bins
    refs = [list(range(i, min(i + chunk, n_big))) for i in range(0, n_big, chunk)]
    refs.append(list(range(n_big, len(K))))
    worst = 0.0
    for bins in refs:
        xr, _, _ = _solve(dm, dev, w, K, bins, case)
        for i, b in enumerate(bins):
            e = _rel(xs[b], xr[i])
            worst = max(worst, e)
            assert e <= tol, (case, b, int(K[b]), e)
    print(f"{case}: streamed vs cache-resident launches: worst rel L2 {worst:.2e}")


def test_streamed_small_bins_match_oracle(dm, dev, orc, band):
    w, K = band
    xs, _, _ = _solve(dm, dev, w, K, list(range(len(K))))
    og = orc.Geometry(w.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    for b in (N_BIG + SMALL.index(65), N_BIG + SMALL.index(130)):
        ref = orc.solve_bin(og, w.freqs[b], w.csm[b], orc.SEL_KEEP_COUNT,
                            keep_count=int(K[b]), iters=ITERS)["x"]
        assert _rel(xs[b], ref) <= 1e-4, (b, int(K[b]))


def test_streamed_graph_replays_match_eager(dm, dev, band):
    # The streamed band captured into a graph (cooperative, non-temporal
    # strip loads, hand-over rows left out of the strips): every replay
    # equals the eager solve bitwise, with eager work between replays.
    import torch
    w, K = band
    mic = _t(w.mic, torch.float64, dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    freq = _t(w.freqs, torch.float64, dev)
    csm = torch.view_as_real(_t(w.csm, torch.complex128, dev)).contiguous()
    kw = dict(select_mode=dm.SEL_KEEP_COUNT, keep_count=[int(k) for k in K],
              iterations=ITERS, precision=dm.PREC_FP32)
    eager = dm.Context(0)
    ref = eager.solve(g, freq, csm, **kw).clone()
    eager.check()
    ctx = dm.Context(0)
    graph = ctx.capture(g, freq, csm, **kw)
    assert graph.workgroups() == eager.last_workgroups() > len(K)
    for _ in range(2):
        graph.x_map.fill_(-1.0)
        out = graph.launch()
        torch.cuda.synchronize()
        ctx.check()
        assert torch.equal(out, ref)
        eager.solve(g, freq, csm, **dict(kw, iterations=5))
        torch.cuda.synchronize()
    graph.close()
    ctx.close()
    eager.close()
