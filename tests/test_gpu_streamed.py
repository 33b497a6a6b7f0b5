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

BIG, N_BIG = 2000, 36
SMALL = [1, 2, 64, 65, 128, 129, 130, 257]
ITERS = 30


def _t(a, dtype, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype)


def _ld(k):
    return (k + 31) // 32 * 32


@pytest.fixture(scope="module")
def band():
    w = synth.batched_fp32(n_bins=N_BIG + len(SMALL), N=61, iterations=ITERS)
    K = np.array([BIG] * N_BIG + SMALL, dtype=np.int32)
    # A of the whole band: beyond the 512 MiB above which sweeps stream it
    assert sum(_ld(int(k)) ** 2 for k in K) * 4 > 512 * 1024 * 1024
    # each reference launch: below it
    assert 30 * _ld(BIG) ** 2 * 4 < 512 * 1024 * 1024
    return w, K


def _solve(dm, dev, w, K, bins):
    import torch
    mic = _t(w.mic, torch.float64, dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    ctx = dm.Context(0)
    x = ctx.solve(g, _t(w.freqs[bins], torch.float64, dev),
                  _t(w.csm[bins], torch.complex128, dev), select_mode=dm.SEL_KEEP_COUNT,
                  keep_count=[int(K[b]) for b in bins], iterations=ITERS,
                  precision=dm.PREC_FP32, batched=True)
    ctx.check()
    out = x.double().cpu().numpy(), ctx.last_workgroups(), ctx.classes(len(bins))
    ctx.close()
    return out


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_streamed_band_equals_cache_resident_launches(dm, dev, band):
    w, K = band
    allb = list(range(len(K)))
    xs, wg, cls = _solve(dm, dev, w, K, allb)
    assert wg > len(K)                      # cooperative job lists
    assert (cls == 2).any() and (cls == 0).any(), cls  # wide and narrow bins
    refs = [list(range(0, 30)), list(range(30, N_BIG)), list(range(N_BIG, len(K)))]
    worst = 0.0
    for bins in refs:
        xr, _, _ = _solve(dm, dev, w, K, bins)
        for i, b in enumerate(bins):
            e = _rel(xs[b], xr[i])
            worst = max(worst, e)
            assert e <= 1e-5, (b, int(K[b]), e)
    print(f"streamed vs cache-resident launches: worst rel L2 {worst:.2e}")


def test_streamed_small_bins_match_oracle(dm, dev, orc, band):
    w, K = band
    xs, _, _ = _solve(dm, dev, w, K, list(range(len(K))))
    og = orc.Geometry(w.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    for b in (N_BIG + SMALL.index(65), N_BIG + SMALL.index(130)):
        ref = orc.solve_bin(og, w.freqs[b], w.csm[b], orc.SEL_KEEP_COUNT,
                            keep_count=int(K[b]), iters=ITERS)["x"]
        assert _rel(xs[b], ref) <= 1e-4, (b, int(K[b]))
