"""The server's batch former: requests on different arrays, grids and kept
counts, queued behind a running one, run as one batch (each request's map,
selection and system on its own grid, one sweep launch over all their
bins).  Each request's result equals its own solve to the summation order
(1e-5 in FP32; bitwise kept sets) and the oracle's iterate to 1e-4;
requests with other sweep settings are not merged."""
import numpy as np
import pytest

from paper_1608_05179_amd import synth

pytestmark = pytest.mark.gpu

ITERS = 100


def _t(a, dtype, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype)


def _direct(dm, dev, w, K, iters):
    import torch
    mic = _t(w.mic, torch.float64, dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    ctx = dm.Context(0)
    st = torch.zeros(w.n_bins, dtype=torch.int32, device=dev)
    x = ctx.solve(g, _t(w.freqs, torch.float64, dev), _t(w.csm, torch.complex128, dev),
                  select_mode=dm.SEL_KEEP_COUNT, keep_count=K, iterations=iters, s_tilde=st)
    ctx.check()
    out = x.cpu().numpy(), st.cpu().numpy()
    ctx.close()
    return out


def _requests():
    a = synth.compressed_fp32(n_bins=3, N=21, iterations=ITERS)
    b = synth.compressed_fp32(n_bins=5, N=41, iterations=ITERS)
    c = synth.batched_fp32(n_bins=4, N=33, iterations=ITERS, kmin=100, kmax=600)
    d = synth.precision_bf16(n_bins=2, N=25, iterations=ITERS)
    return [(a, [a.keep_count] * 3), (b, [90, 200, 337, 500, 60]),
            (c, [int(k) for k in c.keep_counts]), (d, [d.S, d.S])]


def _submit(srv, dm, w, K, iters):
    return srv.submit(w.mic, w.N, (w.x0, w.x1, w.y0, w.y1), w.z0, w.freqs, w.csm,
                      select_mode=dm.SEL_KEEP_COUNT, keep_count=K, iterations=iters,
                      precision=dm.PREC_FP32)


def _blocker(srv, dm):
    # a long request the single worker starts at once, so the others queue
    w = synth.compressed_fp32(n_bins=8, N=61, iterations=3000)
    return _submit(srv, dm, w, [3000] * 8, 3000)


def test_batch_former_merges_different_grids(orc, dm, dev):
    reqs = _requests()
    want = [_direct(dm, dev, w, K, ITERS) for w, K in reqs]
    srv = dm.Server(hbm_budget=16 << 30, cache_budget=0, slots=1, max_batch=8)
    tb = _blocker(srv, dm)
    tickets = [_submit(srv, dm, w, K, ITERS) for w, K in reqs]
    srv.wait(tb)
    outs = [srv.wait(t) for t in tickets]
    s = srv.stats()
    assert s["merged"] == len(reqs) and s["batches"] == 2, s
    for (x, st, info), (xr, str_), (w, K) in zip(outs, want, reqs):
        assert info["status"] == 0
        assert np.array_equal(st, str_)
        e = np.linalg.norm(x.astype(np.float64) - xr) / np.linalg.norm(xr)
        assert e <= 1e-5, e
    # the oracle on one bin of each request
    for (x, st, _), (w, K) in zip(outs, reqs):
        og = orc.Geometry(w.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
        f = w.n_bins - 1
        ref = orc.solve_bin(og, w.freqs[f], w.csm[f], orc.SEL_KEEP_COUNT, keep_count=K[f],
                            iters=ITERS)
        e = np.linalg.norm(x[f].astype(np.float64) - ref["x"]) / np.linalg.norm(ref["x"])
        assert e <= 1e-4, (w.N, f, e)
    srv.close()


def test_batch_former_keeps_incompatible_requests_apart(dm, dev):
    reqs = _requests()[:2]
    srv = dm.Server(hbm_budget=16 << 30, cache_budget=0, slots=1, max_batch=8)
    tb = _blocker(srv, dm)
    (wa, Ka), (wb, Kb) = reqs
    t1 = _submit(srv, dm, wa, Ka, ITERS)
    t2 = _submit(srv, dm, wb, Kb, ITERS + 20)  # other sweep count: not merged
    srv.wait(tb)
    x1, _, i1 = srv.wait(t1)
    x2, _, i2 = srv.wait(t2)
    assert i1["status"] == 0 and i2["status"] == 0
    s = srv.stats()
    assert s["merged"] == 0 and s["batches"] == 3, s
    xr, _ = _direct(dm, dev, wa, Ka, ITERS)
    assert np.array_equal(x1, xr)
    srv.close()
