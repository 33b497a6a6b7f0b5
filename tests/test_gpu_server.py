"""The request server: results equal the context's batched solve bitwise,
repeated scenes hit the PSF cache with identical results, requests that can
never fit are refused (DAMAS_EADMIT), a full queue refuses (DAMAS_EBUSY),
and a budget that fits one request at a time still completes every request
correctly."""
import numpy as np
import pytest

from paper_1608_05179_amd import synth

pytestmark = pytest.mark.gpu


def _t(a, dtype, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype)


def _direct(dm, dev, w, K, iters, prec=None):
    import torch
    prec = dm.PREC_FP32 if prec is None else prec
    mic = _t(w.mic, torch.float64, dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    ctx = dm.Context(0)
    x = ctx.solve(g, _t(w.freqs, torch.float64, dev), _t(w.csm, torch.complex128, dev),
                  select_mode=dm.SEL_KEEP_COUNT, keep_count=K, iterations=iters,
                  precision=prec)
    ctx.check()
    out = x.cpu().numpy()
    ctx.close()
    return out


def _submit(srv, dm, w, K, iters, prec=None):
    return srv.submit(w.mic, w.N, (w.x0, w.x1, w.y0, w.y1), w.z0, w.freqs, w.csm,
                      select_mode=dm.SEL_KEEP_COUNT, keep_count=K, iterations=iters,
                      precision=dm.PREC_FP32 if prec is None else prec)


def _requests():
    a = synth.compressed_fp32(n_bins=3, N=21, iterations=80)
    b = synth.compressed_fp32(n_bins=5, N=41, iterations=120)
    c = synth.batched_fp32(n_bins=4, N=33, iterations=60, kmin=100, kmax=600)
    return [(a, a.keep_count, 80), (b, [90, 200, 337, 500, 60], 120),
            (c, [int(k) for k in c.keep_counts], 60)]


def test_server_results_equal_direct_solves(dm, dev):
    reqs = _requests()
    want = [_direct(dm, dev, w, K, it) for w, K, it in reqs]
    srv = dm.Server(hbm_budget=8 << 30, cache_budget=1 << 30, slots=2)
    tickets = [_submit(srv, dm, w, K, it) for w, K, it in reqs]
    for t, ref, (w, K, _) in zip(tickets, want, reqs):
        x, st, info = srv.wait(t)
        assert info["status"] == 0 and not info["cache_hit"]
        assert np.array_equal(x, ref)
        kk = np.minimum(np.maximum(np.asarray(K if not isinstance(K, int) else [K] * w.n_bins),
                                   dm.coarse_count(w.N)), w.S)
        assert np.array_equal(st, kk)
        assert info["total_ms"] >= info["run_ms"] > 0
    s = srv.stats()
    assert s["submitted"] == 3 and s["completed"] == 3 and s["queued"] == 0
    srv.close()


def test_server_cache_hit_is_identical(dm, dev):
    w, K, it = _requests()[1]
    srv = dm.Server(hbm_budget=8 << 30, cache_budget=1 << 30, slots=1)
    x1, _, i1 = srv.wait(_submit(srv, dm, w, K, it))
    x2, _, i2 = srv.wait(_submit(srv, dm, w, K, it))
    assert not i1["cache_hit"] and i2["cache_hit"]
    assert np.array_equal(x1, x2)
    # another scene (other bins) misses
    w2 = synth.compressed_fp32(n_bins=5, N=41, iterations=120)
    w2.freqs, w2.csm = w2.freqs[::-1].copy(), w2.csm[::-1].copy()
    _, _, i3 = srv.wait(_submit(srv, dm, w2, K, it))
    assert not i3["cache_hit"]
    s = srv.stats()
    assert s["cache_hits"] == 1 and s["cache_misses"] == 2 and s["cache_bytes"] > 0
    srv.close()


def test_server_refuses_what_never_fits(dm, dev):
    w, K, it = _requests()[1]
    need = dm.query_footprint(w.M, w.N, w.n_bins, select_mode=dm.SEL_KEEP_COUNT,
                              keep_count=K, iterations=it)
    srv = dm.Server(hbm_budget=need - 1, cache_budget=0, slots=1)
    with pytest.raises(dm.DamasError) as ei:
        _submit(srv, dm, w, K, it)
    assert ei.value.code == dm.EADMIT
    assert srv.stats()["rejected"] == 1
    srv.close()


def test_server_full_queue_is_busy(dm, dev):
    w = synth.compressed_fp32(n_bins=8, N=41, iterations=3000)
    srv = dm.Server(hbm_budget=8 << 30, cache_budget=0, slots=1, max_queue=1)
    first = _submit(srv, dm, w, w.keep_count, 3000)
    codes = []
    tickets = []
    for _ in range(3):
        try:
            tickets.append(_submit(srv, dm, w, w.keep_count, 3000))
        except dm.DamasError as e:
            codes.append(e.code)
    assert codes and all(c == dm.EBUSY for c in codes)
    for t in [first] + tickets:
        srv.wait(t)
    srv.close()


def test_server_tight_budget_runs_one_at_a_time(dm, dev):
    reqs = _requests()
    want = [_direct(dm, dev, w, K, it) for w, K, it in reqs]
    fps = [dm.query_footprint(w.M, w.N, w.n_bins, select_mode=dm.SEL_KEEP_COUNT,
                              keep_count=K, iterations=it) for w, K, it in reqs]
    srv = dm.Server(hbm_budget=max(fps) + (1 << 20), cache_budget=0, slots=3)
    tickets = [_submit(srv, dm, w, K, it) for w, K, it in reqs]
    for t, ref in zip(tickets, want):
        x, _, info = srv.wait(t)
        assert np.array_equal(x, ref)
    assert srv.stats()["held_bytes"] <= max(fps) + (1 << 20)
    srv.close()


def test_server_poll_and_timeout(dm, dev):
    w = synth.compressed_fp32(n_bins=16, N=41, iterations=4000)
    srv = dm.Server(hbm_budget=8 << 30, cache_budget=0, slots=1)
    t = _submit(srv, dm, w, w.keep_count, 4000)
    with pytest.raises(dm.DamasError) as ei:
        srv.wait(t, timeout_ms=0)
    assert ei.value.code == dm.ETIMEDOUT
    x, _, info = srv.wait(t)
    assert info["status"] == 0 and np.isfinite(x).all()
    with pytest.raises(dm.DamasError):
        srv.poll(t)  # retired
    srv.close()


def _submit_eps(srv, dm, w, eps, max_kept, iters):
    return srv.submit(w.mic, w.N, (w.x0, w.x1, w.y0, w.y1), w.z0, w.freqs, w.csm,
                      select_mode=dm.SEL_EPS_REL, eps=eps, max_kept=max_kept,
                      iterations=iters, precision=dm.PREC_FP32)


def _direct_eps(dm, dev, w, eps, max_kept, iters):
    import torch
    mic = _t(w.mic, torch.float64, dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    ctx = dm.Context(0)
    x = ctx.solve(g, _t(w.freqs, torch.float64, dev), _t(w.csm, torch.complex128, dev),
                  select_mode=dm.SEL_EPS_REL, eps=eps, max_kept=max_kept, iterations=iters,
                  precision=dm.PREC_FP32)
    ctx.check()
    out = x.cpu().numpy()
    ctx.close()
    return out


def test_server_fault_is_charged_to_its_own_request(dm, dev):
    # Two slots run at once: one request keeps more points than its
    # max_kept (a device-side capacity fault of its own context), the other
    # is a long ordinary solve.  Only the faulting request fails, and the
    # slot that ran it serves the next request cleanly.
    good, K, it = _requests()[1]
    want = _direct(dm, dev, good, K, 600)
    bad = synth.compressed_fp32(n_bins=2, N=21, iterations=50)
    srv = dm.Server(hbm_budget=8 << 30, cache_budget=0, slots=2)
    t_good = _submit(srv, dm, good, K, 600)
    t_bad = _submit_eps(srv, dm, bad, 0.0, 50, 50)  # eps = 0 keeps all 441 points
    with pytest.raises(dm.DamasError) as ei:
        srv.wait(t_bad)
    assert ei.value.code == dm.ECAPACITY
    x, _, info = srv.wait(t_good)
    assert info["status"] == 0 and np.array_equal(x, want)
    w3, K3, it3 = _requests()[0]
    want3 = _direct(dm, dev, w3, K3, it3)
    x3, _, info3 = srv.wait(_submit(srv, dm, w3, K3, it3))
    assert info3["status"] == 0 and np.array_equal(x3, want3)
    srv.close()


def test_server_cache_hit_under_eps_rel_with_a_larger_max_kept(dm, dev):
    # The same scene under EPS_REL with two arena bounds: the second request
    # hits the cache (same kept sets) and copies exactly the packed systems
    # of those kept counts, whatever its max_kept sizes the arena to.
    w = synth.compressed_fp32(n_bins=4, N=41, iterations=100)
    srv = dm.Server(hbm_budget=8 << 30, cache_budget=1 << 30, slots=1)
    x1, st1, i1 = srv.wait(_submit_eps(srv, dm, w, 0.05, 900, 100))
    x2, st2, i2 = srv.wait(_submit_eps(srv, dm, w, 0.05, w.S, 100))
    assert not i1["cache_hit"] and i2["cache_hit"]
    assert np.array_equal(st1, st2) and st1.max() <= 900
    assert np.array_equal(x1, x2)
    assert np.array_equal(x2, _direct_eps(dm, dev, w, 0.05, w.S, 100))
    srv.close()
