"""KEEP_FRAC: the KEEP_COUNT rule with ceil(p N^2) points in every bin.

On the compressed workload's grid (41 x 41) p = 0.1, 0.2, 0.3 keep 169, 337
and 505 points.  A KEEP_FRAC solve equals the KEEP_COUNT solve of that
count bitwise (context, allocation-free and server paths), and its kept
sets and maps match the oracle's selection and sweeps for that count."""
import math

import numpy as np
import pytest

from paper_1608_05179_amd import synth

pytestmark = pytest.mark.gpu


def _t(a, dtype, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dtype)


@pytest.mark.parametrize("p", [0.1, 0.2, 0.3])
def test_keep_frac_matches_keep_count_and_oracle(orc, dm, dev, p):
    import torch
    w = synth.compressed_fp32(n_bins=3, N=41, iterations=120)
    K = math.ceil(p * w.S)
    mic = _t(w.mic, torch.float64, dev)
    g = dm.geometry(mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    freq = _t(w.freqs, torch.float64, dev)
    csm = _t(w.csm, torch.complex128, dev)
    ctx = dm.Context(0)
    runs = []
    for kw in (dict(select_mode=dm.SEL_KEEP_FRAC, keep_frac=p),
               dict(select_mode=dm.SEL_KEEP_COUNT, keep_count=K)):
        st = torch.zeros(w.n_bins, dtype=torch.int32, device=dev)
        idx = torch.zeros(w.n_bins, w.S, dtype=torch.int32, device=dev)
        x = ctx.solve(g, freq, csm, iterations=w.iterations, s_tilde=st, idx=idx, **kw)
        ctx.check()
        runs.append((x.clone(), st.clone(), idx.clone()))
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][2], runs[1][2])
    st = runs[0][1].cpu().numpy()
    assert (st == K).all()
    # the allocation-free path, counts formed on the host
    st2 = torch.zeros(w.n_bins, dtype=torch.int32, device=dev)
    xs = dm.solve_static(g, freq, csm, select_mode=dm.SEL_KEEP_FRAC, keep_frac=p,
                         iterations=w.iterations, s_tilde=st2)
    dm.check(None)
    assert torch.equal(st2, runs[0][1])
    x = runs[0][0].double().cpu().numpy()
    assert np.linalg.norm(xs.double().cpu().numpy() - x) <= 1e-5 * np.linalg.norm(x)
    idx = runs[0][2].cpu().numpy()
    og = orc.Geometry(w.mic, w.N, w.x0, w.x1, w.y0, w.y1, w.z0, w.c)
    for f in range(w.n_bins):
        ref = orc.solve_bin(og, w.freqs[f], w.csm[f], orc.SEL_KEEP_COUNT, keep_count=K,
                            iters=w.iterations)
        if ref["margin"] > 1e-12:
            assert np.array_equal(idx[f, :K], ref["idx"]), f
        err = np.linalg.norm(x[f] - ref["x"]) / np.linalg.norm(ref["x"])
        assert err <= 1e-4, (f, err)
    ctx.close()


def test_keep_frac_server(dm, dev):
    w = synth.compressed_fp32(n_bins=2, N=41, iterations=80)
    K = math.ceil(0.2 * w.S)
    srv = dm.Server(slots=1)
    out = []
    for kw in (dict(select_mode=dm.SEL_KEEP_FRAC, keep_frac=0.2),
               dict(select_mode=dm.SEL_KEEP_COUNT, keep_count=K)):
        t = srv.submit(w.mic, w.N, (w.x0, w.x1, w.y0, w.y1), w.z0, w.freqs, w.csm,
                       iterations=w.iterations, **kw)
        out.append(srv.wait(t))
    srv.close()
    (xa, sa, _), (xb, sb, _) = out[0], out[1]
    assert (sa == K).all() and np.array_equal(sa, sb) and np.array_equal(xa, xb)
