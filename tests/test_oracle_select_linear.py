"""Pins of Algorithm 1 with the linear interpolating predictor (a point of
level l predicted by the mean of its two or four neighbours on G^(l-1))
against closed forms: bilinear fields are predicted exactly, and a spike
on a coarse point spreads 1/2 to its axis neighbours and 1/4 to its
diagonal neighbours at every finer spacing (predictions read the original
samples of the coarser grids, which include the spike).
"""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _bilinear(N):
    iy, ix = np.divmod(np.arange(N * N), N)
    return 3.0 + 2.0 * ix + 5.0 * iy + 0.5 * ix * iy  # increasing in both axes


def _uses_mirror(orc, N, p):
    ix, iy = p % N, p // N
    lv, _, _ = orc.level(N, ix, iy)
    if lv == 0:
        return False
    J = int(np.floor(np.log2(N)))
    h = 1 << (J - lv)
    return bool((ix % (2 * h) and ix + h > N - 1) or (iy % (2 * h) and iy + h > N - 1))


def test_bilinear_field_has_no_detail_where_the_stencil_fits(orc):
    for N in (17, 33):  # 2^J + 1: every stencil fits
        b = _bilinear(N)
        idx, det, _ = orc.select(N, b, orc.SEL_EPS_REL, eps=1e-12,
                                 predictor=orc.PRED_LINEAR)
        assert (det == 0).all(), N
        coarse = [p for p in range(N * N) if orc.level(N, p % N, p // N)[0] == 0]
        assert list(idx) == coarse
        # the order-0 predictor sees the slope everywhere
        _, det0, _ = orc.select(N, b, orc.SEL_EPS_REL, eps=1e-12)
        assert (det0 > 0).sum() == N * N - len(coarse)
    for N in (21, 41):  # mirrored neighbours at the far edges
        b = _bilinear(N)
        _, det, _ = orc.select(N, b, orc.SEL_EPS_REL, eps=1e-12,
                               predictor=orc.PRED_LINEAR)
        mirrored = np.array([_uses_mirror(orc, N, p) for p in range(N * N)])
        assert mirrored.any()
        assert (det[~mirrored] == 0).all(), N
        assert (det[mirrored] > 0).all(), N


def test_spike_on_a_coarse_point(orc):
    N, q = 17, 8 * 17 + 8  # (8, 8): level 1 of J = 4, spacing 8
    b = np.zeros(N * N)
    b[q] = 1.0
    _, det, _ = orc.select(N, b, orc.SEL_EPS_REL, eps=1e-12, predictor=orc.PRED_LINEAR)
    want = np.zeros(N * N)
    want[q] = 1.0  # its own corners (G^0) are 0
    for h in (4, 2, 1):  # spacings of levels 2, 3, 4
        for dx, dy, v in ((h, 0, 0.5), (-h, 0, 0.5), (0, h, 0.5), (0, -h, 0.5),
                          (h, h, 0.25), (-h, h, 0.25), (h, -h, 0.25), (-h, -h, 0.25)):
            want[(8 + dy) * N + 8 + dx] = v
    assert np.array_equal(det, want)


def test_keep_count_with_the_linear_predictor(orc):
    N = 21
    rng = np.random.default_rng(8)
    b = rng.standard_normal(N * N) ** 2
    for K in (4, 30, 200, N * N):
        idx, det, _ = orc.select(N, b, orc.SEL_KEEP_COUNT, keep_count=K,
                                 predictor=orc.PRED_LINEAR)
        assert len(idx) == K and (np.diff(idx) > 0).all()
        coarse = {p for p in range(N * N) if orc.level(N, p % N, p // N)[0] == 0}
        assert coarse <= set(idx.tolist())
        rest = sorted(set(range(N * N)) - coarse, key=lambda p: (-det[p], p))
        assert set(idx.tolist()) == coarse | set(rest[:K - len(coarse)])


def _mirrored_detail_closed_form(N, ix, iy, h):
    """Detail of the bilinear field b = 3 + 2 ix + 5 iy + 0.5 ix iy at a
    point whose stencil is mirrored at the far edge, written out by hand:
    with only x mirrored the prediction is b(ix - h, iy) (the x neighbours
    coincide and the field is linear in y at fixed x), with only y mirrored
    b(ix, iy - h), with both b(ix - h, iy - h)."""
    ox, oy = ix % (2 * h) != 0, iy % (2 * h) != 0
    mx, my = ox and ix + h > N - 1, oy and iy + h > N - 1
    if mx and my:
        return 7.0 * h + 0.5 * h * (ix + iy - h)
    if mx:
        return h * (2.0 + 0.5 * iy)
    if my:
        return h * (5.0 + 0.5 * ix)
    raise AssertionError("not a mirrored point")


def test_bilinear_field_detail_at_mirrored_points(orc):
    # A clamp-to-the-last-line reading, or one that drops the mirrored
    # neighbour, gives other values at these points.
    for N in (21, 41, 100):
        b = _bilinear(N)
        _, det, _ = orc.select(N, b, orc.SEL_EPS_REL, eps=1e-12, predictor=orc.PRED_LINEAR)
        J = int(np.floor(np.log2(N)))
        n_checked = 0
        for p in range(N * N):
            if not _uses_mirror(orc, N, p):
                continue
            ix, iy = p % N, p // N
            h = 1 << (J - orc.level(N, ix, iy)[0])
            assert det[p] == _mirrored_detail_closed_form(N, ix, iy, h), (N, ix, iy)
            n_checked += 1
        assert n_checked > 0


def test_spike_golden_mirror_fixture(orc):
    with open(os.path.join(GOLDEN, "select_linear_mirror_N21.json")) as fh:
        g = json.load(fh)
    N = g["N"]
    b = np.zeros(N * N)
    b[g["spike"][1] * N + g["spike"][0]] = 1.0
    _, det, _ = orc.select(N, b, orc.SEL_EPS_REL, eps=1e-12, predictor=orc.PRED_LINEAR)
    want = np.zeros(N * N)
    for ix, iy, v in g["detail"]:
        want[iy * N + ix] = v
    assert np.array_equal(det, want)
    # the mirrored point is kept at eps = 1 and would not be under a clamp
    idx, _, _ = orc.select(N, b, orc.SEL_EPS_REL, eps=1.0, predictor=orc.PRED_LINEAR)
    assert 20 in set(idx.tolist())
