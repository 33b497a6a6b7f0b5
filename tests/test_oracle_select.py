"""Pins of the oracle's wavelet-compressed grid (Algorithm 1).

The oracle finds each point's level and parent in closed form (2-adic
valuations).  These tests check it against hand-derived fixtures, against a
literal level-by-level transcription of Algorithm 1's loops written here
independently, and against properties any correct threshold must have.
"""
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_levels_and_parents_fixture(orc):
    fx = _load("select_delta_N9.json")
    counts = {}
    for iy in range(9):
        for ix in range(9):
            lv, _, _ = orc.level(9, ix, iy)
            counts[lv] = counts.get(lv, 0) + 1
    assert {str(k): v for k, v in counts.items()} == fx["level_counts"]
    for case in fx["parents"]:
        lv, px, py = orc.level(9, *case["p"])
        assert lv == case["level"]
        assert [px, py] == case["parent"]


def test_delta_maps_fixture(orc):
    fx = _load("select_delta_N9.json")
    for case in fx["delta_maps"]:
        b = np.zeros(81)
        ix, iy = case["spike"]
        b[iy * 9 + ix] = 1.0
        for eps in (1e-6, 0.5, 1.0):
            idx, _, _ = orc.select(9, b, orc.SEL_EPS_REL, eps)
            assert idx.tolist() == case["kept"], (case["spike"], eps)


def _algorithm1_literal(N, b, eps):
    """Algorithm 1 written out level by level: nested grids G^j from the
    restriction x_k^j = x_{2k}^{j+1}, interpolation from G^j to
    G^{j+1} \\ G^j by the nearest coarser point below-left, threshold
    |interp - b| >= eps * max|b|, G^0 always kept, union over levels."""
    J = int(np.floor(np.log2(N)))
    tau = eps * np.max(np.abs(b))
    B = b.reshape(N, N)  # B[iy, ix]

    def grid(j):
        h = 2 ** (J - j)
        return {(ix, iy) for ix in range(0, N, h) for iy in range(0, N, h)}

    kept = set()
    for j in range(J - 1, -1, -1):
        coarse, fine = grid(j), grid(j + 1)
        H = 2 ** (J - j)
        for (ix, iy) in fine - coarse:
            interp = B[(iy // H) * H, (ix // H) * H]
            if abs(interp - B[iy, ix]) >= tau:
                kept.add((ix, iy))
    kept |= grid(0)
    return sorted(iy * N + ix for ix, iy in kept)


@pytest.mark.parametrize("N", [1, 2, 5, 9, 10, 16, 17, 21, 33, 41])
def test_matches_literal_algorithm1(orc, N):
    rng = np.random.default_rng(N)
    for trial in range(4):
        b = rng.random(N * N) ** 3
        if trial == 3:  # many exact ties
            b = np.round(b * 4) / 4
        for eps in (0.0, 0.02, 0.1, 0.3):
            idx, _, _ = orc.select(N, b, orc.SEL_EPS_REL, eps)
            assert idx.tolist() == _algorithm1_literal(N, b, eps)


def test_constant_map_keeps_coarsest_grid_only(orc):
    for N in (9, 21, 41, 101):
        idx, _, _ = orc.select(N, np.full(N * N, 0.7), orc.SEL_EPS_REL, 1e-9)
        J = int(np.floor(np.log2(N)))
        h = 2 ** J
        g0 = sorted(iy * N + ix for ix in range(0, N, h) for iy in range(0, N, h))
        assert idx.tolist() == g0


def test_eps_zero_and_keep_all_keep_everything(orc):
    b = np.random.default_rng(1).random(41 * 41)
    for mode, eps in ((orc.SEL_EPS_REL, 0.0), (orc.SEL_KEEP_ALL, 0.5)):
        idx, _, _ = orc.select(41, b, mode, eps)
        assert idx.tolist() == list(range(41 * 41))


def test_threshold_ties_are_kept(orc):
    # |d| == tau exactly keeps the point (>= in Algorithm 1).
    N = 5
    b = np.zeros(N * N)
    b[0] = 1.0       # max|b| = 1 at a G^0 point
    b[1] = 0.25      # (1,0): parent (0,0), |d| = 0.75
    b[2] = 0.5       # (2,0): parent (0,0), |d| = 0.5
    idx, _, mg = orc.select(N, b, orc.SEL_EPS_REL, 0.5)
    assert 2 in idx.tolist()
    assert mg == 0.0


def test_nesting_in_eps(orc):
    # Larger thresholds keep subsets (the trend of the paper's epsilon table).
    rng = np.random.default_rng(7)
    b = rng.random(41 * 41) ** 4
    prev = None
    for eps in (0.3, 0.2, 0.1, 0.05, 0.01, 0.0):
        idx, _, _ = orc.select(41, b, orc.SEL_EPS_REL, eps)
        s = set(idx.tolist())
        if prev is not None:
            assert prev <= s
        prev = s


def test_keep_count(orc):
    rng = np.random.default_rng(3)
    N = 41
    b = rng.random(N * N)
    _, det, _ = orc.select(N, b, orc.SEL_KEEP_ALL)
    lv = np.array([orc.level(N, p % N, p // N)[0] for p in range(N * N)])
    g0 = np.flatnonzero(lv == 0)
    for K in (0, 3, 4, 5, 169, 337, 505, N * N - 1, N * N, N * N + 7):
        idx, _, mg = orc.select(N, b, orc.SEL_KEEP_COUNT, keep_count=K)
        assert len(idx) == min(max(K, len(g0)), N * N)
        assert set(g0.tolist()) <= set(idx.tolist())
        assert np.all(np.diff(idx) > 0)
        # brute force: the K - |G0| largest details among the other points
        cand = np.flatnonzero(lv != 0)
        order = sorted(cand.tolist(), key=lambda p: (-det[p], p))
        want = sorted(g0.tolist() + order[:max(0, K - len(g0))])
        assert idx.tolist() == want
    # ties in |d| are broken by grid index
    bt = np.zeros(N * N)
    bt[np.flatnonzero(lv != 0)[::2]] = 1.0
    _, dt, _ = orc.select(N, bt, orc.SEL_KEEP_ALL)
    tied = [p for p in range(N * N) if lv[p] != 0 and dt[p] == 1.0]
    assert len(tied) > 50
    idx, _, mg = orc.select(N, bt, orc.SEL_KEEP_COUNT, keep_count=len(g0) + 30)
    assert idx.tolist() == sorted(g0.tolist() + tied[:30])
    assert mg == 0.0


def test_detail_is_difference_from_parent(orc):
    rng = np.random.default_rng(11)
    N = 21
    b = rng.standard_normal(N * N)
    _, det, _ = orc.select(N, b, orc.SEL_KEEP_ALL)
    for p in range(N * N):
        lv, px, py = orc.level(N, p % N, p // N)
        want = 0.0 if lv == 0 else abs(b[p] - b[py * N + px])
        assert det[p] == want
