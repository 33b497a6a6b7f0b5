"""The C ABI library on a machine without a GPU: it loads, exports every
function include/damas.h declares, and rejects invalid arguments on the host
(before any device work) with the documented codes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "damas.h")
LIB = os.path.join(ROOT, "paper_1608_05179_amd", "libdamas_hip.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(damas_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1608_05179_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    lib.damas_strerror.restype = ctypes.c_char_p
    assert lib.damas_strerror(0) == b"success"
    assert lib.damas_strerror(-1) == b"invalid argument"
    assert lib.damas_strerror(-7) == b"device-side capacity exceeded"
    assert lib.damas_strerror(-99) == b"unknown status"


def test_layout_helpers(lib):
    lib.damas_ld.restype = ctypes.c_int64
    # rows rounded up to 32 elements: float rows start on whole 128-byte lines
    assert [lib.damas_ld(v) for v in (0, 1, 8, 9, 32, 33, 337)] == [0, 32, 32, 32, 32, 64, 352]
    # |G^0| = 4 unless N is a power of two (then only index 0 of each axis)
    assert [lib.damas_coarse_count(n) for n in (1, 2, 3, 4, 5, 16, 17, 21, 41, 101)] == \
        [1, 1, 4, 1, 4, 1, 4, 4, 4, 4]
    assert [lib.damas_mp(m) for m in (0, 1, 16, 17, 64, 128)] == [0, 16, 16, 32, 64, 128]


def test_gs_capacity(lib):
    from paper_1608_05179_amd import damas as dm
    # One sweep workgroup's LDS (160 KB less a margin) beside the partial sums
    # and the two hand-over blocks of the larger (cooperative) kernel: x~ of
    # 1,856 unknowns with double A, 10,112 with float A; bf16 sweeps would
    # hold 14,496 but a bf16 solve ends with FP32 sweeps.  Capacities are
    # multiples of the row alignment (32), so damas_ld(cap) == cap.
    assert [lib.damas_gs_capacity(p) for p in (dm.PREC_FP64, dm.PREC_FP32, dm.PREC_BF16)] == \
        [1856, 10112, 10112]
    assert lib.damas_gs_capacity(9) == 0 and lib.damas_gs_capacity(-1) == 0
    fake = ctypes.c_void_p(0x1000)
    for p in (dm.PREC_FP64, dm.PREC_FP32, dm.PREC_BF16):
        cap = lib.damas_gs_capacity(p)
        assert dm._lib.damas_gs(101, 1, fake, cap + 1, fake, fake, p, 1, fake, fake, 1,
                                None, fake, None) == dm.EINVAL


def test_coarse_count_matches_oracle(lib, orc):
    for N in (1, 2, 3, 7, 8, 9, 33, 50, 64, 101):
        n0 = sum(orc.level(N, ix, iy)[0] == 0 for ix in range(N) for iy in range(N))
        assert lib.damas_coarse_count(N) == n0


def test_invalid_arguments_rejected_on_host(lib):
    from paper_1608_05179_amd import damas as dm
    lib.damas_last_error.restype = ctypes.c_char_p
    G = dm.Geometry
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    # NULL geometry / bad M / bad N / non-positive c
    assert dm._lib.damas_das_map(None, 1, fake, fake, fake, None) == dm.EINVAL
    g = G(0, 0x1000, 21, -1, 1, -1, 1, 1.5, 343.0)
    assert dm._lib.damas_das_map(ctypes.byref(g), 1, fake, fake, fake, None) == dm.EINVAL
    assert b"M = 0" in lib.damas_last_error()
    g = G(16, 0x1000, 0, -1, 1, -1, 1, 1.5, 343.0)
    assert dm._lib.damas_das_map(ctypes.byref(g), 1, fake, fake, fake, None) == dm.EINVAL
    g = G(16, 0x1000, 21, -1, 1, -1, 1, 1.5, -1.0)
    assert dm._lib.damas_das_map(ctypes.byref(g), 1, fake, fake, fake, None) == dm.EINVAL
    g = G(16, 0x1000, 21, -1, 1, -1, float("nan"), 1.5, 343.0)
    assert dm._lib.damas_das_map(ctypes.byref(g), 1, fake, fake, fake, None) == dm.EINVAL
    # selection: unknown mode, negative eps, KEEP_COUNT without counts
    assert dm._lib.damas_select(21, 1, fake, 7, 0.0, None, fake, fake, None) == dm.EINVAL
    assert dm._lib.damas_select(21, 1, fake, dm.SEL_EPS_REL, -0.1, None, fake, fake, None) == dm.EINVAL
    assert dm._lib.damas_select(21, 1, fake, dm.SEL_KEEP_COUNT, 0.0, None, fake, fake, None) == dm.EINVAL
    # sweeps: max_kept beyond the grid, beyond on-chip capacity, bad precision
    assert dm._lib.damas_gs(21, 1, fake, 442, fake, fake, dm.PREC_FP32, 1, fake, fake, 10,
                            None, fake, None) == dm.EINVAL
    assert dm._lib.damas_gs(301, 1, fake, 60000, fake, fake, dm.PREC_FP32, 1, fake, fake, 10,
                            None, fake, None) == dm.EINVAL
    assert b"on chip" in lib.damas_last_error()
    assert dm._lib.damas_gs(21, 1, fake, 100, fake, fake, 9, 1, fake, fake, 10,
                            None, fake, None) == dm.EINVAL
    assert dm._lib.damas_gs(21, 1, fake, 100, fake, fake, dm.PREC_FP32, 1, fake, fake, -1,
                            None, fake, None) == dm.EINVAL
    # layout and PSF argument checks
    assert dm._lib.damas_layout(1, None, 10, 100, fake, None) == dm.EINVAL
    assert dm._lib.damas_psf(0, 1, fake, 10, dm.PREC_FP32, fake, 1000, fake, fake, None) == dm.EINVAL
    assert dm._lib.damas_psf(16, 2, fake, 10, dm.PREC_FP32, fake, 10, fake, fake, None) == dm.EINVAL
    # bf16 steering / PSF checks; damas_psf stores only double or float
    gb = ctypes.byref(G(16, 0x1000, 21, -1, 1, -1, 1, 1, 343.0))
    assert dm._lib.damas_steer_bf16(gb, 2, fake, fake, fake, 100, fake, 10, None) == dm.EINVAL
    assert dm._lib.damas_steer_bf16(gb, 1, fake, fake, fake, 442, fake, 0, None) == dm.EINVAL
    assert dm._lib.damas_psf_bf16(129, 1, fake, 10, fake, 0, fake, fake, None) == dm.EINVAL
    assert dm._lib.damas_psf_bf16(16, 2, fake, 100, fake, 10, fake, fake, None) == dm.EINVAL
    assert dm._lib.damas_psf(16, 1, fake, 10, dm.PREC_BF16, fake, 1000, fake, fake, None) == dm.EINVAL
    assert b"damas_psf_bf16" in lib.damas_last_error()
    # autotuner and graphs: NULL handles are refused on the host
    assert dm._lib.damas_ctx_autotune(None, gb, 1, fake, fake, None, 10, None, None) == dm.EINVAL
    assert dm._lib.damas_graph_launch(None, None) == dm.EINVAL
    assert dm._lib.damas_graph_capture(None, gb, 1, fake, fake, None, None, fake, None, None,
                                       None, None) == dm.EINVAL
    assert dm._lib.damas_ctx_set_coop(None, -1) == dm.EINVAL
    # whole-path: NULL context / NULL params
    assert dm._lib.damas_solve_dev(None, ctypes.byref(G(16, 0x1000, 21, -1, 1, -1, 1, 1, 343.0)),
                                   1, fake, fake, None, None, fake, None, None, None,
                                   None) == dm.EINVAL


def test_query_footprint_closed_form(lib):
    """Footprint of a solve = inputs + x map + s_tilde + the context's b,
    idx, offsets, steering rows and A arena (host-only call)."""
    from paper_1608_05179_amd import damas as dm
    M, N, S = 16, 21, 441
    L = dm.ld(S)
    want = 8 * (3 * M + 1 + M * M * 2)            # mic, freq, CSM
    want += 8 * S + 4                              # x map (double), s_tilde
    want += 8 * S + 4 * S + 8 * 2                  # b, idx, offsets
    want += 8 * L * 2 * M + 8 * L * L              # steering rows, A (double)
    assert dm.query_footprint(M, N, 1, precision=dm.PREC_FP64, iterations=10) == want
    # float A, two bins of KEEP_COUNT 100 (ld 104): per-bin arenas packed
    L2 = dm.ld(100)
    want2 = 8 * (3 * M + 2 + 2 * M * M * 2) + 4 * 2 * S + 4 * 2
    want2 += 8 * 2 * S + 4 * 2 * S + 4 * 2 + 8 * 3
    want2 += 8 * 2 * L2 * 2 * M + 4 * 2 * L2 * L2
    assert dm.query_footprint(M, N, 2, select_mode=dm.SEL_KEEP_COUNT, keep_count=100,
                              iterations=10, policy=dm.POLICY_FIXED) == want2
    # the per-bin precision classes (default policy) add the bf16 residual
    # arena, the PSF's tile sums (ld 104: 2 x 2 tiles, 3 in the upper
    # triangle) and one class byte per bin
    want2 += 2 * 2 * L2 * L2 + 8 * 2 * 3 + 2
    assert dm.query_footprint(M, N, 2, select_mode=dm.SEL_KEEP_COUNT, keep_count=100,
                              iterations=10) == want2
    # BF16 with refinement holds both arenas and both steering tables
    fb = dm.query_footprint(M, N, 1, precision=dm.PREC_BF16, refine_sweeps=5, iterations=10)
    f32 = dm.query_footprint(M, N, 1, precision=dm.PREC_FP32, iterations=10)
    assert fb == f32 + 2 * L * L + 2 * L * 2 * dm.mp(M)
    with pytest.raises(dm.DamasError):
        dm.query_footprint(0, N, 1)
    with pytest.raises(dm.DamasError):
        dm.query_footprint(M, N, 1, precision=dm.PREC_BF16, refine_sweeps=11, iterations=10)


def test_csm_rejects_invalid_arguments_on_the_host(lib):
    f = lib.damas_csm
    f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p]
    p = ctypes.c_void_p(16)  # never dereferenced: every call fails validation
    assert f(0, 4, 1, p, p, None) == -1
    assert f(8193, 4, 1, p, p, None) == -1
    assert f(8, 0, 1, p, p, None) == -1
    assert f(8, 4, -1, p, p, None) == -1
    assert f(8, 4, 1, None, p, None) == -1
    assert f(8, 4, 1, p, None, None) == -1
    assert f(8, 4, 0, None, None, None) == 0  # nothing to do, nothing launched


def test_select_pred_rejects_unknown_predictor(lib):
    f = lib.damas_select_pred
    f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                  ctypes.c_double, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p]
    p = ctypes.c_void_p(16)  # never dereferenced: the call fails validation
    assert f(9, 1, p, 1, 0.1, 2, None, p, p, None) == -1
    assert f(9, 1, p, 1, 0.1, -1, None, p, p, None) == -1
    assert f(9, 0, None, 1, 0.1, 1, None, None, None, None) == 0


def test_host_solve_validates_on_the_host(lib):
    f = lib.damas_solve
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 8
    p = ctypes.c_void_p(16)  # never dereferenced: the call fails validation
    assert f(None, p, 1, p, p, p, None, p, None, None, None) == -1


def test_keep_frac_is_keep_count_of_its_ceiling(lib):
    # KEEP_FRAC keeps ceil(p N^2) points in every bin (level-0 points
    # included): p = 0.1, 0.2, 0.3 on a 41 x 41 grid keep 169, 337, 505.
    import math
    from paper_1608_05179_amd import damas as dm
    M, N = 64, 41
    for p, K in ((0.1, 169), (0.2, 337), (0.3, 505)):
        assert math.ceil(p * N * N) == K
        for prec in (dm.PREC_FP32, dm.PREC_FP64):
            assert dm.query_footprint(M, N, 3, select_mode=dm.SEL_KEEP_FRAC, keep_frac=p,
                                      precision=prec, iterations=10) == \
                dm.query_footprint(M, N, 3, select_mode=dm.SEL_KEEP_COUNT, keep_count=K,
                                   precision=prec, iterations=10)
    # the whole grid, and a fraction below one point: clamped like KEEP_COUNT
    assert dm.query_footprint(M, N, 1, select_mode=dm.SEL_KEEP_FRAC, keep_frac=1.0) == \
        dm.query_footprint(M, N, 1, select_mode=dm.SEL_KEEP_COUNT, keep_count=N * N)
    assert dm.query_footprint(M, N, 1, select_mode=dm.SEL_KEEP_FRAC, keep_frac=1e-9) == \
        dm.query_footprint(M, N, 1, select_mode=dm.SEL_KEEP_COUNT, keep_count=1)
    for bad in (0.0, -0.1, 1.5, float("nan"), float("inf")):
        with pytest.raises(dm.DamasError) as ei:
            dm.query_footprint(M, N, 1, select_mode=dm.SEL_KEEP_FRAC, keep_frac=bad)
        assert ei.value.code == dm.EINVAL
    # the step-level selection takes counts, not fractions
    fake = ctypes.c_void_p(0x1000)
    assert lib.damas_select(N, 1, fake, dm.SEL_KEEP_FRAC, ctypes.c_double(0.0), fake, fake,
                            fake, None) == dm.EINVAL
