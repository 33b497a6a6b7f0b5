"""Host-side logic of bench.py (no GPU): the algorithmic bytes the sweeps'
roofline divides by, the HBM-traffic record that applies only to the
sources it was taken on, the kept-count histogram, and the refusal of more
than one GPU."""
import importlib.util
import json
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_sweep_bytes_per_storage_class(bench):
    from paper_1608_05179_amd import damas as dm
    I, R = 100, 10
    st = [300, 1000, 7]
    def pb(prec):
        return SimpleNamespace(w=SimpleNamespace(iterations=I), R=R, prec=prec)
    sq = [s * s for s in st]
    # FP64: 8 B per entry every sweep
    assert bench._sweep_bytes(pb(dm.PREC_FP64), st, None) == sum(sq) * I * 8
    # FP32: 4 B, a wide bin 4 + 2 B
    cls = [0, dm.CLASS_WIDE, 0]
    assert bench._sweep_bytes(pb(dm.PREC_FP32), st, cls) == (sq[0] + sq[2]) * I * 4 + sq[1] * I * 6
    # bf16: 2 B for the bulk sweeps and 4 B for the R refinement sweeps; a
    # bin of the FP32 class 4 B every sweep
    cls = [0, dm.CLASS_FP32, 0]
    assert bench._sweep_bytes(pb(dm.PREC_BF16), st, cls) == \
        (sq[0] + sq[2]) * ((I - R) * 2 + R * 4) + sq[1] * I * 4


def test_traffic_record_applies_only_to_its_sources(bench, monkeypatch):
    path = os.path.join(ROOT, "profiles", "gs_traffic_batched.json")
    with open(path) as fh:
        rec = json.load(fh)
    monkeypatch.setattr(bench, "sources_sha256", lambda: rec["sources_sha256"])
    assert bench._traffic("batched") == rec["hbm_bytes_per_launch"]
    monkeypatch.setattr(bench, "sources_sha256", lambda: "0" * 64)
    assert bench._traffic("batched") is None
    assert bench._traffic("no_such_workload") is None


def test_sources_digest_is_stable(bench):
    a, b = bench.sources_sha256(), bench.sources_sha256()
    assert a == b and len(a) == 64 and int(a, 16) >= 0


def test_kept_count_histogram(bench):
    import numpy as np
    h = bench._histogram(np.array([1, 499, 500, 999, 4000]))
    assert h == {"0-499": 2, "500-999": 2, "4000-4499": 1}
