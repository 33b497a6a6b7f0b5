"""Register spills of the sweep kernels, from the compiler's resource report
for gfx950 (host only: hipcc cross-compiles).  A spill in a sweep kernel
costs several times its run time (a 32-group head of the double kernel
spilling 400 bytes per lane made the plain FP64 band 3.8 times slower), and
nothing but the timings would show it."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def scratch():
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    from paper_1608_05179_amd import build
    cmd = [HIPCC, *build.FLAGS, "-c", os.path.join(build.CSRC, "gs.hip"), "-o", os.devnull,
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    out, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            out[name] = int(m.group(1))
    assert out, "no resource report"
    return out


def test_plain_sweep_kernels_do_not_spill(scratch):
    plain = {k: v for k, v in scratch.items() if "gs_kernel" in k}
    assert len(plain) >= 12
    assert all(v == 0 for v in plain.values()), {k: v for k, v in plain.items() if v}


def test_cooperative_sweep_kernels_spill_at_most_job_state(scratch):
    # the cooperative kernel keeps a few job-level values in scratch
    # (reloaded once per job, not per period)
    coop = {k: v for k, v in scratch.items() if "gs_coop_kernel" in k}
    assert len(coop) >= 24
    assert max(coop.values()) <= 48, {k: v for k, v in coop.items() if v > 48}
