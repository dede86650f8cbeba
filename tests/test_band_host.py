"""The label pass's brick skip test (tlmpm_band.h, Eqs. 3, 4, 6) on the CPU.

tests/native/band_check.hip is built with hipcc as a host program and places
particles on the faces of the blade band with FP32 positions whose rounded value
fl(X + u) differs from the exact X + u that the side predicate reads.  A brick
whose particle gets a digit must never be skipped; the same test without the ulp
widening of the brick box is shown to skip some of them.
"""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC), reason="hipcc not available")
def test_brick_skip_test_never_skips_a_labelled_particle(tmp_path):
    exe = tmp_path / "band_check"
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-x", "hip",
                           os.path.join(HERE, "native", "band_check.hip"), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    m = re.search(r"cases (\d+) labelled (\d+) outside (\d+) unwidened_missed (\d+) missed (\d+)", out.stdout)
    assert m, out.stdout + out.stderr
    cases, labelled, outside, unwidened, missed = map(int, m.groups())
    assert out.returncode == 0 and missed == 0, out.stdout
    assert labelled > 0.3 * cases
    assert outside > 1000       # exact positions outside the FP32 box are common ...
    assert unwidened > 100      # ... and without the widening some bricks would be skipped
