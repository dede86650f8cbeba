"""Rigid contact's brick skip test (tlmpm_reach.h, Eq. 14) on the CPU.

tests/native/reach_check.hip is built with hipcc as a host program.  It draws blade
rectangles in random orientations, moving and spinning, and particles about their
faces, edges and corners at distances around the contact reach; the contact
predicate is evaluated there from its definition in FP64.  A brick holding a
particle that takes an impulse must never be skipped; without the tool's spin in
the reach some would be, and the blade-axis tests skip bricks that the rectangle's
bounding box alone would keep.
"""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC), reason="hipcc not available")
def test_rigid_brick_skip_never_skips_a_touched_particle(tmp_path):
    exe = tmp_path / "reach_check"
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-x", "hip",
                           os.path.join(HERE, "native", "reach_check.hip"), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    m = re.search(r"cases (\d+) contact (\d+) missed (\d+) norot_missed (\d+) pruned (\d+)", out.stdout)
    assert m, out.stdout + out.stderr
    cases, contact, missed, norot, pruned = map(int, m.groups())
    assert out.returncode == 0 and missed == 0, out.stdout
    assert contact > 0.3 * cases
    assert norot > 50        # the spin term of the reach is needed ...
    assert pruned > 1000     # ... and the blade axes skip bricks the bounding box keeps
