"""The material-contact search skip (tlmpm_reach.h, pair_skip_bounds_ok; Sec. III-E,
Eqs. 10-13 with the reference-neighbour exclusion) on the CPU.

tests/native/pair_skip_check.hip builds bodies of jittered particles, deforms them
(translation, rotation, strain, noise, a slip of about a cell, a second piece pushed
against the body to below the bin edge), forms the per-brick displacement anchors
and spreads as the transfer pass does, and brute-forces every pair within the bin
edge: a candidate the rule skips must have no partner (every particle within reach
a reference neighbour with a compatible side code).  Loosening either of the rule's
two bounds must let skipped candidates with partners through.
"""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC), reason="hipcc not available")
def test_skipped_candidates_have_no_partner(tmp_path):
    exe = tmp_path / "pair_skip_check"
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "--offload-arch=gfx950", "-x", "hip",
                           os.path.join(HERE, "native", "pair_skip_check.hip"), "-o", str(exe)])
    res = {}
    for mode in (0, 1, 2):
        out = subprocess.run([str(exe), str(mode)], capture_output=True, text=True, timeout=120)
        m = re.search(r"trials (\d+) candidates (\d+) skipped (\d+) violations (\d+)", out.stdout)
        assert m, out.stdout + out.stderr
        res[mode] = tuple(map(int, m.groups()))
    _, cand, skipped, viol = res[0]
    assert viol == 0, res
    assert skipped > 0.05 * cand            # the rule does skip ...
    assert res[1][3] > 100                  # ... and the foreign-brick bound is needed
    assert res[2][3] > 100                  # ... and so is the neighbour bound
