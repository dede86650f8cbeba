"""The large scene (14.2M particles) over its whole schedule of 2000 substeps on
the GPU: three blades cut from the first substep, two of them crossing, and a
fourth cut from substep 1000 through the line where the first two cross, so that
nodes there hold up to 3 x 2 x 2 side codes.  Checked at any length (the oracle
cannot follow 14.2M particles): status OK after every call of at most 200
substeps (no slot, box or lookup overflow, finite state with det F > 0), labels
persist (Sec. III-D: a digit once 1 or 2 never changes), every cut labels both
sides, and the material-contact search skip stays active (Sec. III-E: the
candidates of undisturbed surfaces have no partner).
"""
import numpy as np
import pytest

from paper_2609_27342_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 2000
CHUNK = 200


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_27342_amd import tlmpm
    tlmpm.lib()
    return tlmpm


@pytest.mark.timeout(600)
def test_large_full_schedule_status_labels_and_skip(tl):
    s = W.large(steps=STEPS)
    n = s["X"].shape[0]
    print(f"[case] large full schedule n={n} steps={STEPS}", flush=True)
    g = tl.Scene(s)
    prev = None
    for j0 in range(0, STEPS, CHUNK):
        for j, cnt, tools in W.segments(s, j0, j0 + CHUNK):
            g.step([dict(t, advance=True) for t in tools], n_substeps=cnt)
        st, detail = g.status_detail()
        assert st == 0, f"status {st} ({detail}) after substep {j0 + CHUNK}"
        c = g.contact_stats()
        dg = g.read(("digits",))["digits"][:, :4]
        if prev is not None:
            held = prev != 0
            assert np.array_equal(dg[held], prev[held]), f"a digit changed before substep {j0 + CHUNK}"
        prev = dg.copy()
        print(f"[large-full] substep {j0 + CHUNK}: candidates {c['candidates']} skipped {c['skipped']} "
              f"pairs {c['pairs']}", flush=True)
        assert c["skipped"] > 0.3 * c["candidates"]
    st = g.read(("u", "H"))
    assert np.isfinite(st["u"]).all() and np.isfinite(st["H"]).all()
    for k in range(4):
        assert (prev[:, k] == 1).sum() > 10000 and (prev[:, k] == 2).sum() > 10000, f"cut {k}"
    g.close()
