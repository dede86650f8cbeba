"""The medium scene over its whole schedule (13,600 substeps: two cuts, each
followed by a 0.3 s push) on the GPU, with the label and state invariants that hold
at any length (the oracle would need about 25 minutes for it):

- labels persist (Sec. III-D): once a particle's digit of a cut is 1 or 2 it never
  changes, checked after every call of at most 200 substeps;
- every cut separates the tube: each side of each cut plane holds thousands of
  labelled particles, and a labelled particle's digit is its side of the cut plane
  at the reference configuration (Eq. 3, side 1 for s < 0) for all but the few
  that had moved across the plane before the band reached them (below 3 %; a sign
  or frame mistake would put about half or all of them on the wrong side);
- the state stays finite with det F > 0 (status OK, finite u and F).
"""
import numpy as np
import pytest

from paper_2609_27342_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 13600
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
def test_medium_full_schedule_label_persistence_and_sides(tl):
    s = W.medium(steps=STEPS)
    X = s["X"].astype(np.float64)
    print(f"[case] medium full schedule n={X.shape[0]} steps={STEPS}", flush=True)
    g = tl.Scene(s)
    prev = np.zeros((X.shape[0], 2), np.uint8)
    planes = {}
    calls = 0
    for j, cnt, tools in W.segments(s, 0, STEPS):
        for t in tools:
            if t["labels"]:
                planes.setdefault(t["blade"]["cut_index"], (np.asarray(t["blade"]["x_e"]), np.asarray(t["blade"]["n"])))
        done = 0
        while done < cnt:
            k = min(CHUNK, cnt - done)
            tk = s["tools_at"](j + done)  # poses at the chunk's first substep
            g.step([dict(t, advance=True) for t in tk], k)
            done += k
            calls += 1
            dg = g.read(("digits",))["digits"][:, :2]
            held = prev != 0
            assert np.array_equal(dg[held], prev[held]), f"a digit changed before substep {j + done}"
            prev = dg.copy()
    assert g.status() == 0
    st = g.read(("u", "H"))
    assert np.isfinite(st["u"]).all() and np.isfinite(st["H"]).all()
    g.close()
    assert set(planes) == {0, 1}
    for k, (xe, n) in planes.items():
        lab = prev[:, k] != 0
        side = np.where((X - xe) @ n < 0.0, 1, 2)
        n1, n2 = int(((prev[:, k] == 1)).sum()), int((prev[:, k] == 2).sum())
        wrong = int((prev[lab, k] != side[lab]).sum())
        print(f"[medium-full] cut {k}: labelled {lab.sum()} (1: {n1}, 2: {n2}), other side of the reference "
              f"plane {wrong}", flush=True)
        assert n1 > 2000 and n2 > 2000
        assert wrong < 0.03 * lab.sum()
    print(f"[medium-full] {calls} calls", flush=True)
