"""The medium scene over its whole schedule (13,600 substeps: two cuts, each
followed by a 0.3 s push) on the GPU, with the label and state invariants that hold
at any length (the oracle would need about 25 minutes for it):

- labels persist (Sec. III-D): once a particle's digit of a cut is 1 or 2 it never
  changes, checked after every call of at most 50 substeps;
- every cut separates the tube: each side of each cut plane holds thousands of
  labelled particles, and a particle's new digit is its side of the blade plane in
  the current configuration right after the call that labelled it (Eq. 3, side 1
  for s < 0; calls of at most 50 substeps, in which a particle moves well below a
  millimetre), for all but 1 % (a sign or frame mistake would put about half or all
  of them on the wrong side).  The reference configuration cannot serve here: the
  first push moves the tube where the second cut is made by centimetres;
- the state stays finite with det F > 0 (status OK, finite u and F).
"""
import numpy as np
import pytest

from paper_2609_27342_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 13600
CHUNK = 50


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
    seen = {0: [0, 0, 0], 1: [0, 0, 0]}  # side 1, side 2, wrong side
    calls = 0
    for j, cnt, tools in W.segments(s, 0, STEPS):
        done = 0
        while done < cnt:
            k = min(CHUNK, cnt - done)
            tk = s["tools_at"](j + done)  # poses at the call's first substep
            g.step([dict(t, advance=True) for t in tk], k)
            done += k
            calls += 1
            st = g.read(("digits", "u"))
            dg = st["digits"][:, :2]
            held = prev != 0
            assert np.array_equal(dg[held], prev[held]), f"a digit changed before substep {j + done}"
            for t in s["tools_at"](j + done - 1):
                if not t["labels"]:
                    continue
                c = t["blade"]["cut_index"]
                new = (prev[:, c] == 0) & (dg[:, c] != 0)
                if not new.any():
                    continue
                x = X[new] + st["u"][new].astype(np.float64)
                side = np.where((x - np.asarray(t["blade"]["x_e"])) @ np.asarray(t["blade"]["n"]) < 0.0, 1, 2)
                seen[c][0] += int((dg[new, c] == 1).sum())
                seen[c][1] += int((dg[new, c] == 2).sum())
                seen[c][2] += int((dg[new, c] != side).sum())
            prev = dg.copy()
    assert g.status() == 0
    st = g.read(("u", "H"))
    assert np.isfinite(st["u"]).all() and np.isfinite(st["H"]).all()
    g.close()
    for c, (n1, n2, wrong) in seen.items():
        lab = int((prev[:, c] != 0).sum())
        print(f"[medium-full] cut {c}: labelled {lab} (1: {n1}, 2: {n2}), on the other side of the blade plane "
              f"after the labelling call: {wrong}", flush=True)
        assert n1 + n2 == lab
        assert n1 > 2000 and n2 > 2000
        assert wrong < 0.01 * lab
    print(f"[medium-full] {calls} calls", flush=True)
