"""The material-contact search skip (Sec. III-E; tlmpm_tuning.pair_skip) changes
no result: the same scenes stepped with the skip on and off end in bitwise the same
state (positions, velocities, deformation gradients, codes, cutting progress,
digits), while the skip is in use (skipped searches > 0 with it on, none with it
off).  Scenes: medium with its blade in the tube from the first substep (300
substeps: cut, contact, pushes) and three many-scene bodies with 1-3 crossing
blades stepped as one batch (150 substeps).
"""
import numpy as np
import pytest

from paper_2609_27342_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("u", "v", "H", "code", "D", "digits")


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_27342_amd import tlmpm
    tlmpm.lib()
    return tlmpm


def _scenes(tl, make, skip):
    tl.set_tuning(pair_skip=skip)
    try:
        return [tl.Scene(s) for s in make()]
    finally:
        tl.set_tuning(None)


def test_medium_skip_on_equals_off(tl):
    sc = W.medium(z_start=0.034)
    print(f"[case] medium n={sc['X'].shape[0]} steps=300", flush=True)
    out = {}
    for skip in (1, 0):
        (g,) = _scenes(tl, lambda: [sc], skip)
        for j, cnt, tools in W.segments(sc, 0, 300):
            g.step([dict(t, advance=True) for t in tools], n_substeps=cnt)
        assert g.status() == 0
        out[skip] = (g.read(FIELDS), g.contact_stats()["skipped"])
        g.close()
    assert out[1][1] > 0 and out[0][1] == 0
    for k in FIELDS:
        assert np.array_equal(out[1][0][k], out[0][0][k]), k


def test_batch_skip_on_equals_off(tl):
    scenes = [W.batch_scene(21, i, 30000, steps=160) for i in (6, 9, 1)]
    print(f"[case] batch n={[s['X'].shape[0] for s in scenes]} steps=150", flush=True)
    out = {}
    for skip in (1, 0):
        gs = _scenes(tl, lambda: scenes, skip)
        with tl.Batch(gs) as bt:
            for j in range(150):
                bt.step([s["tools_at"](j) for s in scenes], 1)
        out[skip] = ([g.read(FIELDS) for g in gs], sum(g.contact_stats()["skipped"] for g in gs),
                     [g.status() for g in gs])
        for g in gs:
            g.close()
    assert out[1][2] == [0, 0, 0] and out[0][2] == [0, 0, 0]
    assert out[1][1] > 0 and out[0][1] == 0
    for a, b in zip(out[1][0], out[0][0]):
        for k in FIELDS:
            assert np.array_equal(a[k], b[k]), k
