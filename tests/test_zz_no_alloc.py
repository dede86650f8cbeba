"""The batch entry point that allocates nothing (tlmpm_batch_create_static) against
the one with a caller workspace (tlmpm_batch_create), through the C ABI: the same
scenes and calls give bitwise the same fields and wrenches, on two batches in a
row on the static array (the second with fewer, smaller scenes, so that it runs
over what the first one left there), and a second live batch on the same device
is refused."""
import numpy as np
import pytest

from paper_2609_27342_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("u", "v", "F", "code", "D", "digits")


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_27342_amd import tlmpm
    tlmpm.lib()
    return tlmpm


def _run(tl, scenes, K, static):
    gs = [tl.Scene(s) for s in scenes]
    ws = []
    with tl.Batch(gs, static=static) as b:
        for j in range(K):
            ws.append(b.step([[dict(t, advance=True) for t in s["tools_at"](j)] for s in scenes], 1, wrench=True))
    out = [g.read(FIELDS) for g in gs]
    st = [g.status() for g in gs]
    for g in gs:
        g.close()
    return out, np.array(ws), st


def _same(tl, scenes, K):
    print(f"[case] no-alloc batch n={[s['X'].shape[0] for s in scenes]} steps={K}", flush=True)
    ref, wref, sref = _run(tl, scenes, K, static=False)
    got, wgot, sgot = _run(tl, scenes, K, static=True)
    assert sref == sgot and all(v == 0 for v in sgot)
    assert np.array_equal(wref, wgot)
    for i in range(len(scenes)):
        for f in FIELDS:
            assert np.array_equal(ref[i][f], got[i][f]), (i, f)
    assert any(np.any(r["code"] != 0) for r in ref)


def test_static_batch_equals_workspace_batch_twice(tl):
    big = [W.batch_scene(23, i, n, steps=20) for i, n in enumerate((14000, 6000, 9000, 4000))]
    _same(tl, big, 12)
    small = [W.batch_scene(24, i, n, steps=20) for i, n in enumerate((3000, 2500))]
    _same(tl, small, 8)


def test_second_live_static_batch_is_refused(tl):
    scenes = [W.batch_scene(25, i, 3000, steps=4) for i in range(3)]
    gs = [tl.Scene(s) for s in scenes]
    b = tl.Batch(gs[:2], static=True)
    with pytest.raises(tl.TlmpmError) as e:
        tl.Batch(gs[2:], static=True)
    assert e.value.code == tl.E_INVALID
    b.close()
    b2 = tl.Batch(gs[2:], static=True)  # the array is free again
    b2.step([[]], 1)
    b2.close()
