"""HIP graph replay of substeps (tlmpm_set_graphs) against plain launches: every
call replays the captured pairs several times with plain launches and host
synchronisation in between; each call's state must agree bitwise."""
import numpy as np
import pytest

from paper_2609_27342_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("u", "v", "F", "code", "D")


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_27342_amd import tlmpm
    tlmpm.lib()
    return tlmpm


def _calls(scene, j0, j1):
    return [([dict(t, advance=True) for t in tools], cnt) for _, cnt, tools in W.segments(scene, j0, j1)]


@pytest.mark.parametrize("name", ["small-deep", "medium"])
def test_graph_replay_equals_plain(tl, name):
    s = W.small(deep=True) if name == "small-deep" else W.medium(z_start=0.02)
    print(f"[case] graphs {name} n={s['X'].shape[0]}", flush=True)
    spans = [(0, 9), (9, 16), (16, 29)]  # odd and even lengths, a new cut at step 0
    ref = tl.Scene(s)
    got = tl.Scene(s)
    got.graphs(True)
    for j0, j1 in spans:
        for tools, cnt in _calls(s, j0, j1):
            wr = ref.step(tools, cnt, wrench=True)
            wg = got.step(tools, cnt, wrench=True)
            assert np.array_equal(wr, wg)
        a, b = ref.read(FIELDS), got.read(FIELDS)
        for f in FIELDS:
            assert np.array_equal(a[f], b[f]), (name, j1, f)
    assert ref.status() == 0 and got.status() == 0


def test_batch_graph_replay_equals_plain(tl):
    scenes = [W.batch_scene(13, i, n, steps=30) for i, n in enumerate([3000, 6000, 4500])]
    print("[case] batch graphs", flush=True)
    outs = []
    for use in (False, True):
        gs = [tl.Scene(sc) for sc in scenes]
        with tl.Batch(gs) as b:
            b.graphs(use)
            for j0, j1 in ((0, 1), (1, 12), (12, 25)):
                b.step([[dict(t, advance=True) for t in sc["tools_at"](j0)] for sc in scenes], j1 - j0)
        outs.append([g.read(FIELDS) for g in gs])
    for a, b in zip(*outs):
        for f in FIELDS:
            assert np.array_equal(a[f], b[f]), f
