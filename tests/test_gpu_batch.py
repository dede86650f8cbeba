"""Many scenes advanced by shared launches (tlmpm_batch_*) against the same scenes
stepped one at a time through tlmpm_step: the batch only groups launches, so every
field and every wrench must agree bitwise."""
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


def _print_case(name, **kw):
    print(f"[case] {name} {kw}", flush=True)


def _scenes():
    """Small scenes of the many-scene workload, plus variants: no material
    contact, no floor, no tools."""
    sizes = [3000, 9000, 5000, 12000, 4000, 7000]
    out = [W.batch_scene(11, i, n, steps=40) for i, n in enumerate(sizes)]
    out[1]["params"] = dict(out[1]["params"], material_contact=0)
    out[2]["params"] = dict(out[2]["params"], floor_on=0)
    out[3]["tools_at"] = lambda j: []
    return out


def _calls(scene, j0, j1):
    """(tools, n_substeps) calls covering steps [j0, j1): the first step of a new
    cut alone, then constant-velocity runs with TLMPM_TOOL_ADVANCE."""
    return [([dict(t, advance=True) for t in tools], cnt) for _, cnt, tools in W.segments(scene, j0, j1)]


def _run_alone(tl, scene, j0, j1, g=None):
    g = g or tl.Scene(scene)
    ws = []
    for tools, cnt in _calls(scene, j0, j1):
        w = g.step(tools, cnt, wrench=True)
        full = np.zeros((tl.MAX_TOOLS, 6))
        full[: len(tools)] = w
        ws.append(full)
    return g, ws


def _run_batch(tl, b, scenes, j0, j1):
    # every scene here changes segments at the same steps (cuts start at step 0)
    per = [_calls(s, j0, j1) for s in scenes]
    ncall = len(per[0])
    assert all(len(p) == ncall for p in per)
    ws = []
    for c in range(ncall):
        cnt = per[0][c][1]
        assert all(p[c][1] == cnt for p in per)
        ws.append(b.step([p[c][0] for p in per], cnt, wrench=True))
    return ws


def _same(a, b):
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), f


def test_batch_equals_alone(tl):
    scenes = _scenes()
    K = 25
    _print_case("batch_equals_alone", n=[s["X"].shape[0] for s in scenes], steps=K)
    alone = []
    for s in scenes:
        g, ws = _run_alone(tl, s, 0, K)
        assert g.status() == 0
        alone.append((g.read(FIELDS), ws))
        g.close()
    gs = [tl.Scene(s) for s in scenes]
    with tl.Batch(gs) as b:
        wsb = _run_batch(tl, b, scenes, 0, K)
    for i, g in enumerate(gs):
        assert g.status() == 0
        _same(g.read(FIELDS), alone[i][0])
        for c in range(len(wsb)):
            assert np.array_equal(wsb[c][i], alone[i][1][c]), (i, c)
    # the cuts did something
    assert any(np.any(a[0]["code"] != 0) for a in alone)


def _split(scene, j0, j1):
    """Calls for steps [j0, j1) of a batch scene (tools at constant velocity): one
    substep, then the rest in one call."""
    adv = lambda tools: [dict(t, advance=True) for t in tools]
    return [(adv(scene["tools_at"](j0)), 1), (adv(scene["tools_at"](j0 + 1)), j1 - j0 - 1)]


def test_batch_joins_running_and_fresh_scenes(tl):
    """A scene already stepped alone (pending F update, other slot-table buffer)
    joins a batch with fresh scenes; each continues exactly as alone."""
    scenes = _scenes()[:3]
    K0, K1 = 7, 16
    _print_case("batch_joins", steps=(K0, K1))
    starts = [K0, 0, 0]
    ref = []
    for s, j0 in zip(scenes, starts):
        g = tl.Scene(s)
        if j0:
            _run_alone(tl, s, 0, j0, g)
        for tools, cnt in _split(s, j0, j0 + K1):
            g.step(tools, cnt)
        ref.append(g.read(FIELDS))
        g.close()
    g0, _ = _run_alone(tl, scenes[0], 0, K0)
    gs = [g0] + [tl.Scene(s) for s in scenes[1:]]
    per = [_split(s, j0, j0 + K1) for s, j0 in zip(scenes, starts)]
    with tl.Batch(gs) as b:
        for c in range(2):
            b.step([p[c][0] for p in per], per[0][c][1])
    for g, r in zip(gs, ref):
        _same(g.read(FIELDS), r)


def test_batch_membership_rules(tl):
    scenes = _scenes()[:2]
    gs = [tl.Scene(s) for s in scenes]
    b = tl.Batch(gs)
    with pytest.raises(tl.TlmpmError) as e:
        gs[0].step([], 1)
    assert e.value.code == tl.E_INVALID
    with pytest.raises(tl.TlmpmError):
        tl.Batch([gs[1]])
    b.close()
    gs[0].step([], 1)
    with pytest.raises(tl.TlmpmError):
        tl.Batch([gs[0], gs[0]])


def test_batch_isolates_a_failing_scene(tl):
    """A state with det F < 0 written into one member makes that scene report
    TLMPM_E_NONFINITE; its batch-mates run on and equal their runs alone bitwise."""
    scenes = _scenes()[:3]
    K = 10
    _print_case("batch_isolates_failure", n=[s["X"].shape[0] for s in scenes], steps=K)
    alone = {}
    for i in (0, 2):
        g, ws = _run_alone(tl, scenes[i], 0, K)
        assert g.status() == 0
        alone[i] = g.read(FIELDS)
        g.close()
    gs = [tl.Scene(s) for s in scenes]
    n1 = scenes[1]["X"].shape[0]
    F = np.tile(np.eye(3, dtype=np.float32), (n1, 1, 1))
    F[n1 // 2] = -np.eye(3)
    gs[1].write(F=F)
    with tl.Batch(gs) as b:
        _run_batch(tl, b, scenes, 0, K)
    assert gs[1].status() == tl.E_NONFINITE
    for i in (0, 2):
        assert gs[i].status() == 0
        _same(gs[i].read(FIELDS), alone[i])


def test_batch_equals_alone_with_split_bricks(tl):
    """Scenes of 512+ bricks run their mixed bricks' later rounds in workgroups of
    their own, alone and in a batch (with a small scene that does not): the batch
    still equals the runs alone bitwise."""
    scenes = [W.batch_scene(11, 0, 280000, steps=40), W.batch_scene(11, 1, 4000, steps=40),
              W.batch_scene(11, 2, 320000, steps=40)]
    K = 20
    _print_case("batch_split", n=[s["X"].shape[0] for s in scenes], steps=K)
    alone = []
    for s in scenes:
        g, ws = _run_alone(tl, s, 0, K)
        assert g.status() == 0
        alone.append(g.read(FIELDS))
        g.close()
    gs = [tl.Scene(s) for s in scenes]
    with tl.Batch(gs) as b:
        _run_batch(tl, b, scenes, 0, K)
    for i, g in enumerate(gs):
        assert g.status() == 0, i
        _same(g.read(FIELDS), alone[i])
