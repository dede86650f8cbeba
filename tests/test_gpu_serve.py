"""Continuous batching: rollouts that join and leave a running batch end exactly
as the same requests stepped alone with the same ticks."""
import numpy as np
import pytest

from paper_2609_27342_amd import workloads as W

pytestmark = pytest.mark.gpu

TICK = 50


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_27342_amd import tlmpm
    tlmpm.lib()
    return tlmpm


def _build(r):
    return W.served_request(r["seed"], r["index"], r["n_target"], r["horizon"], r["tick"])


def test_served_rollouts_equal_alone(tl):
    from paper_2609_27342_amd import serve
    reqs = W.served(seed=7, n_requests=6, n_range=(2500, 8000), horizon_s=(0.01, 0.03), tick=TICK)
    sds = [_build(r) for r in reqs]
    fp = [tl.footprint(s) for s in sds]
    # room for about three rollouts at a time: requests join and leave mid-flight
    budget = sum(sorted(fp)[-3:]) + 1
    print(f"[case] served n={[s['X'].shape[0] for s in sds]} horizons={[r['horizon'] for r in reqs]}", flush=True)
    srv = serve.Server(_build, budget, tick=TICK, read_fields=("u", "v", "F", "D", "digits"))
    stats = srv.run(reqs, realtime=False)
    assert stats["requests"] == len(reqs)
    assert stats["mean_batch"] > 1.0
    for r, sd in zip(reqs, sds):
        g = tl.Scene(sd)
        for j in range(0, r["horizon"], TICK):
            g.step([dict(t, advance=True) for t in sd["tools_at"](j)], TICK)
        ref = g.read(("u", "v", "F", "D", "digits"))
        got = srv.results[r["index"]]
        assert got["status"] == 0 and g.status() == 0
        for f in ref:
            assert np.array_equal(got["fields"][f], ref[f]), (r["index"], f)
        g.close()


def test_admission_budget_and_refusal(tl):
    """Admission holds the running rollouts' scene workspaces plus their bounds on
    the batch workspace within the budget (the batch the loop builds fits what was
    reserved, checked inside the loop); a request larger than the whole budget is
    refused with TLMPM_E_NOMEM, and the others are served."""
    from paper_2609_27342_amd import serve
    reqs = W.served(seed=8, n_requests=5, n_range=(2500, 6000), horizon_s=(0.01, 0.02), tick=TICK)
    big = W.served(seed=9, n_requests=1, n_range=(60000, 60000), horizon_s=(0.01, 0.01), tick=TICK)[0]
    big = dict(big, index=99, arrival=reqs[1]["arrival"])
    sds = {r["index"]: _build(r) for r in reqs + [big]}
    need = {i: serve.request_bytes(sd) for i, sd in sds.items()}
    budget = sum(sorted(need[r["index"]] for r in reqs)[-2:]) + 1  # two small rollouts at a time
    assert need[99] > budget
    print(f"[case] admission budget={budget} bytes={need}", flush=True)
    srv = serve.Server(lambda r: sds[r["index"]], budget, tick=TICK)
    stats = srv.run(reqs + [big], realtime=False)
    assert stats["refused"] == 1 and srv.results[99]["status"] == tl.E_NOMEM
    assert srv.results[99]["fields"] is None
    assert stats["requests"] == len(reqs)
    assert all(srv.results[r["index"]]["status"] == 0 for r in reqs)
    assert 0 < stats["peak_bytes"] <= budget
    # the per-scene bounds cover the batch workspace of any set of these scenes
    gs = [tl.Scene(sds[r["index"]]) for r in reqs]
    with tl.Batch(gs) as b:
        assert b.bytes <= sum(tl.batch_scene_bytes(sds[r["index"]]) for r in reqs)
