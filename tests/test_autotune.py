"""The autotuner's search and cache (CPU: the trial timing is replaced by a cost
function of the setting)."""
import json

from paper_2609_27342_amd import autotune


def test_coordinate_descent_finds_the_cheapest_choice_and_caches_it(tmp_path, monkeypatch):
    cost = {"pair_div": {128: 3.0, 64: 1.0, 256: 4.0, 512: 5.0},
            "pair_cap": {4096: 2.0, 1024: 3.0, 2048: 0.5, 8192: 2.5},
            "split": {"default": 1.0, "off": 0.25, "wide": 2.0},
            "one_stream_bricks": {2048: 1.0, 0: 1.5, 1 << 30: 1.0}}
    calls = []

    def fake(choice, make, step, steps, warmup):
        calls.append(dict(choice))
        return sum(cost[k][v] for k, v in choice.items()), 0

    monkeypatch.setattr(autotune, "time_setting", fake)
    cache = str(tmp_path / "cache.json")
    best, trials, src = autotune.tune("w", None, None, cache=cache)
    assert src == "tuned"
    assert best == {"pair_div": 64, "pair_cap": 2048, "split": "off", "one_stream_bricks": 2048}
    assert len(trials) == len(calls) == 1 + sum(len(v) - 1 for v in autotune.KNOBS.values())
    rec = json.load(open(cache))["w"]
    assert rec["choice"] == best and abs(rec["ms_per_substep"] - 2.75) < 1e-12
    calls.clear()
    best2, trials2, src2 = autotune.tune("w", None, None, cache=cache)
    assert src2 == "cache" and best2 == best and not calls
    best3, _, src3 = autotune.tune("w", None, None, cache=cache, force=True)
    assert src3 == "tuned" and best3 == best and calls


def test_settings_of_choices_are_valid_tunings():
    for v in autotune.SPLIT:
        s = autotune.setting_of({"pair_div": 64, "split": v})
        assert s["pair_div"] == 64 and s["split_hi"] >= s["split_lo"] >= 0 and s["split_div"] >= 1


def test_signature_counts_scenes_particles_and_contact():
    import numpy as np
    sc = {"X": np.zeros((1234567, 3), np.float32), "params": {"material_contact": 1}}
    assert autotune.signature([sc, sc]) == "2x2470000-contact1-stencil0"
