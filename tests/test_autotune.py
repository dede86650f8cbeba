"""The autotuner's search and cache (CPU: the trial timing is replaced by a cost
function of the setting)."""
import json

from paper_2609_27342_amd import autotune


def test_coordinate_descent_finds_the_cheapest_choice_and_caches_it(tmp_path, monkeypatch):
    cost = {"pair_div": {128: 3.0, 64: 1.0, 256: 4.0, 512: 5.0},  # margins far above the 2 % noise bound
            "pair_cap": {4096: 2.0, 1024: 3.0, 2048: 0.5, 8192: 2.5},
            "split": {"default": 1.0, "off": 0.25, "wide": 2.0},
            "one_stream_bricks": {2048: 1.0, 0: 1.5, 1 << 30: 1.0}}
    calls = []

    def fake(choice, make, step, steps, warmup, repeats=3):
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


def test_equal_launch_shapes_are_timed_once_and_small_gains_are_noise(monkeypatch):
    import numpy as np
    from paper_2609_27342_amd import workloads as W
    sc = W.box_scene(n_cells=(8, 8, 8), dx=0.01, material_contact=1)  # 4096 particles, 8 bricks
    calls = []

    def fake(choice, make, step, steps, warmup, repeats=3):
        calls.append(dict(choice))
        return 1.0 - 0.01 * (choice["pair_div"] == 64), 0  # 1 % faster: within the margin

    monkeypatch.setattr(autotune, "time_setting", fake)
    best, trials, _ = autotune.tune("w", None, None, cache=None, scene_dicts=[sc], single=True)
    assert best == {k: v[0] for k, v in autotune.KNOBS.items()}
    # 4096 particles: pair_div 128 -> 32 blocks, 64 -> 64, 256 -> 16, 512 -> 8 (4 shapes); the pair cap,
    # the split range (8 bricks) and the one-stream threshold (0 vs 2048 bricks) give 1 + 1 more
    assert len(calls) == 5 and len(trials) == 1 + sum(len(v) - 1 for v in autotune.KNOBS.values())
