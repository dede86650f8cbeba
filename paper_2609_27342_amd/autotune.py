"""Autotuner of the launch-shape settings (tlmpm_set_tuning).

A workload is given as two functions: make() builds its tlmpm.Scene objects (under
the setting in force) and step(scenes, j0, j1) advances them over substeps
[j0, j1).  Each trial sets a candidate, builds the scenes, runs `warmup` untimed
substeps and times `steps` substeps by the wall clock between two device
synchronisations; the scenes are then freed.  The search is coordinate descent
from the defaults: each knob in turn takes each of its values with the others at
the best so far, and keeps the fastest.  Results are cached in a JSON file keyed
by the workload's signature, so a later run takes the stored setting without
timing again.

The settings divide work among workgroups and streams; the physics does not
depend on them (splitting mixed bricks changes the rounding of their sums only).
"""
import json
import os
import time

from . import tlmpm

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")

# knob -> values tried (the default first)
KNOBS = {
    "pair_div": (128, 64, 256, 512),
    "pair_cap": (4096, 1024, 2048, 8192),
    "split": ("default", "off", "wide"),
    "one_stream_bricks": (2048, 0, 1 << 30),
}

SPLIT = {  # split_lo, split_hi, split_div, split_cap
    "default": dict(split_lo=512, split_hi=4096, split_div=4, split_cap=256),
    "off": dict(split_lo=512, split_hi=4096, split_div=4, split_cap=0),
    "wide": dict(split_lo=128, split_hi=1 << 30, split_div=4, split_cap=1024),
}


def signature(scene_dicts):
    """Cache key of a workload: scene count, total particles (3 significant digits),
    material contact, stencil."""
    n = sum(int(s["X"].shape[0]) for s in scene_dicts)
    mc = any(s["params"].get("material_contact") for s in scene_dicts)
    st = max(int(s["params"].get("stencil", 0)) for s in scene_dicts)
    return f"{len(scene_dicts)}x{float(f'{n:.3g}'):.0f}-contact{int(bool(mc))}-stencil{st}"


def setting_of(choice):
    """tlmpm_tuning fields of a knob choice {knob: value}."""
    out = {}
    for k, v in choice.items():
        if k == "split":
            out.update(SPLIT[v])
        else:
            out[k] = int(v)
    return out


def time_setting(choice, make, step, steps, warmup):
    """ms per substep of the workload with the setting `choice`."""
    import torch
    tlmpm.set_tuning(None)
    tlmpm.set_tuning(**setting_of(choice))
    scenes = make()
    try:
        step(scenes, 0, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step(scenes, warmup, warmup + steps)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        status = max(g.status() for g in scenes)
    finally:
        for g in scenes:
            g.close()
        tlmpm.set_tuning(None)
    return ms, status


def tune(key, make, step, knobs=None, steps=20, warmup=5, cache=DEFAULT_CACHE, force=False, log=None):
    """Best setting of the workload `key` (signature()): from the cache, or by
    coordinate descent over `knobs` (default KNOBS).  Returns (choice, trials, source)
    with trials [(choice, ms per substep)]; stores new results in the cache."""
    knobs = dict(knobs or KNOBS)
    store = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            store = json.load(fh)
    if not force and key in store:
        rec = store[key]
        return rec["choice"], [(c, ms) for c, ms in rec["trials"]], "cache"
    best = {k: v[0] for k, v in knobs.items()}
    seen = {}

    def measure(choice):
        tag = json.dumps(choice, sort_keys=True)
        if tag not in seen:
            ms, st = time_setting(choice, make, step, steps, warmup)
            if st != 0:
                raise RuntimeError(f"status {st} under tuning {choice}")
            seen[tag] = ms
            if log:
                log(f"[tune] {key} {choice}: {ms:.4f} ms/substep")
        return seen[tag]

    best_ms = measure(best)
    for k, values in knobs.items():
        for v in values[1:]:
            c = dict(best, **{k: v})
            ms = measure(c)
            if ms < best_ms:
                best, best_ms = c, ms
    trials = [(json.loads(t), ms) for t, ms in seen.items()]
    if cache:
        store[key] = {"choice": best, "ms_per_substep": best_ms, "trials": trials, "steps": steps,
                      "warmup": warmup}
        with open(cache, "w") as fh:
            json.dump(store, fh, indent=1, sort_keys=True)
    return best, trials, "tuned"


def apply(choice):
    """Sets the tuning of `choice` for the scenes created from now on."""
    tlmpm.set_tuning(None)
    tlmpm.set_tuning(**setting_of(choice))


__all__ = ["KNOBS", "SPLIT", "signature", "setting_of", "time_setting", "tune", "apply", "DEFAULT_CACHE"]
