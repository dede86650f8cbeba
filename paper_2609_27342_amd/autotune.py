"""Autotuner of the launch-shape settings (tlmpm_set_tuning).

A workload is given as two functions: make() builds its tlmpm.Scene objects (under
the setting in force) and step(scenes, j0, j1) advances them over substeps
[j0, j1).  Each trial sets a candidate, builds the scenes, runs `warmup` untimed
substeps and times `steps` substeps by the wall clock between two device
synchronisations (the fastest of a few such stretches); the scenes are then
freed.  The search is coordinate descent
from the defaults: each knob in turn takes each of its values with the others at
the best so far, and keeps the fastest.  Results are cached in a JSON file keyed
by the workload's signature, so a later run takes the stored setting without
timing again.  Settings that give every scene the same launch shape are timed once,
and a candidate must beat the best by more than a noise margin.

The settings divide work among workgroups and streams; the physics does not
depend on them (splitting mixed bricks changes the rounding of their sums only).
"""
import json
import os
import time

import numpy as np

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


def active_bricks(scene):
    """Bricks (4x4x4 reference cells) holding a particle of a scene dict."""
    p = scene["params"]
    c = np.floor((scene["X"].astype(np.float64) - np.asarray(p["origin"])) / p["dx"]).astype(np.int64) >> 2
    return int(np.unique(c[:, 0] + (c[:, 1] << 20) + (c[:, 2] << 40)).shape[0])


def scene_info(scene_dicts):
    """(particles, active bricks, material contact) of each scene dict."""
    return [(int(sc["X"].shape[0]), active_bricks(sc), bool(sc["params"].get("material_contact")))
            for sc in scene_dicts]


def effective(choice, info, single):
    """The launch shape a setting gives each scene (info: scene_info()): pair-search
    workgroups, extra split workgroups and (a single scene) the one-stream
    arrangement.  Settings with equal shapes launch the same work and are timed
    once."""
    t = dict(SPLIT["default"], pair_div=128, pair_cap=4096, one_stream_bricks=2048)
    t.update(setting_of(choice))
    out = []
    for n, na, contact in info:
        pb = min(t["pair_cap"], max(1, n // t["pair_div"])) if contact else 0
        xc = min(t["split_cap"], na // t["split_div"]) if t["split_lo"] <= na <= t["split_hi"] else 0
        out.append((pb, xc, bool(single and na <= t["one_stream_bricks"])))
    return tuple(out)


def time_setting(choice, make, step, steps, warmup, repeats=3):
    """ms per substep of the workload with the setting `choice`: the fastest of
    `repeats` timed stretches of `steps` substeps after `warmup` substeps."""
    import torch
    tlmpm.set_tuning(None)
    tlmpm.set_tuning(**setting_of(choice))
    scenes = make()
    try:
        step(scenes, 0, warmup)
        best = None
        j = warmup
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            step(scenes, j, j + steps)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            best = ms if best is None else min(best, ms)
            j += steps
        status = max(g.status() for g in scenes)
    finally:
        for g in scenes:
            g.close()
        tlmpm.set_tuning(None)
    return best, status


def tune(key, make, step, knobs=None, steps=20, warmup=5, cache=DEFAULT_CACHE, force=False, log=None,
         scene_dicts=None, single=False, margin=0.02):
    """Best setting of the workload `key` (signature()): from the cache, or by
    coordinate descent over `knobs` (default KNOBS).  A candidate replaces the best
    only when faster by more than `margin` (run-to-run noise); with scene_dicts,
    candidates whose launch shape (effective()) equals one already timed reuse that
    time.  Returns (choice, trials, source) with trials [(choice, ms per substep)];
    stores new results in the cache."""
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
    by_shape = {}
    info = scene_info(scene_dicts) if scene_dicts is not None else None

    def measure(choice):
        tag = json.dumps(choice, sort_keys=True)
        if tag not in seen:
            shape = effective(choice, info, single) if info is not None else tag
            if shape in by_shape:
                seen[tag] = by_shape[shape]
                if log:
                    log(f"[tune] {key} {choice}: same launch shape as a setting timed before")
            else:
                ms, st = time_setting(choice, make, step, steps, warmup)
                if st != 0:
                    raise RuntimeError(f"status {st} under tuning {choice}")
                seen[tag] = by_shape[shape] = ms
                if log:
                    log(f"[tune] {key} {choice}: {ms:.4f} ms/substep")
        return seen[tag]

    best_ms = measure(best)
    for k, values in knobs.items():
        for v in values[1:]:
            c = dict(best, **{k: v})
            ms = measure(c)
            if ms < best_ms * (1.0 - margin):
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


__all__ = ["KNOBS", "SPLIT", "signature", "setting_of", "active_bricks", "scene_info", "effective", "time_setting",
           "tune", "apply", "DEFAULT_CACHE"]
