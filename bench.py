#!/usr/bin/env python3
"""Throughput benchmark of the TLMPM cutting hot path on one MI355X.

A step is one substep of the whole path: side-label pass of the active blades,
slot-table maintenance, tool/floor/material contact, label-masked P2G, coupling
and grid update, G2P, MUSL re-scatter and the deformation-gradient update.  The
workload is a seeded synthetic scene (paper_2609_27342_amd.workloads) resident in
HBM before timing; tool schedules run as constant-velocity segments.

Default workload: the large box (14.2M particles, three blades cutting from the
first substep), the HBM-bound configuration; the many-scene workload (plain one
scene per call against one batch) is reported beside it in config.batched.

Prints ONE JSON line with particle-steps/s, the roofline of the dominant kernel
(P2G: algorithmic bytes over its duration, timed by HIP events on the scene's
stream around its launches inside the timed region) and the FP64 CPU oracle timed
on a bounded sample of the same workload, on one thread and on all threads.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per particle and launch (FP32 state, each field counted once):
#   P2G kernel: read X 12, code 4, v 12, F 36; write F 36            -> 100 B
#   G2P kernel: read X 12, code 4, u 12, v 12; write u 12, v 12       ->  64 B
#   whole substep (each persistent field read/written once)           -> 136 B
ALG_BYTES = {"p2g": 100, "g2p": 64}
# quadratic stencil: P2G reads X, code, v and F (64 B); the F update is a kernel of its own
ALG_BYTES_QUAD = {"p2g": 64, "g2p": 64}
ALG_STEP_BYTES = 136  # + 4 with per-particle E
DEFAULTS = {"small": (100, 10), "small-deep": (100, 10), "medium": (3000, 300), "large": (100, 10),
            "batched": (100, 10), "knife": (600, 50), "thrown-knives": (300, 20)}
# the part of the large box the CPU baseline runs on: where cuts 0 and 2 cross
LARGE_SAMPLE = ((0.07, 0.13), (0.07, 0.13))


def step_calls(scene, j0, j1):
    """The (tools, n_substeps) calls for steps [j0, j1): the tool schedule is an input
    of the workload, computed before the timed region (in Python it costs ~40 us per
    substep, a third of a medium substep on the GPU)."""
    from paper_2609_27342_amd import workloads as W
    return [([dict(t, advance=True) for t in tools], cnt) for j, cnt, tools in W.segments(scene, j0, j1)]


def run_calls(g, calls):
    for tools, cnt in calls:
        g.step(tools, n_substeps=cnt)


def run_steps(g, scene, j0, j1):
    run_calls(g, step_calls(scene, j0, j1))


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def oracle_rate(scene, threads, budget_s, max_steps=400):
    """(particle-steps/s, substeps) of the FP64 oracle from the first substep of
    `scene`, until about budget_s seconds have been spent."""
    import oracle
    oracle.set_threads(threads)
    o = oracle.OracleScene(scene)
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps and (steps == 0 or time.perf_counter() - t0 < budget_s):
        tools = scene["tools_at"](steps)
        blades = [t["blade"] for t in tools if t["labels"]]
        if blades:
            o.assign_labels(blades)
        o.step([dict(t, contact=int(t["contact"]), cutting=int(t["cutting"])) for t in tools])
        steps += 1
    dt = time.perf_counter() - t0
    return scene["X"].shape[0] * steps / dt, steps


def cpu_baseline(scene, budget_s=10.0, sample=None):
    """The FP64 oracle as it stands on a bounded sample of the same workload (the
    whole scene, or the particles of `sample` = (x range, y range)), from its first
    substep: one thread, then all threads (OpenMP over the loops with independent
    iterations; the results do not depend on the thread count)."""
    from paper_2609_27342_amd import workloads as W
    sc = W.crop(scene, *sample) if sample else scene
    n = sc["X"].shape[0]
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    v1, s1 = oracle_rate(sc, 1, budget_s)
    va, sa = oracle_rate(sc, threads, budget_s)
    where = (f"particles of {scene['name']} with x in {list(sample[0])} m and y in {list(sample[1])} m "
             f"({n} of {scene['X'].shape[0]}; the same grid, parameters and blades)") if sample else \
        f"{scene['name']} ({n} particles)"
    return {"value": va, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first {sa} substeps of {where}, FP64 C oracle, {threads} OpenMP threads",
            "single_thread": {"value": v1, "cores": 1, "substeps": s1},
            "nproc": os.cpu_count(), "cpu_model": cpu_info()}


def kernel_source_hash():
    """First 16 hex digits of the sha256 of the kernel sources (the key under which
    measured hardware traffic is stored in profiles/traffic.json)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("tlmpm_common.h", "tlmpm_device.h", "tlmpm_band.h", "tlmpm_reach.h", "tlmpm_kernels.hip",
              "tlmpm_contact.hip", "tlmpm_quad.hip", "tlmpm_surface.hip"):
        with open(os.path.join(ROOT, "paper_2609_27342_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, cls):
    """HBM bytes per launch of a kernel class from the committed rocprofv3 counter
    summary, or None when it was taken on other kernel sources or workloads."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_hash") != kernel_source_hash():
        return None
    rec = t.get("workloads", {}).get(workload, {}).get(cls)
    return rec["bytes"] if rec else None


def roofline_of(prof, value, n, step_bytes, own=None, workload=None):
    """Roofline of the dominant kernel (P2G or G2P by summed duration) from event
    timings {class: (ms, launches)}: achieved = step_bytes (the substep's
    algorithmic bytes per particle, each persistent field read or written once)
    times the N particles one launch covers, over the kernel's average launch
    duration.  `own`: the kernel's own algorithmic bytes per particle, reported
    beside it."""
    own = own or ALG_BYTES
    kern = {k: {"ms_avg": (v[0] / v[1]) if v[1] else None, "launches": v[1]} for k, v in prof.items()}
    dom = max(("p2g", "g2p"), key=lambda k: prof[k][0])
    avg_s = prof[dom][0] / prof[dom][1] * 1e-3
    achieved = step_bytes * n / avg_s / 1e9
    own_gbs = {k: own[k] * n / (prof[k][0] / prof[k][1] * 1e-3) / 1e9 for k in ("p2g", "g2p") if prof[k][1]}
    return {"bound": "hbm", "kernel": "k_" + dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(workload, dom) if workload else None,
            "alg_bytes_per_launch": step_bytes * n, "alg_bytes_per_particle": step_bytes,
            "own_bytes_per_particle": {k: own[k] for k in own},
            "own_frac": {k: v / HBM_PEAK_GBS for k, v in own_gbs.items()},
            "step_alg_frac": value * step_bytes / (HBM_PEAK_GBS * 1e9), "kernels": kern}


def batch_calls(scene, j0, j1):
    """(tools, n_substeps) calls for steps [j0, j1) of a many-scene workload scene:
    its tools move at constant velocity and start their cuts at step 0."""
    adv = [dict(t, advance=True) for t in scene["tools_at"](j0)]
    if j0 == 0 and j1 > 1:
        return [(adv, 1)] + batch_calls(scene, 1, j1)
    return [(adv, j1 - j0)] if j1 > j0 else []


def bench_batched(args, K, Wm, cpu=True):
    """The many-scene workload stepped (a) one scene at a time, each scene's K
    substeps in one call, and (b) as one batch, every launch covering all scenes."""
    import torch
    from paper_2609_27342_amd import tlmpm, workloads as W
    B = W.batched()
    scenes = B["scenes"]
    n = sum(s["X"].shape[0] for s in scenes)
    torch.cuda.set_device(0)
    tuning = tuned(args, "batched", scenes, True) if args.tune else None
    print(f"[bench] workload=batched scenes={len(scenes)} n={n} warmup={Wm} steps={K}", file=sys.stderr, flush=True)

    def fresh():
        return [tlmpm.Scene(s) for s in scenes]

    # (a) plain
    gs = fresh()
    for g, s in zip(gs, scenes):
        for tools, cnt in batch_calls(s, 0, Wm):
            g.step(tools, cnt)
    plan = [batch_calls(s, Wm, Wm + K) for s in scenes]  # the tool schedule, before timing
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g, calls in zip(gs, plan):
        for tools, cnt in calls:
            g.step(tools, cnt)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    status_plain = max(g.status() for g in gs)
    for g in gs:
        g.close()
    del gs
    print(f"[bench] plain: {t_plain * 1e3 / K:.4f} ms/step", file=sys.stderr, flush=True)

    # (b) batched
    gs = fresh()
    bt = tlmpm.Batch(gs)
    bt.graphs(args.graphs)

    def plan_of(j0, j1):
        return [batch_calls(s, j0, j1) for s in scenes]

    def run(per):
        for c in range(len(per[0])):
            bt.step([p[c][0] for p in per], per[0][c][1])

    run(plan_of(0, Wm))
    per = plan_of(Wm, Wm + K)
    bt.profile("transfers")  # events around the P2G and G2P launches of the timed region
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(per)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    prof = bt.profile_read()
    bt.profile(False)
    bt.close()
    status = max(g.status() for g in gs)
    contact = contact_of(gs)
    if tuning is not None:
        tlmpm.set_tuning(None)
    value = n * K / t_batch
    plain_value = n * K / t_plain
    print(f"[bench] batched: {t_batch * 1e3 / K:.4f} ms/step, status={status}", file=sys.stderr, flush=True)
    cpu_b = None
    if cpu and not args.no_cpu_baseline:
        cpu_b = cpu_baseline(scenes[0])
        cpu_b["sample"] = "scene 0 of the batch: " + cpu_b["sample"]
    for g in gs:
        g.close()
    return {
        "metric": "particle-steps/s per GPU",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": t_batch * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched", "scenes": len(scenes), "particles": n, "dt": scenes[0]["params"]["dt"],
                   "material_contact": True, "path": "batched+graph" if args.graphs else "batched",
                   "plain": {"value": plain_value, "ms_per_step": t_plain * 1e3 / K, "status": status_plain},
                   "batched_over_plain": value / plain_value, "tuning": tuning, "contact": contact},
        "status": status,
        "roofline": roofline_of(prof, value, n, ALG_STEP_BYTES, None, "batched"),
        "cpu_baseline": cpu_b,
    }


def bench_knife(args, K, Wm):
    """Two-way coupled knife (free rigid knife on a soft block): every interval the
    knife's tool record is held over `interval` substeps, the interval-averaged
    wrench comes back to the host and advances the knife; the timed region includes
    those round trips."""
    import torch
    from paper_2609_27342_amd import tlmpm, workloads as W
    from paper_2609_27342_amd.coupling import KnifeRollout
    torch.cuda.set_device(0)
    sc = W.knife() if args.workload == "knife" else W.thrown_knives()
    n = sc["X"].shape[0]
    iv = sc["knife"]["interval"] if "knife" in sc else sc["knives"]["interval"]
    g = tlmpm.Scene(sc)
    g.graphs(args.graphs)
    ro = KnifeRollout(g, sc)
    ro.advance(max(1, Wm // iv))
    torch.cuda.synchronize()
    ki = max(1, K // iv)
    t0 = time.perf_counter()
    ro.advance(ki)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    steps = ki * iv
    value = n * steps / (t1 - t0)
    status = g.status()
    P = max(1, min(args.profile_steps, K) // iv)
    g.profile(True)
    ro.advance(P)
    prof = g.profile_read()
    g.profile(False)
    ends = [b.state() for b in ro.bodies]
    mass = sc["knife"]["body"]["mass"] if "knife" in sc else [k["body"]["mass"] for k in sc["knives"]["bodies"]]
    return {
        "metric": "particle-steps/s per GPU",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": max(1, Wm // iv) * iv,
        "ms_per_step": (t1 - t0) * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "particles": n, "dt": sc["params"]["dt"], "interval": iv,
                   "material": sc["params"].get("material", 0), "yield_stress": sc["params"].get("yield_stress", 0.0),
                   "knife_mass": mass, "path": "graph" if args.graphs else "plain",
                   "knife_end": [{"x": st["x"].tolist(), "v": st["v"].tolist(), "omega": st["omega"].tolist()}
                                 for st in ends]},
        "status": status,
        "roofline": roofline_of(prof, value, n, ALG_STEP_BYTES + material_extra_bytes(sc["params"]),
                                dict(ALG_BYTES, p2g=ALG_BYTES["p2g"] + material_extra_bytes(sc["params"]))),
        "cpu_baseline": None,
    }


def material_extra_bytes(params):
    """P2G bytes per particle beyond the Neo-Hookean path: the plastic state F_p^-1
    read (36 B; written only where the particle yields), the viscous rate Fdot read
    and written (72 B)."""
    extra = 0
    if params.get("material", 0) == 1 and params.get("yield_stress", 0.0) > 0.0:
        extra += 36
    if params.get("material", 0) == 1 and params.get("viscosity", 0.0) > 0.0:
        extra += 72
    return extra


def served_roofline(kernel_time, value):
    """Roofline of the served loop's dominant kernel over every batch it ran:
    achieved = substep algorithmic bytes x (particles x launches) summed over the
    batches, over the summed launch durations (HIP events, mode 2)."""
    if not kernel_time:
        return None
    dom = max(("p2g", "g2p"), key=lambda k: kernel_time.get(k, [0.0])[0])
    ms, launches, pl = kernel_time[dom]
    achieved = ALG_STEP_BYTES * pl / (ms * 1e-3) / 1e9
    own = {k: ALG_BYTES[k] * kernel_time[k][2] / (kernel_time[k][0] * 1e-3) / 1e9 / HBM_PEAK_GBS
           for k in ("p2g", "g2p") if k in kernel_time and kernel_time[k][0] > 0}
    return {"bound": "hbm", "kernel": "k_" + dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "alg_bytes_per_launch": ALG_STEP_BYTES * pl / max(1, launches), "alg_bytes_per_particle": ALG_STEP_BYTES,
            "own_frac": own, "step_alg_frac": value * ALG_STEP_BYTES / (HBM_PEAK_GBS * 1e9),
            "kernels": {k: {"ms_avg": v[0] / v[1] if v[1] else None, "launches": v[1]} for k, v in kernel_time.items()}}


def served_run(args, reqs, log=None, realtime=True):
    """One served run of `reqs` (warm kernels and allocator first); returns
    (server, stats) with P2G/G2P launch timings collected."""
    import torch
    from paper_2609_27342_amd import serve, workloads as W
    build = lambda r: W.served_request(r["seed"], r["index"], r["n_target"], r["horizon"], r["tick"])
    warm = W.served(seed=6, n_requests=1, n_range=(20000, 20000), horizon_s=(0.02, 0.02), tick=args.tick)
    serve.Server(build, args.budget_gb * 1e9, tick=args.tick).run(warm, realtime=False)
    torch.cuda.synchronize()
    srv = serve.Server(build, args.budget_gb * 1e9, tick=args.tick, profile=True)
    st = srv.run(reqs, realtime=realtime, log=log)
    return srv, st


def served_summary(srv, st, reqs, rate):
    """The served figures of one run: latency from arrival to result (p50, p99),
    queueing before admission, throughput, batch sizes, admission."""
    from paper_2609_27342_amd import tlmpm
    res = [srv.results[r["index"]] for r in reqs]
    done = [r for r in res if r["status"] != tlmpm.E_NOMEM]
    wait = np.array([r["admitted"] - r["arrival"] for r in done]) if done else np.zeros(0)
    lat = np.array([r["done"] - r["arrival"] for r in done]) if done else np.zeros(0)
    work = np.array([r["n"] * r["steps"] for r in res], np.float64)
    return {"requests": len(reqs), "completed": st["requests"], "refused": st["refused"],
            "rate_per_s": rate, "arrival_span_s": reqs[-1]["arrival"] if reqs else 0.0,
            "latency_s": {"p50": st["p50_s"], "p99": st["p99_s"], "mean": float(lat.mean()) if len(lat) else None,
                          "max": float(lat.max()) if len(lat) else None},
            "queue_wait_s": {"p50": float(np.percentile(wait, 50)) if len(wait) else None,
                             "p99": float(np.percentile(wait, 99)) if len(wait) else None},
            "throughput": st["throughput"], "wall_s": st["wall_s"], "iterations": st["iterations"],
            "mean_batch": st["mean_batch"], "peak_bytes": int(st["peak_bytes"]),
            "particles": {"mean": float(np.mean([r["n"] for r in res])), "max": int(max(r["n"] for r in res))},
            "horizon_substeps": {"mean": float(np.mean([r["steps"] for r in res])),
                                 "min": int(min(r["steps"] for r in res)), "max": int(max(r["steps"] for r in res))},
            "capacity_requests_per_s": st["throughput"] / float(work.mean()),
            "status": max((r["status"] for r in done), default=0),
            "failed": [{"index": q["index"], "status": r["status"], "detail": r.get("detail", ""), "n": r["n"],
                        "steps": r["steps"]} for q, r in zip(reqs, res)
                       if r["status"] not in (0, tlmpm.E_NOMEM)]}


def bench_served(args):
    """Continuous batching of arriving rollouts (Poisson arrivals, log-uniform
    particle counts, horizons U[0.5, 2] s, HBM-budget admission); latency from
    arrival to result.  --capacity-frac F first measures the capacity (requests/s)
    with the first --capacity-requests requests all queued at once, then serves
    --requests arrivals at F times that rate."""
    import torch
    from paper_2609_27342_amd import workloads as W
    torch.cuda.set_device(0)
    log = (lambda m: print(m, file=sys.stderr, flush=True)) if args.verbose else None
    rate = args.rate
    capacity = None
    if args.capacity_frac:
        probe = W.served(seed=args.served_seed, n_requests=args.capacity_requests, rate=args.rate, tick=args.tick)
        srv, st = served_run(args, probe, log, realtime=False)
        capacity = served_summary(srv, st, probe, None)
        rate = args.capacity_frac * capacity["capacity_requests_per_s"]
        print(f"[bench] capacity {capacity['capacity_requests_per_s']:.3f} requests/s from {len(probe)} queued "
              f"requests; serving at {rate:.3f}/s", file=sys.stderr, flush=True)
    reqs = W.served(seed=args.served_seed + (1 if args.capacity_frac else 0), n_requests=args.requests, rate=rate,
                    tick=args.tick)
    print(f"[bench] served: {len(reqs)} requests at {rate:.3f}/s, tick {args.tick}", file=sys.stderr, flush=True)
    srv, st = served_run(args, reqs, log)
    sm = served_summary(srv, st, reqs, rate)
    print(f"[bench] served: p50 {sm['latency_s']['p50']:.2f} s p99 {sm['latency_s']['p99']:.2f} s "
          f"throughput {sm['throughput']:.3e} wall {sm['wall_s']:.1f} s", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        r0 = reqs[0]
        sd = W.served_request(r0["seed"], r0["index"], r0["n_target"], r0["horizon"], r0["tick"])
        cpu = cpu_baseline(sd)
        cpu["sample"] = "request 0 of the stream: " + cpu["sample"]
    cfg = {"workload": "served", "tick": args.tick, "budget_gb": args.budget_gb, "path": "served",
           "horizon_s": [0.5, 2.0], "n_range": [10000, 1000000]}
    cfg.update(sm)
    if capacity is not None:
        cfg["capacity_probe"] = {k: capacity[k] for k in ("requests", "throughput", "wall_s", "mean_batch",
                                                           "capacity_requests_per_s")}
        cfg["capacity_frac"] = args.capacity_frac
    return {
        "metric": "particle-steps/s per GPU",
        "value": st["throughput"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": int(st["iterations"]),
        "warmup": 1,
        "ms_per_step": st["wall_s"] * 1e3 / max(1, st["iterations"]),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": cfg,
        "status": sm["status"],
        "roofline": served_roofline(srv.kernel_time, st["throughput"]),
        "cpu_baseline": cpu,
    }


def contact_of(gs):
    """Material-contact search of the last substep summed over scenes: candidates,
    pairs in contact and the pair search's algorithmic bytes (40 B per candidate:
    its record and bucket reads; 24 B per pair: the partner's state)."""
    c = [g.contact_stats() for g in gs]
    cand = sum(x["candidates"] for x in c)
    pairs = sum(x["pairs"] for x in c)
    skipped = sum(x["skipped"] for x in c)
    return {"candidates": cand, "pairs": pairs, "searches_skipped": skipped,
            "pair_search_alg_bytes": 40 * cand + 24 * pairs}


def bench_scene(args, name, scene, K, Wm):
    """One scene stepped K substeps after Wm untimed ones; returns (figures,
    event timings of the P2G and G2P launches in the timed region)."""
    import torch
    from paper_2609_27342_amd import tlmpm
    n = scene["X"].shape[0]
    g = tlmpm.Scene(scene)
    g.graphs(args.graphs)
    print(f"[bench] workload={name} n={n} warmup={Wm} steps={K} graphs={args.graphs}", file=sys.stderr, flush=True)
    run_steps(g, scene, 0, Wm)
    calls = step_calls(scene, Wm, Wm + K)
    labelled_steps = sum(cnt for tools, cnt in calls if any(t["labels"] for t in tools))
    # HIP events on the scene's stream around the P2G and G2P launches of the timed
    # region (the launch arrangement is unchanged)
    g.profile("transfers")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_calls(g, calls)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.profile_read()
    g.profile(False)
    status = g.status()
    tot_slots, max_slots = g.slot_stats()
    hist = g.slot_histogram()
    contact = contact_of([g])
    g.close()
    print(f"[bench] {name}: {(t1 - t0) * 1e3 / K:.4f} ms/step, status={status}", file=sys.stderr, flush=True)
    quad = scene["params"].get("stencil", 0) == 1
    per_E = scene["E"].min() != scene["E"].max()
    step_bytes = ALG_STEP_BYTES + (4 if per_E else 0)
    own = dict(ALG_BYTES_QUAD if quad else ALG_BYTES)
    own["p2g"] += 4 if per_E else 0
    value = n * K / (t1 - t0)
    fig = {"value": value, "ms_per_step": (t1 - t0) * 1e3 / K, "status": status, "particles": n,
           "timed_substeps": [Wm, Wm + K], "substeps_with_label_pass": labelled_steps,
           "slots": {"total": tot_slots, "max_per_node": max_slots,
                     "nodes_by_slots": {str(c): h for c, h in enumerate(hist) if h and c}},
           "contact": contact,
           "stencil": "quadratic" if quad else "trilinear",
           "roofline": roofline_of(prof, value, n, step_bytes, own, name)}
    return fig


class _BatchRun:
    """A batch of scenes as one object with the status()/close() of a scene (for the
    autotuner's trials)."""

    def __init__(self, scene_dicts):
        from paper_2609_27342_amd import tlmpm
        self.dicts = scene_dicts
        self.gs = [tlmpm.Scene(s) for s in scene_dicts]
        self.bt = tlmpm.Batch(self.gs)

    def status(self):
        # member scenes answer once their batch is gone
        if self.bt is not None:
            self.bt.close()
            self.bt = None
        return max(g.status() for g in self.gs)

    def close(self):
        if self.bt is not None:
            self.bt.close()
            self.bt = None
        for g in self.gs:
            g.close()


def tuned(args, name, scene_dicts, batch):
    """Applies the autotuned launch shape of this workload (cached per signature in
    paper_2609_27342_amd/tuning_cache.json; timed now when absent or with
    --retune).  Returns the record reported in config.tuning."""
    from paper_2609_27342_amd import autotune, tlmpm
    key = f"{name}:" + autotune.signature(scene_dicts)
    if batch:
        def make():
            return [_BatchRun(scene_dicts)]

        def step(objs, j0, j1):
            br = objs[0]
            per = [batch_calls(s, j0, j1) for s in br.dicts]
            for c in range(len(per[0])):
                br.bt.step([p[c][0] for p in per], per[0][c][1])
    else:
        sc = scene_dicts[0]

        def make():
            return [tlmpm.Scene(sc)]

        def step(objs, j0, j1):
            run_steps(objs[0], sc, j0, j1)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    choice, trials, source = autotune.tune(key, make, step, steps=args.tune_steps, warmup=5, force=args.retune,
                                           log=log, scene_dicts=scene_dicts, single=not batch)
    autotune.apply(choice)
    default = {k: v[0] for k, v in autotune.KNOBS.items()}
    ms = {json.dumps(c, sort_keys=True): m for c, m in trials}
    return {"key": key, "choice": choice, "source": source, "setting": tlmpm.get_tuning(),
            "best_ms_per_substep": ms.get(json.dumps(choice, sort_keys=True)),
            "default_ms_per_substep": ms.get(json.dumps(default, sort_keys=True)), "trials": len(trials)}


def bench_scenes(args, W):
    """The scene for --workload: medium starts with the first blade inside the tube
    (z = 0.034 m), so every timed substep cuts."""
    if args.workload == "medium":
        return W.medium(z_start=0.034)
    return W.CONFIGS[args.workload]()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default=os.environ.get("TLMPM_BENCH_WORKLOAD", "large"))
    ap.add_argument("--no-batched", action="store_true", help="large: skip the many-scene run beside it")
    ap.add_argument("--batched-steps", type=int, default=20, help="large: timed substeps of the many-scene run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=200)
    ap.add_argument("--requests", type=int, default=500, help="served: number of requests")
    ap.add_argument("--served-seed", type=int, default=5, help="served: seed of the arrival stream")
    ap.add_argument("--capacity-frac", type=float, default=0.0,
                    help="served: serve at this fraction of the capacity measured first (0: at --rate)")
    ap.add_argument("--capacity-requests", type=int, default=24, help="served: requests of the capacity probe")
    ap.add_argument("--served-requests", type=int, default=40,
                    help="large: requests of the served stream run beside the headline (0: none)")
    ap.add_argument("--no-others", dest="others", action="store_false",
                    help="large: skip the small and medium scenes beside the headline")
    ap.add_argument("--rate", type=float, default=40.0, help="served: Poisson arrival rate per second")
    ap.add_argument("--tick", type=int, default=100, help="served: substeps per batched iteration")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="served: device bytes for running rollouts")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="run the timed scenes under the autotuned launch shape (cached per workload)")
    ap.add_argument("--retune", action="store_true", help="with --tune: time the candidates again")
    ap.add_argument("--tune-steps", type=int, default=20, help="timed substeps per autotuner trial")
    ap.add_argument("--graphs", action="store_true",
                    help="replay pairs of substeps as captured HIP graphs (tlmpm_set_graphs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (5 times) and exit; used to scale "
                         "hardware traffic counters")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        nb = args.copy_calibration
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nb}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 (sharding across GPUs "
                                   "is not implemented)"}))
        sys.exit(2)

    import torch
    from paper_2609_27342_amd import tlmpm, workloads as W

    steps_d, warm_d = DEFAULTS.get(args.workload, (200, 10))
    K = args.steps if args.steps is not None else steps_d
    Wm = args.warmup if args.warmup is not None else warm_d
    if args.workload == "served":
        print(json.dumps(bench_served(args)))
        return
    if args.workload == "batched":
        print(json.dumps(bench_batched(args, K, max(Wm, 1))))
        return
    if args.workload in ("knife", "thrown-knives"):
        print(json.dumps(bench_knife(args, K, Wm)))
        return
    scene = bench_scenes(args, W)
    n = scene["X"].shape[0]
    torch.cuda.set_device(0)
    tuning = tuned(args, args.workload, [scene], False) if args.tune else None
    fig = bench_scene(args, args.workload, scene, K, Wm)
    if args.tune:
        tlmpm.set_tuning(None)
    extra = {}
    if args.workload == "large" and not args.no_batched:
        # the many-scene workload beside the headline: plain one scene per call
        # against one batch, the same substeps
        bk = bench_batched(args, args.batched_steps, 5, cpu=False)
        extra["batched"] = {
            "value": bk["value"], "ms_per_step": bk["ms_per_step"], "steps": bk["steps"], "warmup": bk["warmup"],
            "scenes": bk["config"]["scenes"], "particles": bk["config"]["particles"], "plain": bk["config"]["plain"],
            "batched_over_plain": bk["config"]["batched_over_plain"], "status": bk["status"],
            "contact": bk["config"]["contact"], "tuning": bk["config"]["tuning"],
            "roofline": {k: bk["roofline"][k] for k in ("kernel", "achieved", "frac", "step_alg_frac", "kernels")}}
    if args.workload == "large" and args.served_requests:
        # the first requests of the served stream (40/s, horizons U[0.5, 2] s)
        reqs = W.served(seed=args.served_seed, n_requests=args.served_requests, rate=args.rate, tick=args.tick)
        srv, st = served_run(args, reqs)
        sm = served_summary(srv, st, reqs, args.rate)
        sm["roofline"] = served_roofline(srv.kernel_time, st["throughput"])
        print(f"[bench] served sample: p50 {sm['latency_s']['p50']:.2f} s p99 {sm['latency_s']['p99']:.2f} s "
              f"throughput {sm['throughput']:.3e}", file=sys.stderr, flush=True)
        extra["served"] = sm
    if args.workload == "large" and args.others:
        # the smaller scene families of the same path, each timed inside its cut
        extra["others"] = {}
        for nm, sc, k, w in (("small", W.small(), 100, 10), ("medium", W.medium(z_start=0.034), 1000, 100),
                             ("large-4.7m", W.CONFIGS["large-4.7m"](), 100, 10)):
            f = bench_scene(args, nm, sc, k, w)
            f["roofline"] = {kk: f["roofline"][kk] for kk in ("kernel", "achieved", "frac", "step_alg_frac",
                                                                "kernels")}
            extra["others"][nm] = f
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(scene, sample=LARGE_SAMPLE if args.workload == "large" else None)
    cfg = {"workload": args.workload, "particles": n, "dt": scene["params"]["dt"],
           "material_contact": bool(scene["params"]["material_contact"]),
           "stencil": fig["stencil"], "path": "graph" if args.graphs else "plain",
           "timed_substeps": fig["timed_substeps"], "substeps_with_label_pass": fig["substeps_with_label_pass"],
           "slots": fig["slots"], "contact": fig["contact"]}
    cfg.update(extra)
    if tuning is not None:
        cfg["tuning"] = tuning
    out = {
        "metric": "particle-steps/s per GPU",
        "value": fig["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": fig["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": cfg,
        "status": fig["status"],
        "roofline": fig["roofline"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
