"""Continuous batching of cutting rollouts on one GPU.

Requests (a scene and its tool schedule over a horizon of substeps) arrive over
time.  A request is admitted (first in, first out) when its device bytes fit the
HBM budget beside those of the running rollouts: its scene workspace
(tlmpm_scene_footprint) plus a bound on its share of the batch workspace
(tlmpm_batch_scene_bytes), so the scene workspaces and the batch workspace together
never exceed the budget.  A request that alone exceeds the budget is refused
(status TLMPM_E_NOMEM) instead of admitted.  Every admitted request advances by one
tick of substeps per iteration through one batched step (tlmpm_batch_step), so
each kernel launch covers all running rollouts.  The batch is rebuilt whenever a
rollout finishes or starts.  New scenes are built on a second stream while the
current tick runs.

The tool schedule of a request is constant over each tick: its tools at the
first substep of the tick, moved by TLMPM_TOOL_ADVANCE within the tick.
"""
import time

import numpy as np

from . import tlmpm


class Admission:
    """Device-byte accounting of the running rollouts against a budget."""

    def __init__(self, budget_bytes):
        self.budget = int(budget_bytes)
        self.used = 0

    def refuses(self, nbytes):
        """A request of nbytes can never run (more than the whole budget)."""
        return nbytes > self.budget

    def fits(self, nbytes):
        return self.used + nbytes <= self.budget

    def take(self, nbytes):
        if not self.fits(nbytes):
            raise ValueError("admission beyond the device budget")
        self.used += nbytes

    def release(self, nbytes):
        self.used -= nbytes
        assert self.used >= 0


def request_bytes(scene_dict):
    """Device bytes a request holds while it runs: its scene workspace plus its
    bound on the batch workspace."""
    return tlmpm.footprint(scene_dict) + tlmpm.batch_scene_bytes(scene_dict)


class Rollout:
    def __init__(self, req, scene_dict, scene, arrival, admitted, nbytes):
        self.req = req
        self.nbytes = nbytes
        self.sd = scene_dict
        self.scene = scene
        self.arrival = arrival
        self.admitted = admitted
        self.done_steps = 0
        self.horizon = int(scene_dict["steps"])
        self.n = int(scene_dict["X"].shape[0])

    def tools(self, tick):
        return [dict(t, advance=True) for t in self.sd["tools_at"](self.done_steps)]


class Server:
    """budget_bytes: device bytes that running rollouts may hold; tick: substeps
    per iteration; build(req) -> scene dict of a request."""

    def __init__(self, build, budget_bytes, tick=100, max_batch=256, read_fields=("u", "D", "digits"),
                 profile=False):
        """profile: time the P2G and G2P launches of every batch with HIP events
        (tlmpm_profile_enable mode 2, the launch arrangement unchanged); the sums are
        in self.kernel_time {class: [ms, launches, particles x launches]}."""
        import torch
        self.torch = torch
        self.build = build
        self.budget = int(budget_bytes)
        self.tick = int(tick)
        self.max_batch = int(max_batch)
        self.read_fields = tuple(read_fields)
        self.stream = torch.cuda.current_stream()
        self.create_stream = torch.cuda.Stream()
        self.results = {}
        self.profile = bool(profile)
        self.kernel_time = {}

    def _close_batch(self, batch, n_particles):
        if self.profile:
            for k, (ms, cnt) in batch.profile_read().items():
                acc = self.kernel_time.setdefault(k, [0.0, 0, 0])
                acc[0] += ms
                acc[1] += cnt
                acc[2] += cnt * n_particles
        batch.close()

    def _admit(self, queue, active, adm, now_fn):
        """Builds scenes for queued requests (FIFO) while they fit; refuses those
        that exceed the whole budget."""
        admitted = []
        while queue and len(active) + len(admitted) < self.max_batch:
            req, sd, nbytes = queue[0]
            if sd is None:
                sd = self.build(req)
                nbytes = request_bytes(sd)
                queue[0] = (req, sd, nbytes)
            if adm.refuses(nbytes):
                queue.pop(0)
                t = now_fn()
                self.results[req["index"]] = dict(fields=None, status=tlmpm.E_NOMEM, n=int(sd["X"].shape[0]),
                                                  steps=int(sd["steps"]), arrival=req["_arrival_wall"], admitted=None,
                                                  done=t, bytes=nbytes)
                continue
            if not adm.fits(nbytes):
                break
            queue.pop(0)
            adm.take(nbytes)
            with self.torch.cuda.stream(self.create_stream):
                ws = self.torch.empty(tlmpm.footprint(sd), dtype=self.torch.uint8, device="cuda")
                g = tlmpm.Scene(sd, stream=self.create_stream, workspace=ws)
            admitted.append(Rollout(req, sd, g, req["_arrival_wall"], now_fn(), nbytes))
        return admitted

    def run(self, requests, realtime=True, log=None):
        """Serves `requests` (dicts with 'arrival' seconds and whatever build()
        needs).  realtime=False admits every request at time zero.  Returns stats
        (latency percentiles from arrival to result, throughput) and fills
        self.results[index] with the final fields and timestamps."""
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        pending = sorted(requests, key=lambda r: r["arrival"])
        queue = []  # (req, scene dict or None, bytes)
        active = []
        adm = Admission(self.budget)
        self.peak_bytes = 0
        batch = None
        batch_n = 0
        lat = {}
        work = 0
        iters = 0
        sizes = []
        last_log = 0.0
        while pending or queue or active:
            tnow = now()
            while pending and (not realtime or pending[0]["arrival"] <= tnow):
                r = dict(pending.pop(0))
                r["_arrival_wall"] = r["arrival"] if realtime else 0.0
                queue.append((r, None, 0))
            if not active and not queue:
                time.sleep(max(0.0, min(0.05, pending[0]["arrival"] - tnow)))
                continue
            # one tick of every running rollout (asynchronous)
            if active:
                tools = [ro.tools(self.tick) for ro in active]
                batch.step(tools, self.tick)
            # build newly admissible scenes while the tick runs
            new = self._admit(queue, active, adm, now)
            self.peak_bytes = max(self.peak_bytes, adm.used)
            if active:
                batch.sync()
                iters += 1
                sizes.append(len(active))
                for ro in active:
                    ro.done_steps += self.tick
                    work += ro.n * self.tick
                if log and now() - last_log > 15.0:
                    last_log = now()
                    log(f"[serve] t={last_log:.1f}s iteration {iters} running={len(active)} "
                        f"particles={sum(ro.n for ro in active)} queued={len(queue)} done={len(lat)} "
                        f"bytes={adm.used}")
            finished = [ro for ro in active if ro.done_steps >= ro.horizon]
            if finished or new:
                if batch is not None:
                    self._close_batch(batch, batch_n)
                    batch = None
                for ro in finished:
                    out = ro.scene.read(self.read_fields)
                    st, detail = ro.scene.status_detail()
                    if st:
                        detail += f"; largest slot count {ro.scene.slot_stats()[1]}"
                    ro.scene.close()
                    adm.release(ro.nbytes)
                    done = now()
                    lat[ro.req["index"]] = done - ro.arrival
                    self.results[ro.req["index"]] = dict(fields=out, status=st, detail=detail, n=ro.n,
                                                         steps=ro.horizon, arrival=ro.arrival, admitted=ro.admitted,
                                                         done=done)
                    if log:
                        log(f"[serve] t={done:.2f}s done request {ro.req['index']} n={ro.n} "
                            f"steps={ro.horizon} latency={done - ro.arrival:.2f}s running={len(active) - 1}")
                active = [ro for ro in active if ro.done_steps < ro.horizon] + new
                if active:
                    self.create_stream.synchronize()
                    batch = tlmpm.Batch([ro.scene for ro in active], stream=self.stream)
                    batch_n = sum(ro.n for ro in active)
                    if self.profile:
                        batch.profile("transfers")
                    # the batch workspace is within the bytes reserved at admission
                    assert adm.used >= sum(ro.scene.bytes for ro in active) + batch.bytes
        wall = now()
        L = np.array([lat[k] for k in sorted(lat)])
        refused = sum(1 for r in self.results.values() if r["status"] == tlmpm.E_NOMEM)
        return dict(requests=len(L), refused=refused, peak_bytes=self.peak_bytes, wall_s=wall, particle_steps=work, throughput=work / wall if wall > 0 else 0.0,
                    p50_s=float(np.percentile(L, 50)) if len(L) else None,
                    p99_s=float(np.percentile(L, 99)) if len(L) else None,
                    mean_batch=float(np.mean(sizes)) if sizes else 0.0, iterations=iters)
