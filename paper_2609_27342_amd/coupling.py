"""Two-way coupling of free rigid knives and the TLMPM scene (Sec. III-A, III-E,
III-G): every interval, each knife's tool record (pose and twist, mass properties)
is held over `interval` substeps of tlmpm_step, whose interval-averaged wrench per
tool then advances each knife (tlmpm_rigid_step).  The first interval starts the
cuts."""
import numpy as np

from . import tlmpm


class KnifeRollout:
    """scene: a tlmpm.Scene; sc: a scene dict with a "knife" entry (one knife: its
    body, blade in body axes and interval, as workloads.knife gives) or a "knives"
    entry (workloads.thrown_knives: a list of body/blade pairs and one interval)."""

    def __init__(self, scene, sc):
        if "knives" in sc:
            ks, iv = sc["knives"]["bodies"], sc["knives"]["interval"]
        else:
            ks, iv = [sc["knife"]], sc["knife"]["interval"]
        self.scene = scene
        self.bodies = [tlmpm.RigidBody(**k["body"]) for k in ks]
        self.blades = [dict(k["blade"]) for k in ks]
        self.body = self.bodies[0]
        self.interval = int(iv)
        self.dt = float(sc["params"]["dt"])
        self.gravity = np.asarray(sc["params"]["gravity"], np.float64)
        self.done = 0  # intervals so far

    def tools(self):
        return [b.tool(dict(bl, new_cut=int(self.done == 0))) for b, bl in zip(self.bodies, self.blades)]

    def tool(self):
        return self.tools()[0]

    def advance(self, n_intervals=1):
        """n_intervals intervals; returns the last interval-averaged wrench of the
        first knife (of every knife: last_wrenches)."""
        for _ in range(n_intervals):
            ws = self.scene.step(self.tools(), self.interval, wrench=True)
            for b, w in zip(self.bodies, ws):
                b.step(w, self.gravity, self.interval * self.dt)
            self.last_wrenches = ws
            self.done += 1
        return self.last_wrenches[0]
