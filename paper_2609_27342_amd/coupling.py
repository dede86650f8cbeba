"""Two-way coupling of a free rigid knife and the TLMPM scene (Sec. III-A, III-F,
III-G): every interval, the knife's tool record (pose and twist, mass properties)
is held over `interval` substeps of tlmpm_step, whose interval-averaged wrench then
advances the knife (tlmpm_rigid_step).  The first interval starts the cut."""
import numpy as np

from . import tlmpm


class KnifeRollout:
    """scene: a tlmpm.Scene; sc: the scene dict of workloads.knife (its "knife"
    entry gives the body, the blade in body axes and the interval)."""

    def __init__(self, scene, sc):
        k = sc["knife"]
        self.scene = scene
        self.body = tlmpm.RigidBody(**k["body"])
        self.blade = dict(k["blade"])
        self.interval = int(k["interval"])
        self.dt = float(sc["params"]["dt"])
        self.gravity = np.asarray(sc["params"]["gravity"], np.float64)
        self.done = 0  # intervals so far

    def tool(self):
        return self.body.tool(dict(self.blade, new_cut=int(self.done == 0)))

    def advance(self, n_intervals=1):
        """n_intervals intervals; returns the last interval-averaged wrench."""
        w = None
        for _ in range(n_intervals):
            w = self.scene.step([self.tool()], self.interval, wrench=True)[0]
            self.body.step(w, self.gravity, self.interval * self.dt)
            self.done += 1
        return w
