"""Shared helpers of the tests: lockstep GPU/oracle rollouts and error metrics."""
import numpy as np


def oracle_tools(tools):
    """Tool dicts for the oracle: every tool keeps its index (history slot)."""
    return [dict(t, contact=int(bool(t.get("contact"))), cutting=int(bool(t.get("cutting")))) for t in tools]


def oracle_substep(o, tools):
    blades = [t["blade"] for t in tools if t.get("labels")]
    if blades:
        o.assign_labels(blades)
    st, w = o.step(oracle_tools(tools))
    return st, w


def field_err(a, b):
    """max_p ||a_p - b_p||_inf / max_p ||b_p||_inf (relative to the field's largest value)."""
    a = np.asarray(a, np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, np.float64).reshape(b.shape[0], -1)
    den = np.abs(b).max()
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


def _rel(a, b, scale):
    a = np.asarray(a, np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, np.float64).reshape(b.shape[0], -1)
    den = max(np.abs(b).max(), scale)
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


def u_err(state, orc, X, dt=0.0):
    """Displacement u = x - X of the GPU against x_orc - X of the oracle (an increment
    compared with an increment), relative to the largest oracle displacement, or to
    dt max|v| (what one substep adds) where that is larger."""
    return _rel(state["u"], orc["x"] - np.asarray(X, np.float64), dt * np.abs(orc["v"]).max())


def H_err(state, orc, dt=0.0, dx=1.0):
    """H = F - I of the GPU against F_orc - I, relative to the largest |F_orc - I|, or
    to dt max|v| / dx (the size of the terms v_i (x) grad N_ip dt that one substep
    sums into it) where that is larger: a uniform velocity field has zero gradient,
    and a sum that cancels to zero has no relative precision."""
    n = orc["F"].shape[0]
    I = np.eye(3).reshape(1, 9)
    # the GPU's own H (read as TLMPM_FIELD_H); F read in FP32 rounds H to multiples of 2^-24
    Hg = state["H"].reshape(n, 9).astype(np.float64) if "H" in state else \
        state["F"].reshape(n, 9).astype(np.float64) - I
    return _rel(Hg, orc["F"].reshape(n, 9) - I, dt * np.abs(orc["v"]).max() / dx)


def state_errs(state, orc, X, params=None):
    """(u, v, H) errors of one comparison; params (dt, dx) set the increment scales."""
    dt = params["dt"] if params else 0.0
    dx = params["dx"] if params else 1.0
    return u_err(state, orc, X, dt), field_err(state["v"], orc["v"]), H_err(state, orc, dt, dx)


def disp_err(x_gpu, x_orc, X):
    """max_p ||x_gpu - x_orc|| / max_p ||x_orc - X|| (displacement-relative)."""
    num = np.linalg.norm(np.asarray(x_gpu, np.float64) - x_orc, axis=1).max()
    den = np.linalg.norm(x_orc - np.asarray(X, np.float64), axis=1).max()
    return num / den


def gpu_x(state, X):
    return np.asarray(X, np.float64) + state["u"].astype(np.float64)


def band_margin(x, v, blade, dt):
    """Distance of each position x [n,3] (velocity v) to the nearest face of the
    band of Eq. 4 that decides an assignment (|s| = h, |l| = L, f = rear bound,
    f = min(b_lead, 0)) or to the side plane s = 0 (Eq. 6), in metres."""
    r = np.asarray(x, np.float64) - np.asarray(blade["x_e"])
    s = r @ np.asarray(blade["n"])
    l = r @ np.asarray(blade["e"])
    f = r @ np.asarray(blade["d"])
    uc = (np.asarray(blade["v_e"]) - np.asarray(v, np.float64)) @ np.asarray(blade["d"])
    lo = -blade["b_back"] - np.maximum(uc * dt, 0.0)
    hi = min(blade["b_lead"], 0.0)
    return np.min(np.stack([np.abs(np.abs(s) - blade["half_width"]), np.abs(np.abs(l) - blade["half_len"]),
                            np.abs(f - lo), np.abs(f - hi), np.abs(s)]), axis=0)


class LabelWatch:
    """Reading R25(b) in an independent rollout: a side digit on which the GPU and
    the oracle disagree must belong to a particle that, at the substep the two first
    disagreed, lay within the FP32-vs-FP64 state difference of a band face or of
    the side plane of that cut.  Call before() ahead of each substep (with its tools)
    and after() once it ran; `bad` lists the mismatches without that excuse."""

    def __init__(self, X, dt):
        self.X = np.asarray(X, np.float64)
        self.dt = dt
        self.prev = None
        self.bad = []
        self.checked = 0

    def before(self, g, o, tools):
        a = g.read(("u", "v"))
        b = o.get()
        self.xg = self.X + a["u"].astype(np.float64)
        self.vg = a["v"].astype(np.float64)
        self.xo, self.vo = b["x"], b["v"]
        self.blades = [t["blade"] for t in tools if t.get("labels")]

    def after(self, g, o):
        dg = g.read(("digits",))["digits"]
        do = o.get()["digits"]
        diff = dg != do
        new = diff & ~self.prev if self.prev is not None else diff
        self.prev = diff
        ps, ks = np.nonzero(new)
        if len(ps) == 0:
            return
        err = np.linalg.norm(self.xg[ps] - self.xo[ps], axis=1) + \
            np.linalg.norm(self.vg[ps] - self.vo[ps], axis=1) * self.dt
        for p, k, e in zip(ps, ks, err):
            self.checked += 1
            bl = [b for b in self.blades if b["cut_index"] == k]
            m = min(band_margin(self.xo[p:p + 1], self.vo[p:p + 1], b, self.dt)[0] for b in bl) if bl else np.inf
            if not m <= e + 1e-12:
                self.bad.append((int(p), int(k), float(m), float(e)))

    def mismatched(self):
        return 0 if self.prev is None else int(self.prev.any(axis=1).sum())
