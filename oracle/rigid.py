"""FP64 oracle of the external rigid-body solver of a free tool (two-way coupling).

Test infrastructure only.  The paper couples the TLMPM solver to an external
rigid-body system (Sec. III-A) that takes the interval-averaged wrench (Sec. III-G)
and returns the tool's next pose and twist; the tool's inverse effective mass at
a contact (Sec. III-E, Eq. 15) comes from the same body.  The integrator is semi-implicit
(symplectic) Euler of the Newton-Euler equations (reading R30):

    v      <- v + h (F / M + g)
    w_b    <- w_b + h I^-1 (tau_b - w_b x I w_b)        (body axes, I diagonal)
    x      <- x + h v
    q      <- normalise(q + h/2 (0, w) q)                 (w in world axes)

Parity unpinned against a published trajectory (the paper gives none); pinned by
closed forms and invariants in tests/test_oracle_rigid.py.
"""
import numpy as np


def qmul(a, b):
    """Hamilton product of quaternions (w, x, y, z)."""
    aw, av = a[0], np.asarray(a[1:])
    bw, bv = b[0], np.asarray(b[1:])
    return np.concatenate(([aw * bw - av @ bv], aw * bv + bw * av + np.cross(av, bv)))


def qrot(q):
    """Rotation matrix of a unit quaternion: R v = q (0, v) q*."""
    q = np.asarray(q, np.float64)
    cols = []
    for e in np.eye(3):
        qe = qmul(qmul(q, np.concatenate(([0.0], e))), q * np.array([1.0, -1.0, -1.0, -1.0]))
        cols.append(qe[1:])
    return np.array(cols).T


class Body:
    """Centre of mass x, orientation q (body -> world), velocity v, angular
    velocity w (world), mass M, principal moments I (body axes)."""

    def __init__(self, x, q, v, w, M, I):
        self.x = np.array(x, np.float64)
        self.q = np.array(q, np.float64) / np.linalg.norm(q)
        self.v = np.array(v, np.float64)
        self.w = np.array(w, np.float64)
        self.M = float(M)
        self.I = np.array(I, np.float64)

    def step(self, wrench, g, h):
        F, tau = np.asarray(wrench[:3], np.float64), np.asarray(wrench[3:], np.float64)
        R = qrot(self.q)
        self.v = self.v + h * (F / self.M + np.asarray(g, np.float64))
        wb = R.T @ self.w
        tb = R.T @ tau
        wb = wb + h * (tb - np.cross(wb, self.I * wb)) / self.I
        self.w = R @ wb
        self.x = self.x + h * self.v
        q = self.q + 0.5 * h * qmul(np.concatenate(([0.0], self.w)), self.q)
        self.q = q / np.linalg.norm(q)

    def inv_inertia_world(self):
        R = qrot(self.q)
        return R @ np.diag(1.0 / self.I) @ R.T

    def point_velocity(self, p):
        return self.v + np.cross(self.w, np.asarray(p, np.float64) - self.x)

    def inverse_effective_mass(self, p, n):
        """Normal velocity change of the body point p per unit impulse along n
        applied there: the response of a free rigid body to an impulse."""
        n = np.asarray(n, np.float64)
        r = np.asarray(p, np.float64) - self.x
        dv = n / self.M
        dw = self.inv_inertia_world() @ np.cross(r, n)
        return float((dv + np.cross(dw, r)) @ n)

    def tool(self, blade_body, labels=True, contact=True, cutting=True):
        """Tool dict of a blade fixed to the body (blade_body in body axes relative
        to the centre of mass), pose and twist of the body."""
        R = qrot(self.q)
        b = dict(blade_body)
        xe = self.x + R @ np.asarray(blade_body["x_e"], np.float64)
        for k in ("n", "e", "d"):
            b[k] = R @ np.asarray(blade_body[k], np.float64)
        b["x_e"] = xe
        b["v_e"] = self.point_velocity(xe)
        return dict(blade=b, x_B=self.x.copy(), v_B=self.v.copy(), omega_B=self.w.copy(), w_B=0.0,
                    inv_mass=1.0 / self.M, inv_inertia=self.inv_inertia_world().reshape(9),
                    labels=labels, contact=contact, cutting=cutting)
