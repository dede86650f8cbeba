"""Seeded synthetic scenes and tool schedules.

Input generation only: particle sampling, material parameters and blade/tool
poses per step.  Nothing here evaluates the method; the same scenes feed the GPU
library, the CPU oracle and the benchmark.

A scene is a dict:
  name, params (dict of scalars), X [n,3] float32, v0 [n,3] float32 or None,
  vol0, mass, E: float32 arrays [n], steps (int), tools_at(j) -> list of tool dicts.

A tool dict: {"blade": blade dict, "x_B", "v_B", "omega_B": 3-vectors, "w_B": float,
"labels": bool (assign side digits from its band), "contact": bool, "cutting": bool}.
A blade dict: cut_index, new_cut, x_e, n, e, d, v_e (float64 3-vectors), half_len,
half_width, b_back, b_lead.  Blade poses are computed in float64 so every consumer
sees bit-identical values.

Particle sampling (jittered lattice): every reference cell is split into 2x2x2
sub-cells; a sub-cell centre that lies inside the body yields one particle, moved by
an independent uniform jitter in [-0.125, 0.125] dx per axis.  V0 = dx^3/8 and
m = rho V0.  Particles are returned in a seeded random order.
"""
import math

import numpy as np

# Default contact and cutting constants (the paper names them without values,
# except G_c, zeta and mu, which are taken from its banana experiment).
CONTACT_DEFAULTS = dict(s_R=1.0, s_n=0.5, gamma_k=0.25, gamma_c=0.5, mu_s=0.2, mu_d=0.2,
                        G_c=700.0, zeta=0.9, u_min=1e-3)


def jittered_lattice(lo, hi, dx, origin, inside, rng, jitter=0.25):
    """Sample the body {inside(P) == True} inside the box [lo, hi] (world units)."""
    origin = np.asarray(origin, np.float64)
    c0 = np.floor((np.asarray(lo) - origin) / dx).astype(np.int64)
    c1 = np.ceil((np.asarray(hi) - origin) / dx).astype(np.int64)
    ii = [np.arange(c0[a], c1[a]) for a in range(3)]
    sub = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)], np.float64)
    out = []
    # iterate over z slabs to bound memory
    for kz in ii[2]:
        gx, gy = np.meshgrid(ii[0], ii[1], indexing="ij")
        cells = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, kz)], axis=1).astype(np.float64)
        centres = (cells[:, None, :] + (sub[None, :, :] + 0.5) * 0.5) * dx + origin
        centres = centres.reshape(-1, 3)
        keep = inside(centres)
        if np.any(keep):
            out.append(centres[keep])
    if not out:
        return np.zeros((0, 3), np.float32)
    P = np.concatenate(out, axis=0)
    P += rng.uniform(-jitter, jitter, size=P.shape) * (0.5 * dx)
    return P.astype(np.float32)


def _finish(name, params, X, rho, E, rng, steps, tools_at, v0=None):
    n = X.shape[0]
    perm = rng.permutation(n)
    X = np.ascontiguousarray(X[perm])
    dx = params["dx"]
    V0 = np.float32(dx ** 3 / 8.0)
    vol0 = np.full(n, V0, np.float32)
    mass = (np.float32(rho) * vol0).astype(np.float32)
    if np.isscalar(E):
        Ea = np.full(n, E, np.float32)
    else:
        Ea = np.ascontiguousarray(np.asarray(E, np.float32)[perm])
    if v0 is not None:
        v0 = np.ascontiguousarray(np.asarray(v0, np.float32)[perm])
    return dict(name=name, params=params, X=X, v0=v0, vol0=vol0, mass=mass, E=Ea, steps=steps,
                tools_at=tools_at, rho=rho)


def _grid(lo, hi, dx, pad=1):
    """Reference grid covering [lo, hi] with `pad` empty cells on every side."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    origin = lo - pad * dx
    cells = [int(math.ceil((hi[a] - lo[a]) / dx - 1e-9)) + 2 * pad for a in range(3)]
    return origin.tolist(), cells


def base_params(dx, origin, cells, dt, nu, **kw):
    """Scene parameters.  A body "on the floor" has its lowest sub-cell centres at
    z = dx/4; with the jitter of +-dx/8 and contact radius dx/4 its lowest spheres
    just touch a floor at z = -dx/8, so the scene starts without penetration."""
    p = dict(dx=float(dx), origin=[float(o) for o in origin], cells=[int(c) for c in cells],
             dt=float(dt), nu=float(nu), gravity=[0.0, 0.0, -9.81], flip_beta=0.95,
             max_cuts=4, material_contact=0, floor_on=1, floor_z=-float(dx) / 8.0, single_field=0)
    p.update(CONTACT_DEFAULTS)
    p.update(kw)
    return p


def blade(cut_index, x_e, n, d, v_e, half_len, half_width, b_back, b_lead, new_cut=False):
    n = np.asarray(n, np.float64)
    d = np.asarray(d, np.float64)
    e = np.cross(n, d)  # (n, e, d) right-handed with e = n x d
    return dict(cut_index=int(cut_index), new_cut=int(bool(new_cut)),
                x_e=np.asarray(x_e, np.float64), n=n, e=e, d=d,
                v_e=np.asarray(v_e, np.float64), half_len=float(half_len),
                half_width=float(half_width), b_back=float(b_back), b_lead=float(b_lead))


def tool(bl, labels=True, contact=True, cutting=True, x_B=None, v_B=None):
    return dict(blade=bl, x_B=np.asarray(bl["x_e"] if x_B is None else x_B, np.float64),
                v_B=np.asarray(bl["v_e"] if v_B is None else v_B, np.float64),
                omega_B=np.zeros(3), w_B=0.0, labels=bool(labels), contact=bool(contact),
                cutting=bool(cutting))


# --------------------------------------------------------------------------- small
def small(seed=1, deep=False, steps=100):
    """Neo-Hookean cube [0, 0.1]^3 on a floor, dx = 5 mm, 8 ppc (64,000 particles),
    E = 1e5, nu = 0.3, rho = 1000, dt = 1e-4.  A planar blade (0.15 x 0.05 m, plane
    x = 0.05) descends at 0.2 m/s; it assigns side labels only (no tool contact).
    deep=True starts the edge at z = 0.06 so the first label pass already cuts."""
    dx = 0.005
    origin, cells = _grid((0, 0, 0), (0.1, 0.1, 0.1), dx, pad=1)
    rng = np.random.default_rng(seed)

    def inside(P):
        return np.all((P >= 0.0) & (P <= 0.1), axis=1)

    X = jittered_lattice((0, 0, 0), (0.1, 0.1, 0.1), dx, origin, inside, rng)
    params = base_params(dx, origin, cells, 1e-4, 0.3, material_contact=0, floor_on=1)
    z0 = 0.06 if deep else 0.10
    dt = params["dt"]

    def tools_at(j):
        z = z0 - 0.2 * (j * dt)
        bl = blade(0, (0.05, 0.05, z), (1, 0, 0), (0, 0, -1), (0, 0, -0.2), 0.075, 6 * dx, 0.05, dx,
                   new_cut=(j == 0))
        return [tool(bl, labels=True, contact=False, cutting=False)]

    return _finish("small-deep" if deep else "small", params, X, 1000.0, 1e5, rng, steps, tools_at)


# -------------------------------------------------------------------------- medium
def medium(seed=2, steps=8000, dx=0.002, z_start=0.038):
    """Curved cylinder: radius 0.018 m around a horizontal centreline arc of radius
    0.3 m and length 0.18 m (0.6 rad), resting on the floor; dx = 2 mm, 8 ppc,
    E = 5e4, nu = 0.3, rho = 1000, dt = 1e-4, material contact on.  Two vertical cuts
    normal to the centreline at +-3 cm of arc from the middle descend at 0.1 m/s from
    z = 0.038 to 0; after each cut the blade pushes along its normal (+n, then -n) at
    0.1 m/s for 0.3 s and is removed.  z_start < 0.036 starts the first cut with
    the edge already inside the tube (labels and blade contact from step 0)."""
    Rc, rt, half_ang = 0.3, 0.018, 0.3
    cy = -Rc  # centre of curvature at (0, cy); the arc passes through (0, 0)
    rng = np.random.default_rng(seed)
    lo = np.array([-Rc * math.sin(half_ang) - rt, -Rc * (1 - math.cos(half_ang)) - rt, 0.0])
    hi = np.array([Rc * math.sin(half_ang) + rt, rt, 2 * rt])
    origin, cells = _grid(lo, hi, dx, pad=1)

    def inside(P):
        qx, qy = P[:, 0], P[:, 1] - cy
        ang = np.arctan2(qx, qy)
        rho = np.hypot(qx, qy)
        return (np.abs(ang) <= half_ang) & ((rho - Rc) ** 2 + (P[:, 2] - rt) ** 2 <= rt * rt)

    X = jittered_lattice(lo, hi, dx, origin, inside, rng)
    params = base_params(dx, origin, cells, 1e-4, 0.3, material_contact=1, floor_on=1)
    dt = params["dt"]
    t_cut = int(round(z_start / 0.1 / dt))  # 3800 steps from z = 0.038
    t_push = int(round(0.3 / dt))          # 3000 steps
    thetas = (-0.1, 0.1)
    pushes = (1.0, -1.0)

    def frame(th):
        cpt = np.array([Rc * math.sin(th), cy + Rc * math.cos(th), 0.0])
        tang = np.array([math.cos(th), -math.sin(th), 0.0])
        return cpt, tang

    def tools_at(j):
        k, r = divmod(j, t_cut + t_push)
        if k >= 2:
            return []
        cpt, nrm = frame(thetas[k])
        if r < t_cut:
            z = z_start - 0.1 * (r * dt)
            bl = blade(k, (cpt[0], cpt[1], z), nrm, (0, 0, -1), (0, 0, -0.1), 0.075, 6 * dx, 0.05, dx,
                       new_cut=(r == 0))
            return [tool(bl, labels=True, contact=True, cutting=True)]
        s = pushes[k] * 0.1 * ((r - t_cut) * dt)
        ve = pushes[k] * 0.1 * nrm
        pos = np.array([cpt[0], cpt[1], 0.0]) + s * nrm
        bl = blade(k, pos, nrm, (0, 0, -1), ve, 0.075, 6 * dx, 0.05, dx)
        return [tool(bl, labels=False, contact=True, cutting=False)]

    return _finish("medium", params, X, 1000.0, 5e4, rng, steps, tools_at)


# --------------------------------------------------------------------------- large
def large(seed=3, steps=2000, dx=0.0015, box=(0.3, 0.2, 0.1)):
    """Box 0.3 x 0.2 x 0.1 m on the floor, 8 ppc, per-particle E log-uniform in
    [2e4, 2e5], nu = 0.3, rho = 1000, dt = 3e-5, contact on.  Blades at 0.2 m/s, edges
    pre-inserted at z = 0.06: k0 plane x = 0.10, k1 plane x = 0.20, k2 vertical and
    rotated 60 degrees from k0, crossing it at (0.10, 0.10); they descend for steps
    0-999 and are withdrawn; k3 (plane y = 0.10, crossing k0 and k2) descends for
    steps 1000-1999.  dx = 1.5 mm gives 14.2M particles; dx and box scale it."""
    bx, by, bz = box
    rng = np.random.default_rng(seed)
    origin, cells = _grid((0, 0, 0), box, dx, pad=1)

    def inside(P):
        return (P[:, 0] >= 0) & (P[:, 0] <= bx) & (P[:, 1] >= 0) & (P[:, 1] <= by) & (P[:, 2] >= 0) & (P[:, 2] <= bz)

    X = jittered_lattice((0, 0, 0), box, dx, origin, inside, rng)
    E = np.exp(rng.uniform(math.log(2e4), math.log(2e5), size=X.shape[0])).astype(np.float32)
    # three cuts cross along the line x = y = 0.10 from step 1000 on: nodes there hold
    # up to 3 x 2 x 2 side codes (a digit 0, 1 or 2 of the newest cut), beyond 8 slots
    params = base_params(dx, origin, cells, 3e-5, 0.3, material_contact=1, floor_on=1, slot_capacity=16)
    dt = params["dt"]
    s = bx / 0.3  # keep the blade layout proportional when the box is scaled
    c60 = (math.cos(math.radians(60)), math.sin(math.radians(60)), 0.0)
    specs = [  # cut index, edge centre (x, y), normal, half length, active steps
        (0, (0.10 * s, by / 2), (1, 0, 0), 0.6 * by, (0, 1000)),
        (1, (0.20 * s, by / 2), (1, 0, 0), 0.6 * by, (0, 1000)),
        (2, (0.10 * s, 0.10 * by / 0.2), c60, 0.6 * by, (0, 1000)),
        (3, (bx / 2, 0.10 * by / 0.2), (0, 1, 0), 0.55 * bx, (1000, 2000)),
    ]

    def tools_at(j):
        out = []
        for k, (cx, cy_), nrm, L, (a, b) in specs:
            if not (a <= j < b):
                continue
            z = 0.06 * bz / 0.1 - 0.2 * ((j - a) * dt)
            bl = blade(k, (cx, cy_, z), nrm, (0, 0, -1), (0, 0, -0.2), L, 6 * dx, 0.05, dx, new_cut=(j == a))
            out.append(tool(bl, labels=True, contact=True, cutting=True))
        return out

    return _finish("large", params, X, 1000.0, E, rng, steps, tools_at)


# ------------------------------------------------------------------------- batched
def _random_dir_down(rng):
    """Unit vector, uniform on the sphere restricted to d_z <= -0.5."""
    while True:
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        if d[2] <= -0.5:
            return d


def _exit_distance(p, w, lo, hi):
    """Distance from p (inside the box [lo, hi]) along the unit vector w to the box
    boundary."""
    t = np.inf
    for a in range(3):
        if w[a] > 1e-12:
            t = min(t, (hi[a] - p[a]) / w[a])
        elif w[a] < -1e-12:
            t = min(t, (lo[a] - p[a]) / w[a])
    return float(t)


def _random_body(rng, n_target, dx):
    """A box (aspect ratios U[0.5, 2]) or a horizontal cylinder (length / diameter
    U[1, 4]), p = 1/2, with about n_target particles at 8 per cell, resting on the
    floor.  Returns (shape, extent, inside)."""
    V = n_target * dx ** 3 / 8.0
    if rng.uniform() < 0.5:
        r1, r2 = rng.uniform(0.5, 2.0, size=2)
        c = (V / (r1 * r2)) ** (1.0 / 3.0)
        ext = np.array([r1 * c, r2 * c, c])

        def inside(P):
            return np.all((P >= 0.0) & (P <= ext), axis=1)
        return "box", ext, inside
    q = rng.uniform(1.0, 4.0)
    r = (V / (2.0 * math.pi * q)) ** (1.0 / 3.0)
    ext = np.array([2.0 * r * q, 2.0 * r, 2.0 * r])

    def inside(P):
        return (P[:, 0] >= 0.0) & (P[:, 0] <= ext[0]) & ((P[:, 1] - r) ** 2 + (P[:, 2] - r) ** 2 <= r * r)
    return "cylinder", ext, inside


def _random_blade(rng, ext):
    """Descent direction d uniform with d_z <= -0.5, normal n uniform with n.d = 0,
    speed U[0.05, 0.3] m/s, edge start on the body's bounding box on the ray from an
    aim point (the centre moved by up to +-25 % of the extent per axis) back along
    -d.  Returns (start, n, d, speed)."""
    d = _random_dir_down(rng)
    a = rng.normal(size=3)
    n = a - np.dot(a, d) * d
    n /= np.linalg.norm(n)
    speed = rng.uniform(0.05, 0.3)
    aim = 0.5 * ext + rng.uniform(-0.25, 0.25, size=3) * ext
    start = aim - d * _exit_distance(aim, -d, np.zeros(3), ext)
    return start, n, d, speed


def _random_scene(rng, n_target, dx, dt):
    shape, ext, inside = _random_body(rng, n_target, dx)
    lo = np.zeros(3)
    origin, cells = _grid(lo, ext, dx, pad=1)
    X = jittered_lattice(lo, ext, dx, origin, inside, rng)
    E = float(np.exp(rng.uniform(math.log(2e4), math.log(1e5))))
    # up to three crossing cuts (many-scene workload) or four slices in a small
    # body: room for 16 logical grids per node
    params = base_params(dx, origin, cells, dt, 0.3, material_contact=1, floor_on=1, slot_capacity=16)
    return shape, ext, X, E, params


def _blade_tool(k, spec, j, j0, diag, dx, dt):
    start, n, d, speed = spec
    ve = speed * d
    bl = blade(k, start + ve * ((j - j0) * dt), n, d, ve, diag, 6 * dx, diag, dx, new_cut=(j == j0))
    return tool(bl, labels=True, contact=True, cutting=True)


def batch_scene(seed, index, n_target, dx=0.0025, steps=1000, dt=1e-4):
    """One scene of the many-scene workload: a random box or cylinder
    (_random_body) with about n_target particles; E log-uniform in [2e4, 1e5],
    nu = 0.3, rho = 1000, floor and material contact on; one to three simultaneous
    blades (_random_blade), each its own cut, half length = body diagonal.  All
    randomness comes from (seed, index), so a scene is the same alone or in any
    batch."""
    rng = np.random.default_rng([seed, index])
    shape, ext, X, E, params = _random_scene(rng, n_target, dx, dt)
    diag = float(np.linalg.norm(ext))
    specs = [_random_blade(rng, ext) for _ in range(int(rng.integers(1, 4)))]

    def tools_at(j):
        return [_blade_tool(k, sp, j, 0, diag, dx, dt) for k, sp in enumerate(specs)]

    sc = _finish(f"batch-{index}-{shape}", params, X, 1000.0, E, rng, steps, tools_at)
    sc["shape"] = shape
    return sc


def _slicing_blades(rng, ext, n_cuts, dx):
    """Sequential slicing (the paper's scenes with successive cuts): one knife
    orientation per request (d and n drawn as in _random_blade), cut k in the plane
    of normal n through the body's centre moved by o_k along n, o_k at the k-th of
    n_cuts interior points dividing [-r, r] into equal parts (r = half the smallest
    extent, so that the plane's point on the centre line lies in the body), each
    jittered by up to +-20 % of a part; the cuts proceed from one side; each has its
    own speed U[0.05, 0.3] m/s and starts where its line through that point along -d
    leaves the bounding box.  Slices are at least 4 dx thick before the jitter: a
    body too small for n_cuts such slices gets fewer cuts (at least one), since
    thinner slices put every particle in the label bands of several cuts at once.  Returns [(start, n, d, speed)] in
    cut order."""
    d = _random_dir_down(rng)
    a = rng.normal(size=3)
    n = a - np.dot(a, d) * d
    n /= np.linalg.norm(n)
    r = 0.5 * float(np.min(ext))
    n_cuts = max(1, min(n_cuts, int(2.0 * r / (4.0 * dx)) - 1))
    part = 2.0 * r / (n_cuts + 1)
    centre = 0.5 * np.asarray(ext, np.float64)
    out = []
    for k in range(n_cuts):
        o = -r + (k + 1) * part + rng.uniform(-0.2, 0.2) * part
        aim = centre + o * n
        start = aim - d * _exit_distance(aim, -d, np.zeros(3), ext)
        out.append((start, n.copy(), d.copy(), rng.uniform(0.05, 0.3)))
    return out


def served_request(seed, index, n_target, horizon_steps, tick, dx=0.0025, dt=1e-4):
    """One request of the served workload: body and material as batch_scene, cut by
    sequential slicing (_slicing_blades): one to four parallel cuts made one after
    another, each in its own window of the horizon (windows are whole ticks; a
    blade is withdrawn when its window ends)."""
    rng = np.random.default_rng([seed, index])
    shape, ext, X, E, params = _random_scene(rng, n_target, dx, dt)
    diag = float(np.linalg.norm(ext))
    specs = _slicing_blades(rng, ext, int(rng.integers(1, 5)), dx)
    n_cuts = len(specs)
    n_ticks = max(1, horizon_steps // tick)
    bounds = [tick * ((n_ticks * k) // n_cuts) for k in range(n_cuts + 1)]

    def tools_at(j):
        for k in range(n_cuts):
            if bounds[k] <= j < bounds[k + 1]:
                return [_blade_tool(k, specs[k], j, bounds[k], diag, dx, dt)]
        return []

    sc = _finish(f"request-{index}-{shape}", params, X, 1000.0, E, rng, tick * n_ticks, tools_at)
    sc["shape"] = shape
    return sc


def crop(scene, xr, yr):
    """The particles of `scene` with x in xr and y in yr, as a scene of their own
    (same grid, parameters and tools)."""
    X = scene["X"]
    keep = (X[:, 0] >= xr[0]) & (X[:, 0] <= xr[1]) & (X[:, 1] >= yr[0]) & (X[:, 1] <= yr[1])
    out = dict(scene, X=np.ascontiguousarray(X[keep]), vol0=scene["vol0"][keep], mass=scene["mass"][keep],
               E=scene["E"][keep], name=scene["name"] + "-sample")
    if scene.get("v0") is not None:
        out["v0"] = scene["v0"][keep]
    return out


def served(seed=5, n_requests=500, rate=40.0, n_range=(10000, 1000000), horizon_s=(0.5, 2.0), tick=100,
           dt=1e-4):
    """Arrivals of the served workload: Poisson at `rate` per second; per request a
    log-uniform particle count in n_range and a horizon U[horizon_s] seconds
    (rounded to whole ticks of `tick` substeps).  Returns a list of dicts
    (index, arrival time, n_target, horizon steps); served_request() builds the
    scene when the request is admitted."""
    rng = np.random.default_rng([seed, 1 << 21])
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        n = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        h = max(tick, int(round(rng.uniform(*horizon_s) / dt / tick)) * tick)
        out.append(dict(index=i, arrival=t, n_target=n, horizon=h, seed=seed, tick=tick))
    return out


def batch_sizes(seed=4, n_scenes=256, median=40000, sigma=0.7, lo=5000, hi=200000):
    """Target particle counts: LogNormal(ln median, sigma) truncated to [lo, hi] by
    resampling."""
    rng = np.random.default_rng([seed, 1 << 20])
    out = []
    while len(out) < n_scenes:
        v = float(np.exp(rng.normal(math.log(median), sigma)))
        if lo <= v <= hi:
            out.append(int(round(v)))
    return out


def batched(seed=4, n_scenes=256, steps=1000, median=40000, lo=5000, hi=200000):
    """The many-scene workload: n_scenes independent batch_scene()s (about 12.5M
    particles in total at the defaults)."""
    sizes = batch_sizes(seed, n_scenes, median, lo=lo, hi=hi)
    return dict(name="batched", scenes=[batch_scene(seed, i, n, steps=steps) for i, n in enumerate(sizes)],
                steps=steps)


# ------------------------------------------------------------------- generic pieces
def box_scene(n_cells=(6, 5, 4), dx=0.01, seed=0, E=1e4, nu=0.3, rho=1000.0, dt=1e-4, v0=None,
              jitter=0.25, **kw):
    """A small box of n_cells reference cells starting at the origin, for unit tests."""
    rng = np.random.default_rng(seed)
    hi = np.array(n_cells, np.float64) * dx
    origin, cells = _grid((0, 0, 0), hi, dx, pad=1)

    def inside(P):
        return np.all((P >= 0) & (P <= hi), axis=1)

    X = jittered_lattice((0, 0, 0), hi, dx, origin, inside, rng, jitter=jitter)
    params = base_params(dx, origin, cells, dt, nu, **kw)
    v = None
    if v0 is not None:
        v = np.broadcast_to(np.asarray(v0, np.float32), X.shape).copy()
    return _finish("box", params, X, rho, E, rng, 1, lambda j: [], v0=v)


def segments(scene, j0, j1):
    """Split steps [j0, j1) into runs over which every tool moves at constant
    velocity (the set of tools and their flags unchanged).  Yields (j, count,
    tools at step j); a run starts a new cut only at its first step."""
    def sig(tools):
        return tuple((t["blade"]["cut_index"], t["labels"], t["contact"], t["cutting"],
                      tuple(np.round(t["blade"]["v_e"], 12)), tuple(np.round(t["blade"]["n"], 12)))
                     for t in tools)
    j = j0
    while j < j1:
        tools = scene["tools_at"](j)
        k = j + 1
        while k < j1:
            nxt = scene["tools_at"](k)
            if sig(nxt) != sig(tools) or any(t["blade"]["new_cut"] for t in nxt):
                break
            k += 1
        yield j, k - j, tools
        j = k


def knife_blade_body(half_len, height, dx=0.002, new_cut=True):
    """Blade of a knife plate in the plate's body frame (centre of mass at the
    origin): edge along x at the bottom (z = -height / 2), front direction -z, plane
    normal +y; band half width 6 dx, rear extent the plate height, lead dx."""
    return blade(0, (0.0, 0.0, -0.5 * height), (0, 1, 0), (0, 0, -1), (0, 0, 0), half_len, 6 * dx, height, dx,
                 new_cut=new_cut)


def knife(dx=0.002, block=(0.08, 0.04, 0.04), seed=9, dt=1e-4, interval=10, steps=2000, tilt_deg=25.0,
          drop=0.001, v_drop=0.3, mass=0.1, plate=(0.1, 0.03, 0.001)):
    """Two-way coupled cutting (the paper's gravity-driven knife): a soft block
    (E = 6 kPa, nu = 0.4, rho = 1100 kg/m^3, dx = 2 mm, 8 ppc: 102,400 particles for
    the default 8 x 4 x 4 cm) on the floor, material contact on; a free 0.1 kg knife,
    a plate of `plate` (length along the edge, height, thickness), tilted by
    tilt_deg about its plane normal, its lowest edge point `drop` above the block and
    moving down at v_drop, then moved by gravity and the material's reaction only.
    The knife is updated every `interval` substeps from the interval-averaged wrench
    (tlmpm_rigid_step); its tool record (tlmpm_rigid_tool) is held over the interval."""
    rng = np.random.default_rng(seed)
    hi = tuple(float(b) for b in block)
    origin, cells = _grid((0, 0, 0), hi, dx, pad=1)

    def inside(P):
        return np.all((P >= 0.0) & (P <= np.asarray(hi)), axis=1)

    X = jittered_lattice((0, 0, 0), hi, dx, origin, inside, rng)
    params = base_params(dx, origin, cells, dt, 0.4, material_contact=1)
    L, H, T = (float(a) for a in plate)
    th = math.radians(tilt_deg)
    # rotation about +y by th maps the +x end of the edge downwards
    q = [math.cos(th / 2), 0.0, math.sin(th / 2), 0.0]
    low = 0.5 * L * math.sin(th) + 0.5 * H * math.cos(th)  # centre of mass above the lowest edge point
    x = [0.5 * hi[0], 0.5 * hi[1], hi[2] + drop + low]
    inertia = [mass * (H * H + T * T) / 12.0, mass * (L * L + H * H) / 12.0, mass * (L * L + T * T) / 12.0]
    body = dict(x=x, q=q, v=[0.0, 0.0, -float(v_drop)], omega=[0.0, 0.0, 0.0], mass=float(mass), inertia=inertia)
    sc = _finish("knife", params, X, 1100.0, 6.0e3, rng, steps, None)
    sc["knife"] = dict(body=body, blade=knife_blade_body(0.5 * L, H, dx), interval=int(interval))
    return sc


def _qmul(a, b):
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return [aw * bw - ax * bx - ay * by - az * bz, aw * bx + ax * bw + ay * bz - az * by,
            aw * by - ax * bz + ay * bw + az * bx, aw * bz + ax * by - ay * bx + az * bw]


def thrown_knives(dx=0.002, block=(0.12, 0.04, 0.04), seed=11, dt=1e-4, interval=10, steps=2000,
                  speeds=(0.5, 0.8, 1.1), tilt_deg=10.0, drop=0.001, mass=0.1, plate=(0.06, 0.03, 0.001)):
    """Several free knives launched at the same block (the paper's thrown-knife
    scene, Sec. IV): the block is fixed-corotated with von Mises plasticity (E =
    20 kPa, nu = 0.4, rho = 1200 kg/m^3, yield stress 2 kPa), dx = 2 mm, 8 ppc
    (192,000 particles for the default 12 x 4 x 4 cm), on the floor, material contact
    on. Knife k (mass `mass`, plate `plate`: edge length, height, thickness) has its
    edge across the block (along y) at x = (k + 1/2) / len(speeds) of the block
    length, tilted by tilt_deg about its plane normal, its lowest edge point `drop`
    above the block, and moves edge first (down) at speeds[k]; each has its own cut
    digit and is moved only by gravity and the material's reaction, updated every
    `interval` substeps from its interval-averaged wrench."""
    rng = np.random.default_rng(seed)
    hi = tuple(float(b) for b in block)
    origin, cells = _grid((0, 0, 0), hi, dx, pad=1)

    def inside(P):
        return np.all((P >= 0.0) & (P <= np.asarray(hi)), axis=1)

    X = jittered_lattice((0, 0, 0), hi, dx, origin, inside, rng)
    params = base_params(dx, origin, cells, dt, 0.4, material_contact=1, material=1, yield_stress=2.0e3)
    L, H, T = (float(a) for a in plate)
    th = math.radians(tilt_deg)
    # body x (the edge) -> world y, body y (plate normal) -> world -x; then the tilt
    # about the plate normal
    qz = [math.cos(math.pi / 4), 0.0, 0.0, math.sin(math.pi / 4)]
    qt = [math.cos(th / 2), -math.sin(th / 2), 0.0, 0.0]
    q = _qmul(qt, qz)
    low = 0.5 * L * math.sin(th) + 0.5 * H * math.cos(th)
    inertia = [mass * (H * H + T * T) / 12.0, mass * (L * L + H * H) / 12.0, mass * (L * L + T * T) / 12.0]
    knives = []
    for k, sp in enumerate(speeds):
        x = [(k + 0.5) / len(speeds) * hi[0], 0.5 * hi[1], hi[2] + drop + low]
        body = dict(x=x, q=q, v=[0.0, 0.0, -float(sp)], omega=[0.0, 0.0, 0.0], mass=float(mass), inertia=inertia)
        bl = dict(knife_blade_body(0.5 * L, H, dx), cut_index=k)
        knives.append(dict(body=body, blade=bl))
    sc = _finish("thrown-knives", params, X, 1200.0, 2.0e4, rng, steps, None)
    sc["knives"] = dict(bodies=knives, interval=int(interval))
    return sc


def quadratic(scene):
    """The same scene on the 27-node quadratic B-spline stencil (reading R33)."""
    scene["params"] = dict(scene["params"], stencil=1)
    scene["name"] = scene.get("name", "") + "-quad"
    return scene


CONFIGS = {"small": small, "small-deep": lambda **k: small(deep=True, **k), "medium": medium,
           "medium-quad": lambda **k: quadratic(medium(**k)), "large-quad": lambda **k: quadratic(large(**k)),
           "large": large,
           # the large box at the particle count the scene description states (~4.7M);
           # its literal dx = 1.5 mm gives 14.2M
           "large-4.7m": lambda **k: large(dx=0.00217, **k)}
