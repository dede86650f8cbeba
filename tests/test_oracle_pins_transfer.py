"""Pins of the oracle's deformation-gradient update, MUSL remap, tool torque and
contact candidate rule, each shown to fail under the mistake it targets.

Every pin is a function of the oracle library it runs on.  The plain test runs it
on oracle/liboracle.so and checks it passes; the mutation test builds a copy of
oracle/tlmpm_oracle.c with one planted mistake (a transposed outer product, the
grid velocity in place of the remapped one, swapped cross-product operands, a
dropped conflict rule) on the CPU and checks that the same pin then fails.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import build as obuild
from paper_2609_27342_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dyadic_params(**kw):
    """Grid and step of power-of-two sizes, so that the hand values are exact."""
    p = W.base_params(2.0 ** -6, (0.0, 0.0, 0.0), (4, 4, 4), 2.0 ** -13, 0.3, floor_on=0,
                      gravity=[0.0, 0.0, 0.0], max_cuts=1)
    p.update(kw)
    return p


# ---------------------------------------------------------------- F update (MUSL)
def pin_homogeneous_deformation(L):
    """Sec. III-B (MUSL F update), Eq. 1: on an unjittered lattice with v = A (X - c)
    and F = I there is no stress, the symmetric lattice makes every node with all
    its cells filled carry v_i = A (x_i - c), linear reproduction gives each
    particle v = A (X - c) again, and sum_i x_i (x) grad N_ip = I; so a particle
    whose stencil nodes see only such particles ends at F = I + dt A exactly, for a
    non-symmetric A.  Returns max |F - (I + dt A)| over those particles."""
    dx = 2.0 ** -7  # lattice positions exact in float32, so the lattice stays symmetric
    s = W.box_scene(n_cells=(8, 8, 8), dx=dx, seed=31, jitter=0.0, floor_on=0, gravity=[0.0, 0.0, 0.0])
    X = s["X"].astype(np.float64)
    A = np.array([[0.3, 1.1, -0.4], [-0.7, 0.2, 0.9], [0.5, -1.3, -0.1]])
    c = np.array([4 * dx, 4 * dx, 4 * dx])
    v = (X - c) @ A.T
    o = oracle.OracleScene(s, L)
    o.set(v=v)
    st, _ = o.step([])
    assert st == 0
    g = o.get()
    dt = s["params"]["dt"]
    cell = np.floor(X / dx).astype(int)
    inner = np.all((cell >= 2) & (cell <= 5), axis=1)
    assert inner.sum() == 4 ** 3 * 8
    return np.abs(g["F"][inner] - (np.eye(3) + dt * A)[None]).max()


def test_homogeneous_deformation_gives_I_plus_dt_A():
    assert pin_homogeneous_deformation(oracle.lib()) < 1e-12


def pin_rigid_rotation(L):
    """A rigid rotation rate v = w x (X - c) is a skew A: F = I + dt A is a rotation
    to first order, F^T F - I = dt^2 A^T A.  Returns max |F^T F - I - dt^2 A^T A|."""
    dx = 2.0 ** -7
    s = W.box_scene(n_cells=(8, 8, 8), dx=dx, seed=32, jitter=0.0, floor_on=0, gravity=[0.0, 0.0, 0.0])
    X = s["X"].astype(np.float64)
    w = np.array([0.8, -1.5, 2.2])
    A = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    c = np.array([4 * dx, 4 * dx, 4 * dx])
    o = oracle.OracleScene(s, L)
    o.set(v=(X - c) @ A.T)
    o.step([])
    F = o.get()["F"]
    dt = s["params"]["dt"]
    cell = np.floor(X / dx).astype(int)
    inner = np.all((cell >= 2) & (cell <= 5), axis=1)
    FtF = np.einsum("pki,pkj->pij", F[inner], F[inner])
    return np.abs(FtF - np.eye(3)[None] - dt * dt * (A.T @ A)[None]).max()


def test_rigid_rotation_keeps_F_orthogonal_to_first_order():
    assert pin_rigid_rotation(oracle.lib()) < 1e-13


def _musl_scene(beta):
    gd = json.load(open(os.path.join(GOLDEN, "musl_two_particles.json")))
    su = gd["setup"]
    p = _dyadic_params(flip_beta=beta)
    assert p["dx"] == su["dx"] and p["dt"] == su["dt"]
    X = np.array([su["X_a"], su["X_b"]], np.float32)
    V0 = np.float32(su["dx"] ** 3 / 8)
    sc = dict(params=p, X=X, v0=np.array([su["v_a"], su["v_b"]], np.float32), vol0=np.full(2, V0, np.float32),
              mass=np.full(2, su["mass"], np.float32), E=np.full(2, 1e4, np.float32))
    return gd, sc


def pin_musl_golden(L):
    """tests/golden/musl_two_particles.json: two particles in one cell moving
    toward each other, worked by hand (Sec. III-B MUSL, Eq. 17); the remapped
    velocity, not the grid velocity, enters F.  Returns the largest deviation from
    the hand values over the cases."""
    gd, _ = _musl_scene(0.0)
    err = 0.0
    for case in gd["cases"]:
        _, sc = _musl_scene(case["beta"])
        o = oracle.OracleScene(sc, L)
        st, _ = o.step([])
        assert st == 0
        g = o.get()
        X = sc["X"].astype(np.float64)
        Fx = np.eye(3)
        Fx[0, 0] = case["F_xx"]
        err = max(err, np.abs(g["v"][0] - case["v_a"]).max(), np.abs(g["v"][1] - case["v_b"]).max(),
                  abs(g["x"][0, 0] - X[0, 0] - case["dx_a"]), abs(g["x"][1, 0] - X[1, 0] + case["dx_a"]),
                  np.abs(g["x"][:, 1:] - X[:, 1:]).max(), np.abs(g["F"][0] - Fx).max(), np.abs(g["F"][1] - Fx).max())
    return err


def test_musl_two_particle_golden():
    assert pin_musl_golden(oracle.lib()) < 1e-14


# ------------------------------------------------------------------ tool torque
def pin_torque(L):
    """Eq. 16: the reaction on the tool is F_B = -J/dt and its torque about x_B is
    (x_c - x_B) x F_B with x_c the contact point on the tool.  One isolated particle
    presses into the face of a blade rectangle at a known point x_c and slides
    along it (friction gives F_B a tangential part, so x_c and the particle position
    give different torques); J is read from the particle's velocity change (an
    isolated particle receives exactly J / m, Sum N = 1).  Returns the relative
    error of the torque."""
    p = W.base_params(0.01, (0.0, 0.0, 0.0), (10, 10, 10), 1e-4, 0.3, floor_on=0, gravity=[0.0, 0.0, 0.0],
                      max_cuts=1)
    V0 = np.float32(0.01 ** 3 / 8)
    m = np.float32(V0 * 1000.0)
    R = 0.5 * float(V0) ** (1.0 / 3.0)
    b = W.blade(0, (0.05, 0.05, 0.05), (1, 0, 0), (0, 0, -1), (0, 0, 0), 0.03, 0.03, 0.04, 0.01)
    nrm = np.asarray(b["n"])
    xp = np.asarray(b["x_e"]) + 0.012 * np.asarray(b["e"]) - 0.021 * np.asarray(b["d"]) + 0.5 * R * nrm
    x32 = xp.astype(np.float32).astype(np.float64)  # the stored reference position
    xc = x32 - ((x32 - np.asarray(b["x_e"])) @ nrm) * nrm  # its foot on the blade face (inside the rectangle)
    v0 = np.array([0.0, 0.05, 0.02])
    sc = dict(params=p, X=xp.astype(np.float32)[None], v0=v0.astype(np.float32)[None],
              vol0=np.array([V0], np.float32), mass=np.array([m], np.float32), E=np.array([1e4], np.float32))
    xB = np.array([0.031, 0.072, 0.093])
    T = dict(W.tool(b, labels=False, contact=True, cutting=False, x_B=xB, v_B=(0, 0, 0)), contact=1, cutting=0)
    o = oracle.OracleScene(sc, L)
    x0 = o.get()["x"][0].copy()
    v_in = o.get()["v"][0].copy()
    st, w = o.step([T])
    assert st == 0
    dv = o.get()["v"][0] - v_in
    J = float(m) * dv
    FB = -J / 1e-4
    assert np.abs(FB[1:]).max() > 1e-3 * np.abs(FB[0])  # a tangential part is present
    assert np.allclose(w[0][:3], FB, rtol=1e-9, atol=0)
    assert np.array_equal(x0, x32)
    tau = np.cross(xc - xB, FB)
    return np.abs(w[0][3:] - tau).max() / np.abs(tau).max()


def test_torque_is_contact_arm_cross_force():
    assert pin_torque(oracle.lib()) < 1e-9


# ------------------------------------------------------- contact candidates (R17)
def pin_conflict_candidates(L):
    """Sec. III-E (reference neighbours are excluded unless their codes conflict),
    reading R17: a particle whose 3x3x3 cell block holds a conflicting code is a
    contact candidate even deep inside the body.  A full box cut at x = 0.04 into
    sides 1 | 2: interior particles (all 27 cells filled) are candidates exactly in
    the two cell layers next to the cut.  Returns the number of interior particles
    that disagree with that."""
    s = W.box_scene(n_cells=(8, 6, 6), dx=0.01, seed=33, floor_on=0, gravity=[0.0, 0.0, 0.0], material_contact=1,
                    max_cuts=1)
    X = s["X"].astype(np.float64)
    o = oracle.OracleScene(s, L)
    o.set(digits=np.where(X[:, 0] < 0.04, 1, 2).astype(np.uint8)[:, None])
    cand = o.candidates()
    cell = np.floor(X / 0.01).astype(int)
    interior = np.all(cell >= 1, axis=1) & (cell[:, 0] <= 6) & (cell[:, 1] <= 4) & (cell[:, 2] <= 4)
    expect = np.isin(cell[:, 0], (3, 4))
    assert interior.sum() > 500 and (interior & expect).sum() > 100
    return int((cand[interior] != expect[interior]).sum())


def test_conflicting_neighbour_makes_interior_candidate():
    assert pin_conflict_candidates(oracle.lib()) == 0


def pin_conflict_exemption(L):
    """Eqs. 10, 11, 13 with the self-contact exclusion of Sec. III-E: two particles
    in adjacent reference cells that overlap.  With conflicting codes (1, 2) they
    are not excluded and receive s_n m_eff / dt * delta_hat; with compatible codes
    (0, 1) they are excluded and receive nothing.  Returns the largest error against
    these two expectations, relative to the impulse."""
    p = W.base_params(0.01, (0.0, 0.0, 0.0), (6, 4, 4), 1e-4, 0.3, floor_on=0, gravity=[0.0, 0.0, 0.0],
                      material_contact=1, max_cuts=1)
    V0 = np.float32(0.01 ** 3 / 8)
    R = 0.5 * float(V0) ** (1.0 / 3.0)
    X = np.array([[0.0195, 0.015, 0.015], [0.0205, 0.015, 0.015]], np.float32)  # cells 1 and 2 along x
    m = np.array([V0 * 1000, V0 * 1000], np.float32)
    sc = dict(params=p, X=X, v0=None, vol0=np.full(2, V0, np.float32), mass=m, E=np.full(2, 1e4, np.float32))
    err = 0.0
    for dig, touch in (((1, 2), True), ((0, 1), False)):
        o = oracle.OracleScene(sc, L)
        o.set(digits=np.array(dig, np.uint8)[:, None])
        o.step([])
        g = o.get()
        d = float(X[1, 0]) - float(X[0, 0])
        meff = float(m[0]) * float(m[1]) / (float(m[0]) + float(m[1]))
        Jx = 0.5 * meff / 1e-4 * (2 * R - d)  # s_n = 0.5, on q along +x, on p along -x
        expect = -Jx / float(m[0]) if touch else 0.0
        err = max(err, abs(g["v"][0, 0] - expect) / (Jx / float(m[0])))
    return err


def test_conflicting_reference_neighbours_are_not_excluded():
    assert pin_conflict_exemption(oracle.lib()) < 1e-9


# -------------------------------------------------------------------- mutations
SRC = obuild.SRC

MUTATIONS = [
    # (name, text in tlmpm_oracle.c, planted replacement, pin, passes-if)
    ("transposed_velocity_gradient",
     "L[3 * a + b] += e->vt[a] * g[3 * k + b];",
     "L[3 * b + a] += e->vt[a] * g[3 * k + b];",
     pin_homogeneous_deformation, lambda r: r < 1e-12),
    ("grid_velocity_instead_of_remap",
     "L[3 * a + b] += e->vt[a] * g[3 * k + b];",
     "L[3 * a + b] += ((e->pbar[a] + e->dpbar[a]) / e->m) * g[3 * k + b];",
     pin_musl_golden, lambda r: r < 1e-14),
    ("dropped_velocity_term",
     "for (int i = 0; i < 9; i++) F[i] += dt * L[i];",
     "for (int i = 0; i < 9; i++) F[i] += dt * L[i] * (i % 4 == 0);",
     pin_rigid_rotation, lambda r: r < 1e-13),
    ("swapped_torque_cross_product",
     "cross3(arm, Fb, tq);",
     "cross3(Fb, arm, tq);",
     pin_torque, lambda r: r < 1e-9),
    ("particle_position_as_torque_arm",
     "double Fb[3] = {-JpB[0] / dt, -JpB[1] / dt, -JpB[2] / dt}, tq[3];",
     "double Fb[3] = {-JpB[0] / dt, -JpB[1] / dt, -JpB[2] / dt}, tq[3];"
     " for (int j = 0; j < 3; j++) arm[j] = x[j] - xB[j];",
     pin_torque, lambda r: r < 1e-9),
    ("conflict_rule_dropped_from_candidates",
     "if (orc_conflict(cp, code_of(s, list[i]), P->max_cuts)) {",
     "if (0) {",
     pin_conflict_candidates, lambda r: r == 0),
    ("conflict_exemption_dropped_from_exclusion",
     "return near && !orc_conflict(code_of(s, p), code_of(s, q), s->P.max_cuts);",
     "return near;",
     pin_conflict_exemption, lambda r: r < 1e-9),
]


@pytest.mark.parametrize("name,old,new,pin,ok", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_fails_under_planted_mistake(tmp_path, name, old, new, pin, ok):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation target of {name} not found exactly once"
    mut = tmp_path / f"oracle_{name}.c"
    mut.write_text(src.replace(old, new))
    lib = obuild.compile_source(str(mut), str(tmp_path / f"lib_{name}.so"))
    L = oracle.load(lib)
    try:
        r = pin(L)
    except AssertionError:
        return  # the pin's own checks caught the mistake
    assert not ok(r), f"pin still passes with {name}: {r}"
