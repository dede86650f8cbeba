"""Contact on the GPU (through the C ABI) against the FP64 oracle.

Floor, blade (with cutting work) and material-pair contact are held to 1e-5 after
one substep and over the first substeps of the full-size curved-cylinder scene,
and checked against closed forms (the cutting-work release count and the wrench
balance, separation under gravity).  The tool contact geometry is evaluated in
FP64 on the GPU from the FP32 state: its normal impulse is s_n m / dt times the
gap, and the normal of a particle next to the zero-thickness blade is the
direction of a short vector, both far more sensitive than the state itself.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2609_27342_amd import workloads as W

from harness import LabelWatch, disp_err, field_err, gpu_x, oracle_substep, oracle_tools, state_errs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_27342_amd import tlmpm
    tlmpm.lib()
    return tlmpm


def _print_case(name, **kw):
    print(f"[case] {name} {kw}", flush=True)


def _pressed_pieces(seed=19):
    """Two pieces of a box labelled 1 | 2, the right one pushed 4 mm into the left."""
    s = W.box_scene(n_cells=(6, 3, 3), seed=seed, floor_on=0, gravity=[0.0, 0.0, 0.0], material_contact=1,
                    max_cuts=1)
    X = s["X"].astype(np.float64)
    left = X[:, 0] < 0.03
    rng = np.random.default_rng(20)
    u = np.zeros_like(X)
    u[~left, 0] = -0.004
    v = rng.normal(size=X.shape) * 0.05
    return s, left, u.astype(np.float32), v.astype(np.float32)


def test_material_contact_parity(tl):
    s, left, u, v = _pressed_pieces()
    n = s["X"].shape[0]
    dig = np.where(left, 1, 2).astype(np.uint8)[:, None]
    _print_case("material_contact", n=n)
    g = tl.Scene(s)
    g.write(u=u, v=v, digits=dig)
    o = oracle.OracleScene(s)
    X = s["X"].astype(np.float64)
    o.set(x=X + u, v=v, digits=dig)
    for _ in range(3):
        g.step([])
        o.step([])
        assert o.last_pairs() > 10
    assert g.status() == 0
    a = g.read(("u", "v", "F", "H"))
    b = o.get()
    eu, ev, eH = state_errs(a, b, X, s["params"])
    print(f"[material_contact] 3 substeps u {eu:.2e} v {ev:.2e} H {eH:.2e}", flush=True)
    assert eu < 1e-5 and ev < 1e-5 and eH < 1e-5, (eu, ev, eH)
    assert disp_err(gpu_x(a, X), b["x"], X) < 1e-3


def test_material_contact_momentum_and_determinism(tl):
    """Pair impulses are equal and opposite (Eq. 13): total momentum is unchanged
    by contact; two runs agree bitwise."""
    s, left, u, v = _pressed_pieces(seed=21)
    dig = np.where(left, 1, 2).astype(np.uint8)[:, None]
    m = s["mass"].astype(np.float64)
    outs = []
    for _ in range(2):
        g = tl.Scene(s)
        g.write(u=u, v=v, digits=dig)
        for _ in range(4):
            g.step([])
        outs.append(g.read(("u", "v")))
    assert np.array_equal(outs[0]["v"], outs[1]["v"]) and np.array_equal(outs[0]["u"], outs[1]["u"])
    P0 = (m[:, None] * v).sum(axis=0)
    P1 = (m[:, None] * outs[0]["v"]).sum(axis=0)
    scale = (m[:, None] * np.abs(outs[0]["v"])).sum()
    assert np.abs(P1 - P0).max() < 1e-5 * scale


def _single_particle(params_kw, X=(0.0025, 0.0025, 0.0025), dens=1000.0):
    p = W.base_params(0.01, (-0.05, -0.05, -0.05), (10, 10, 10), 1e-4, 0.3, **params_kw)
    V0 = np.float32(0.01 ** 3 / 8)
    return dict(params=p, X=np.array([X], np.float32), v0=None, vol0=np.array([V0], np.float32),
                mass=np.array([V0 * dens], np.float32), E=np.array([1e4], np.float32), name="one")


def test_cutting_work_release_and_wrench(tl):
    """Eq. 5 on the GPU: the forward impulse is applied for exactly
    ceil(W_th / (J_c u_c)) substeps under a constant load, then released; Eq. 16:
    m dv = -F_B dt."""
    s = _single_particle(dict(floor_on=0, gravity=[0.0, 0.0, 0.0], G_c=50.0, zeta=0.5))
    V0 = float(s["vol0"][0])
    m = float(s["mass"][0])
    R = 0.5 * V0 ** (1.0 / 3.0)
    X0 = s["X"][0].astype(np.float64)
    b = W.blade(0, (0.0, 0.0, 0.001 + R * 0.5), (1, 0, 0), (0, 0, -1), (0, 0, -1.0), 0.05, 0.03, 0.04, 0.01,
                new_cut=True)
    T = W.tool(b, labels=False, contact=True, cutting=True, x_B=(0, 0, 0.02), v_B=(0, 0, -1.0))
    g = tl.Scene(s)
    g.assign_labels([b])
    dt = 1e-4
    gap = 0.001 + 0.5 * R - R
    phihat = gap + dt * min(-1.0, 0.0)
    Jn = 0.5 * m / dt * max(-phihat, 0.0)
    Wth = 50.0 * V0 ** (2.0 / 3.0)
    expect = math.ceil(Wth / (Jn * 1.0))
    pushed = 0
    u0 = (np.zeros(3) - X0).astype(np.float32)[None, :]  # current position at the origin
    for j in range(expect + 3):
        g.write(u=u0, v=np.zeros((1, 3), np.float32))
        w = g.step([dict(T, blade=dict(b, new_cut=0))], wrench=True)
        dv = g.read(("v",))["v"][0].astype(np.float64)
        if dv[2] < -1e-6:
            pushed += 1
            assert np.allclose(m * dv, -w[0][:3] * dt, rtol=1e-5, atol=1e-12)
            assert abs(m * dv[2] + Jn) < 1e-5 * Jn
        else:
            assert np.abs(dv).max() < 1e-7
    assert pushed == expect
    assert g.read(("D",))["D"][0] == 1.0


def test_separation_under_gravity_gpu(tl):
    """Fully cut bar on a support plate: the overhang falls freely on the GPU as in
    the oracle; with one shared grid it is held."""
    t = 300 * 1e-4
    free = -0.5 * 9.81 * t * t
    res = {}
    for sf in (0, 1):
        s = W.box_scene(n_cells=(10, 2, 2), dx=0.01, seed=18, E=2e5, floor_on=0, max_cuts=1, single_field=sf,
                        dt=1e-4)
        X = s["X"].astype(np.float64)
        right = X[:, 0] >= 0.05
        plate = W.blade(0, (0.045, 0.01, -0.00125), (0, 0, 1), (1, 0, 0), (0, 0, 0), 0.03, 0.0, 0.055, 0.0)
        T = W.tool(plate, labels=False, contact=True, cutting=False)
        g = tl.Scene(s)
        dig = np.where(right, 2, 1).astype(np.uint8)[:, None]
        g.write(digits=dig)
        o = oracle.OracleScene(s)
        o.set(digits=dig)
        for _ in range(300):
            g.step([T])
            o.step(oracle_tools([T]))
        a = g.read(("u",))
        b = o.get()
        dr = a["u"][right, 2].mean()
        res[sf] = dr
        assert abs(dr - (b["x"][right, 2] - X[right, 2]).mean()) < 0.02 * abs(free)
    assert res[0] < 0.9 * free
    assert res[1] > 0.7 * free


def test_medium_one_substep_contact_parity(tl):
    """One substep of the curved-cylinder scene (full size) with the cutting blade
    inserted to z = 0.02: floor contact, blade contact with cutting work and
    material pairs across the fresh cut all act in this substep.  Labels equal and
    u, v, H within 1e-5 of the oracle's, each relative to its own largest value."""
    s = W.medium(z_start=0.02)
    _print_case("medium one substep", n=s["X"].shape[0])
    g = tl.Scene(s)
    o = oracle.OracleScene(s)
    X = s["X"].astype(np.float64)
    tools = s["tools_at"](0)
    g.step(tools)
    oracle_substep(o, tools)
    assert o.last_pairs() > 100
    assert g.status() == 0
    a = g.read(("u", "v", "F", "H", "digits"))
    b = o.get()
    assert np.array_equal(a["digits"], b["digits"])
    assert (b["digits"] != 0).sum() > 1000
    eu, ev, eH = state_errs(a, b, X, s["params"])
    print(f"[medium one substep] u {eu:.2e} v {ev:.2e} H {eH:.2e} pairs {o.last_pairs()}", flush=True)
    assert eu < 1e-5 and ev < 1e-5 and eH < 1e-5, (eu, ev, eH)


def test_medium_first_substeps_parity(tl):
    """The same scene over its first 5 substeps: labels equal and u, v, H within 1e-5
    after every substep."""
    s = W.medium(z_start=0.02)
    _print_case("medium", n=s["X"].shape[0])
    g = tl.Scene(s)
    o = oracle.OracleScene(s)
    X = s["X"].astype(np.float64)
    for j in range(5):
        tools = s["tools_at"](j)
        g.step(tools)
        oracle_substep(o, tools)
        a = g.read(("u", "v", "F", "H"))
        print(f"[medium] substep {j + 1} u/v/H " + " ".join(f"{e:.2e}" for e in state_errs(a, o.get(), X, s["params"])),
              flush=True)
    assert g.status() == 0
    a = g.read(("u", "v", "F", "H", "digits"))
    b = o.get()
    assert np.array_equal(a["digits"], b["digits"])
    eu, ev, eH = state_errs(a, b, X, s["params"])
    assert eu < 1e-5 and ev < 1e-5 and eH < 1e-5, (eu, ev, eH)
    assert disp_err(gpu_x(a, X), b["x"], X) < 1e-3
