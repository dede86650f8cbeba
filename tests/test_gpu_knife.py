"""Two-way coupling (a free knife, reading R30): the GPU path with the library's
rigid step against the FP64 oracle with its own rigid step, each driving its knife
by its own interval-averaged wrench.

Small knife scene (16,000 particles, dx = 4 mm), 16 intervals of 5 substeps; the
knife reaches the block in the fourth interval and starts the cut in the sixth.
Thrown knives (three free knives at 0.5, 0.8 and 1.1 m/s on a fixed-corotated block
with von Mises plasticity; 24,000 particles, dx = 4 mm), 16 intervals of 5 substeps:
all three cuts start.
Tolerances (FP32 state against FP64, the two knives moved by their own wrenches):
knife position and velocity within 1e-3 of their change over the run, angular
velocity within 2 % of its largest component plus 1e-3 rad/s, particle positions
within 1e-3 relative to the largest displacement, side digits equal for at least
99.5 % of the particles (the two knives move apart by their own rounding).  Label
parity proper (reading R25b) is checked with both sides driven by the same knife:
the oracle's tool records, interval by interval, stepped one substep at a time.
"""
import numpy as np
import pytest

import oracle
from oracle.rigid import Body
from paper_2609_27342_amd import workloads as W

from harness import LabelWatch, disp_err, gpu_x, oracle_substep

pytestmark = pytest.mark.gpu

N_INTERVALS = 16


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_27342_amd import tlmpm
    tlmpm.lib()
    return tlmpm


def _scene():
    return W.knife(dx=0.004, interval=5, drop=0.0005, v_drop=0.5)


def _oracle_run(sc):
    o = oracle.OracleScene(sc)
    k = sc["knife"]
    b = Body(k["body"]["x"], k["body"]["q"], k["body"]["v"], k["body"]["omega"], k["body"]["mass"],
             k["body"]["inertia"])
    g = np.asarray(sc["params"]["gravity"], np.float64)
    dt, n = sc["params"]["dt"], k["interval"]
    forces = []
    for it in range(N_INTERVALS):
        tool = b.tool(dict(k["blade"], new_cut=int(it == 0)))
        ws = np.zeros(6)
        for _ in range(n):
            st, w = oracle_substep(o, [tool])
            assert st == 0
            ws += w[0]
        ws /= n
        forces.append(ws)
        b.step(ws, g, n * dt)
    return o.get(), b, np.array(forces)


def test_knife_two_way_coupling_parity(tl):
    from paper_2609_27342_amd.coupling import KnifeRollout
    sc = _scene()
    print(f"[case] knife n={sc['X'].shape[0]} intervals={N_INTERVALS}", flush=True)
    g = tl.Scene(sc)
    ro = KnifeRollout(g, sc)
    forces = []
    for _ in range(N_INTERVALS):
        forces.append(ro.advance(1))
    assert g.status() == 0
    a = g.read(("u", "v", "digits"))
    b, ob, of = _oracle_run(sc)
    gs = ro.body.state()
    k0 = sc["knife"]["body"]
    # the knife touched the material and the cut started
    assert np.abs(of[:, :3]).max() > 1e-3
    assert (b["digits"] > 0).sum() > 10
    dx_ref = np.linalg.norm(ob.x - np.asarray(k0["x"]))
    dv_ref = np.linalg.norm(ob.v - np.asarray(k0["v"]))
    assert np.linalg.norm(gs["x"] - ob.x) < 1e-3 * dx_ref
    assert np.linalg.norm(gs["v"] - ob.v) < 1e-3 * dv_ref
    assert np.abs(gs["omega"] - ob.w).max() < 0.02 * np.abs(ob.w).max() + 1e-3
    assert disp_err(gpu_x(a, sc["X"]), b["x"], sc["X"]) < 1e-3
    agree = np.mean(np.all(a["digits"] == b["digits"], axis=1))
    assert agree >= 0.995
    print(f"[knife] dx {np.linalg.norm(gs['x'] - ob.x) / dx_ref:.2e} dv {np.linalg.norm(gs['v'] - ob.v) / dv_ref:.2e} "
          f"dw {np.abs(gs['omega'] - ob.w).max():.2e} (|w| {np.abs(ob.w).max():.3f}) "
          f"disp {disp_err(gpu_x(a, sc['X']), b['x'], sc['X']):.2e} digits {agree:.5f}", flush=True)


def test_heavy_knife_is_kinematic(tl):
    """A knife of huge mass and inertia has a vanishing inverse effective mass: its
    contacts match those of the same pose and twist given as a prescribed tool."""
    sc = _scene()
    k = sc["knife"]
    heavy = dict(k["body"], mass=1e12, inertia=[1e12, 1e12, 1e12])
    body = tl.RigidBody(**heavy)
    g1, g2 = tl.Scene(sc), tl.Scene(sc)
    for it in range(8):
        t = body.tool(dict(k["blade"], new_cut=int(it == 0)))
        g1.step([t], k["interval"])
        g2.step([dict(t, inv_mass=0.0, inv_inertia=np.zeros(9))], k["interval"])
        body.step(np.zeros(6), [0.0, 0.0, 0.0], k["interval"] * sc["params"]["dt"])
    a, b = g1.read(("u", "v", "digits")), g2.read(("u", "v", "digits"))
    assert np.array_equal(a["digits"], b["digits"])
    assert np.abs(a["v"] - b["v"]).max() <= 1e-6 * max(1.0, np.abs(b["v"]).max())
    assert np.abs(a["u"] - b["u"]).max() <= 1e-9


def _oracle_run_many(sc, n_intervals):
    o = oracle.OracleScene(sc)
    ks = sc["knives"]["bodies"]
    bs = [Body(k["body"]["x"], k["body"]["q"], k["body"]["v"], k["body"]["omega"], k["body"]["mass"],
               k["body"]["inertia"]) for k in ks]
    g = np.asarray(sc["params"]["gravity"], np.float64)
    dt, n = sc["params"]["dt"], sc["knives"]["interval"]
    for it in range(n_intervals):
        tools = [b.tool(dict(k["blade"], new_cut=int(it == 0))) for b, k in zip(bs, ks)]
        ws = np.zeros((len(bs), 6))
        for _ in range(n):
            st, w = oracle_substep(o, tools)
            assert st == 0
            ws += np.asarray(w)
        ws /= n
        for b, w in zip(bs, ws):
            b.step(w, g, n * dt)
    return o.get(), bs


def test_thrown_knives_parity(tl):
    from paper_2609_27342_amd.coupling import KnifeRollout
    sc = W.thrown_knives(dx=0.004, interval=5, drop=0.0005)
    print(f"[case] thrown knives n={sc['X'].shape[0]} intervals={N_INTERVALS}", flush=True)
    g = tl.Scene(sc)
    ro = KnifeRollout(g, sc)
    ro.advance(N_INTERVALS)
    assert g.status() == 0
    a = g.read(("u", "v", "digits"))
    b, obs = _oracle_run_many(sc, N_INTERVALS)
    for c in range(3):
        assert (b["digits"][:, c] > 0).sum() > 0, c
    for gb, ob, k in zip(ro.bodies, obs, sc["knives"]["bodies"]):
        gs = gb.state()
        dx_ref = np.linalg.norm(ob.x - np.asarray(k["body"]["x"]))
        dv_ref = np.linalg.norm(ob.v - np.asarray(k["body"]["v"]))
        assert np.linalg.norm(gs["x"] - ob.x) < 1e-3 * dx_ref
        assert np.linalg.norm(gs["v"] - ob.v) < 1e-3 * dv_ref
        assert np.abs(gs["omega"] - ob.w).max() < 0.02 * np.abs(ob.w).max() + 1e-3
    e = disp_err(gpu_x(a, sc["X"]), b["x"], sc["X"])
    agree = np.mean(np.all(a["digits"] == b["digits"], axis=1))
    print(f"[thrown] disp {e:.2e} digits {agree:.5f}", flush=True)
    assert e < 1e-3
    assert agree >= 0.995


@pytest.mark.parametrize("which", ["knife", "thrown"])
def test_knife_labels_with_shared_tool_records(tl, which):
    """Reading R25b on the free-knife scenes: the GPU scene and the oracle are both
    driven by the oracle's knives (their tool records, held over each interval and
    advanced by the oracle's interval-averaged wrench), one substep at a time in
    lockstep; every label that differs must belong to a particle within the
    FP32-vs-FP64 state difference of a band face."""
    sc = _scene() if which == "knife" else W.thrown_knives(dx=0.004, interval=5, drop=0.0005)
    ks = [sc["knife"]] if which == "knife" else sc["knives"]["bodies"]
    n = sc["knife"]["interval"] if which == "knife" else sc["knives"]["interval"]
    X = sc["X"].astype(np.float64)
    dt = sc["params"]["dt"]
    grav = np.asarray(sc["params"]["gravity"], np.float64)
    print(f"[case] knife labels {which} n={X.shape[0]}", flush=True)
    g = tl.Scene(sc)
    o = oracle.OracleScene(sc)
    bodies = [Body(k["body"]["x"], k["body"]["q"], k["body"]["v"], k["body"]["omega"], k["body"]["mass"],
                   k["body"]["inertia"]) for k in ks]
    watch = LabelWatch(X, dt)
    for it in range(N_INTERVALS):
        tools = [b.tool(dict(k["blade"], new_cut=int(it == 0))) for b, k in zip(bodies, ks)]
        ws = np.zeros((len(tools), 6))
        for sub in range(n):
            tk = tools if sub == 0 else [dict(t, blade=dict(t["blade"], new_cut=0)) for t in tools]
            watch.before(g, o, tk)
            g.step(tk, 1)
            st, w = oracle_substep(o, tk)
            assert st == 0
            watch.after(g, o)
            ws += np.asarray(w)
        ws /= n
        for b, w in zip(bodies, ws):
            b.step(w, grav, n * dt)
    assert g.status() == 0
    b = o.get()
    a = g.read(("u", "digits"))
    e = disp_err(gpu_x(a, X), b["x"], X)
    print(f"[knife labels {which}] disp {e:.2e} labelled {(b['digits'] != 0).sum()} mismatches {watch.mismatched()} "
          f"checked {watch.checked}", flush=True)
    assert (b["digits"] != 0).sum() > 10
    assert not watch.bad, watch.bad[:5]
    assert e < 1e-3
