"""GPU path (through the C ABI) against the FP64 oracle on the same seeded inputs.

Tolerances: labels bit-exact in shared-input mode, and in independent rollouts any
label that differs must come from a particle within the FP32-vs-FP64 state
difference of a band face (reading R25b); after one substep the displacement
u = x - X, the velocity and H = F - I are within 1e-5 of the oracle's, each
relative to its own largest value; after 100 substeps positions are within 1e-3
relative to the largest displacement.
"""
import numpy as np
import pytest

import oracle
from paper_2609_27342_amd import workloads as W

from harness import LabelWatch, disp_err, field_err, gpu_x, oracle_substep, state_errs

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


@pytest.mark.parametrize("deep", [False, True])
def test_one_substep_parity(tl, deep):
    s = W.small(deep=deep)
    _print_case("one_substep", scene=s["name"], n=s["X"].shape[0])
    g = tl.Scene(s)
    o = oracle.OracleScene(s)
    tools = s["tools_at"](0)
    g.step(tools)
    oracle_substep(o, tools)
    a = g.read(("u", "v", "F", "H", "digits"))
    b = o.get()
    assert np.array_equal(a["digits"], b["digits"])
    eu, ev, eH = state_errs(a, b, s["X"], s["params"])
    print(f"[one_substep] {s['name']} u {eu:.2e} v {ev:.2e} H {eH:.2e}", flush=True)
    assert eu < 1e-5 and ev < 1e-5 and eH < 1e-5, (eu, ev, eH)
    assert g.status() == 0
    if deep:
        tot, mx = g.slot_stats()
        assert mx >= 2  # 0/1/2 mixes exist at step 1


def test_labels_bit_exact_shared_input(tl):
    """Reading R25(a): the oracle's label pass on the GPU's own FP32 state gives
    the GPU's labels exactly, substep after substep."""
    s = W.small(deep=True)
    _print_case("labels_shared", scene=s["name"])
    g = tl.Scene(s)
    dt = s["params"]["dt"]
    for j in range(0, 40, 3):
        tools = s["tools_at"](j)
        pre = g.read(("u", "v", "digits"))
        g.assign_labels([t["blade"] for t in tools])
        post = g.read(("digits",))["digits"]
        ref = oracle.labels_on(s["X"], pre["u"], pre["v"], pre["digits"], [t["blade"] for t in tools], dt)
        assert np.array_equal(post, ref), j
        g.step([dict(t, labels=False) for t in tools])
    assert (post != 0).sum() > 1000


def test_hundred_substeps_positions(tl):
    s = W.small(deep=True)
    _print_case("hundred", scene=s["name"])
    g = tl.Scene(s)
    o = oracle.OracleScene(s)
    watch = LabelWatch(s["X"], s["params"]["dt"])
    for j in range(100):
        tools = s["tools_at"](j)
        watch.before(g, o, tools)
        g.step(tools)
        oracle_substep(o, tools)
        watch.after(g, o)
    a = g.read(("u", "v", "digits"))
    b = o.get()
    e = disp_err(gpu_x(a, s["X"]), b["x"], s["X"])
    print(f"[hundred] disp {e:.2e} label mismatches {watch.mismatched()} checked {watch.checked}", flush=True)
    assert not watch.bad, watch.bad[:5]
    assert e < 1e-3
    assert g.status() == 0


def test_determinism_bitwise(tl):
    s = W.small(deep=True)
    outs = []
    for _ in range(2):
        g = tl.Scene(s)
        for j in range(5):
            g.step(s["tools_at"](j))
        outs.append(g.read(("u", "v", "F", "H")))
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


@pytest.mark.parametrize("beta,cuts", [(0.0, 1), (0.95, 1), (1.0, 1), (0.95, 2)])
def test_momentum_conservation_gpu(tl, beta, cuts):
    """Prop. 1 on the GPU: no external force, random F, v and codes; total
    momentum is kept to FP32 rounding and the state matches the oracle's.  With one
    cut every particle draws a random digit (up to 3 logical grids per node); with
    two cuts each half of the box draws one of the digits."""
    s = W.box_scene(n_cells=(9, 7, 6), seed=12, floor_on=0, gravity=[0.0, 0.0, 0.0], flip_beta=beta,
                    max_cuts=cuts)
    n = s["X"].shape[0]
    rng = np.random.default_rng(13)
    F = (np.eye(3)[None] + 0.05 * rng.normal(size=(n, 3, 3))).astype(np.float32)
    v = (rng.normal(size=(n, 3)) * 0.1).astype(np.float32)
    dig = np.zeros((n, cuts), np.uint8)
    if cuts == 1:
        dig[:, 0] = rng.integers(0, 3, size=n)
    else:
        left = s["X"][:, 0] < 0.045
        dig[left, 0] = rng.integers(0, 3, size=left.sum())
        dig[~left, 1] = rng.integers(0, 3, size=(~left).sum())
    _print_case("momentum", beta=beta, cuts=cuts, n=n)
    g = tl.Scene(s)
    g.write(v=v, F=F, digits=dig)
    o = oracle.OracleScene(s)
    o.set(v=v, F=F.reshape(n, 9), digits=dig)
    m = s["mass"].astype(np.float64)
    P0 = (m[:, None] * v).sum(axis=0)
    scale = (m[:, None] * np.abs(v)).sum()
    for _ in range(3):
        g.step([])
        o.step([])
    assert g.status() == 0
    a = g.read(("u", "v", "F", "H"))
    P1 = (m[:, None] * a["v"]).sum(axis=0)
    assert np.abs(P1 - P0).max() < 1e-5 * scale
    b = o.get()
    eu, ev, eH = state_errs(a, b, s["X"], s["params"])
    print(f"[momentum] beta={beta} cuts={cuts} u {eu:.2e} v {ev:.2e} H {eH:.2e}", flush=True)
    assert eu < 1e-5 and ev < 1e-5 and eH < 1e-5, (eu, ev, eH)


def test_zero_exchange_gpu(tl):
    """Opposite labels everywhere a node is shared: the resting half stays exactly
    at rest (bitwise zero velocity and displacement)."""
    s = W.box_scene(n_cells=(8, 4, 4), seed=16, floor_on=0, gravity=[0.0, 0.0, 0.0], max_cuts=1)
    X = s["X"].astype(np.float64)
    n = X.shape[0]
    A = X[:, 0] < 0.04
    rng = np.random.default_rng(17)
    v = np.zeros((n, 3), np.float32)
    v[A] = rng.normal(size=(A.sum(), 3)) * 0.2
    F = np.tile(np.eye(3, dtype=np.float32), (n, 1, 1))
    F[A] += (0.02 * rng.normal(size=(A.sum(), 3, 3))).astype(np.float32)
    g = tl.Scene(s)
    g.write(v=v, F=F, digits=np.where(A, 1, 2).astype(np.uint8)[:, None])
    for _ in range(5):
        g.step([])
    a = g.read(("u", "v"))
    assert np.all(a["v"][~A] == 0.0)
    assert np.all(a["u"][~A] == 0.0)
    assert np.abs(a["v"][A]).max() > 0.01


def test_uniform_translation_gpu(tl):
    v0 = (0.3, -0.2, 0.1)
    s = W.box_scene(n_cells=(9, 6, 5), seed=14, floor_on=0, gravity=[0.0, 0.0, 0.0], v0=v0)
    g = tl.Scene(s)
    dt = s["params"]["dt"]
    g.step([], n_substeps=4)
    a = g.read(("u", "v", "F", "H"))
    vv = np.array(v0, np.float32).astype(np.float64)
    assert np.abs(a["v"] - vv).max() < 1e-6
    assert np.abs(a["F"] - np.eye(3)).max() < 1e-6
    assert np.abs(a["u"] - 4 * dt * vv).max() < 1e-9


def test_nonfinite_status(tl):
    s = W.box_scene(n_cells=(5, 5, 5), seed=3, floor_on=0)
    g = tl.Scene(s)
    n = s["X"].shape[0]
    F = np.tile(np.eye(3, dtype=np.float32), (n, 1, 1))
    F[7] = -np.eye(3)  # det F < 0
    g.write(F=F)
    g.step([])
    assert g.status() == tl.E_NONFINITE


def test_split_bricks_parity_and_determinism(tl):
    """A scene of 512+ bricks (its mixed bricks' later same-code rounds run in
    workgroups of their own): a blade cuts a 22 x 16 x 8 cm block with material
    contact; 20 substeps against the oracle, and two GPU runs bitwise equal."""
    s = W.box_scene(n_cells=(44, 32, 16), dx=0.005, seed=41, floor_on=1, material_contact=1, max_cuts=1)
    n = s["X"].shape[0]
    dt = s["params"]["dt"]

    def tools_at(j):
        b = W.blade(0, (0.081, 0.08, 0.07 - 0.3 * j * dt), (1, 0, 0), (0, 0, -1), (0, 0, -0.3), 0.12, 0.03, 0.05,
                    0.005, new_cut=(j == 0))
        return [W.tool(b, labels=True, contact=True, cutting=True)]

    _print_case("split_bricks", n=n)
    runs = []
    for _ in range(2):
        g = tl.Scene(s)
        for j in range(20):
            g.step(tools_at(j))
        assert g.status() == 0
        runs.append(g.read(("u", "v", "F", "H", "digits")))
    for f in ("u", "v", "F", "digits"):
        assert np.array_equal(runs[0][f], runs[1][f]), f
    o = oracle.OracleScene(s)
    g = tl.Scene(s)
    watch = LabelWatch(s["X"], dt)
    for j in range(20):
        watch.before(g, o, tools_at(j))
        g.step(tools_at(j))
        oracle_substep(o, tools_at(j))
        watch.after(g, o)
    b = o.get()
    a = g.read(("u", "v", "F", "H", "digits"))
    for f in ("u", "v", "F", "digits"):
        assert np.array_equal(a[f], runs[0][f]), f
    assert (b["digits"] > 0).sum() > 1000  # the cut went through many cells
    e = disp_err(gpu_x(a, s["X"]), b["x"], s["X"])
    print(f"[split] disp {e:.2e} label mismatches {watch.mismatched()} checked {watch.checked}", flush=True)
    assert not watch.bad, watch.bad[:5]
    assert e < 1e-3


def test_one_stream_launches_equal_two_stream_launches(tl):
    """A small scene's substeps with a label pass run on one stream (label pass and
    rigid contact in one launch, slot tables in the pair-search launch); with kernel
    timing on they run one kernel per launch instead.  Both orders give the same
    state bitwise: the kernels paired in one launch touch disjoint data."""
    s = W.small(deep=True)
    s["params"] = dict(s["params"], material_contact=1)
    _print_case("one stream vs timed launches", n=s["X"].shape[0])
    outs = []
    for timed in (False, True):
        g = tl.Scene(s)
        g.profile(timed)
        for j in range(30):
            g.step(s["tools_at"](j))
        assert g.status() == 0
        outs.append(g.read(("u", "v", "F", "H", "digits")))
    assert outs[0]["digits"].any()
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k
