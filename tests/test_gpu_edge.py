"""Edge cases of the GPU path, for both stencils: an empty scene, a single particle
(free fall in closed form), the largest number of cuts (15 ternary digits), and a
slot table too small for the codes at a node (a status error, not a fault)."""
import numpy as np
import pytest

import oracle
from paper_2609_27342_amd import workloads as W

from harness import field_err, gpu_x, state_errs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_27342_amd import tlmpm
    tlmpm.lib()
    return tlmpm


def _cloud(X, **kw):
    p = W.base_params(0.01, (-0.05, -0.05, -0.05), (10, 10, 10), 1e-4, 0.3, **kw)
    n = X.shape[0]
    V0 = np.float32(0.01 ** 3 / 8)
    return dict(params=p, X=np.asarray(X, np.float32).reshape(n, 3), v0=None, vol0=np.full(n, V0, np.float32),
                mass=np.full(n, V0 * 1000, np.float32), E=np.full(n, 1e4, np.float32), name="cloud")


@pytest.mark.parametrize("stencil", [0, 1])
def test_empty_scene(tl, stencil):
    s = _cloud(np.zeros((0, 3)), stencil=stencil, material_contact=1)
    print(f"[case] empty scene stencil={stencil}", flush=True)
    g = tl.Scene(s)
    b = W.blade(0, (0.0, 0.0, 0.01), (1, 0, 0), (0, 0, -1), (0, 0, -0.2), 0.05, 0.01, 0.04, 0.01, new_cut=True)
    w = g.step([W.tool(b)], n_substeps=3, wrench=True)
    assert g.status() == 0
    assert np.all(w == 0.0)
    a = g.read(("u", "v", "F", "H", "digits"))
    assert a["u"].shape == (0, 3) and a["F"].shape == (0, 3, 3)


@pytest.mark.parametrize("stencil", [0, 1])
def test_single_particle_free_fall(tl, stencil):
    """One particle, gravity, nothing else: the grid carries its momentum plus
    m g dt at every node, so v_n = v_0 + n g dt and x_n = x_0 + dt sum_k v_k exactly
    (to FP32 rounding), F stays I; the oracle agrees."""
    s = _cloud(np.array([[0.0031, -0.0012, 0.0047]]), stencil=stencil, floor_on=0, flip_beta=0.95)
    print(f"[case] single particle stencil={stencil}", flush=True)
    g = tl.Scene(s)
    o = oracle.OracleScene(s)
    n, dt = 20, s["params"]["dt"]
    for _ in range(n):
        g.step([])
        o.step([])
    assert g.status() == 0
    a, b = g.read(("u", "v", "F", "H")), o.get()
    gz = -9.81
    assert abs(a["v"][0, 2] - n * gz * dt) < 1e-6
    assert np.abs(a["v"][0, :2]).max() < 1e-7
    assert abs(a["u"][0, 2] - dt * dt * gz * n * (n + 1) / 2) < 1e-8
    assert np.abs(a["F"][0] - np.eye(3)).max() < 1e-6
    assert np.abs(b["v"][0] - [0.0, 0.0, n * gz * dt]).max() < 1e-12
    assert field_err(gpu_x(a, s["X"]), b["x"]) < 1e-6


@pytest.mark.parametrize("stencil", [0, 1])
def test_fifteen_cuts(tl, stencil):
    """max_cuts = 15 (the most the 15-bit side masks hold): random digits on all 15
    cuts, one substep against the oracle; the digits read back bit-exactly."""
    s = W.box_scene(n_cells=(6, 5, 4), seed=21, floor_on=0, gravity=[0.0, 0.0, 0.0], max_cuts=15, stencil=stencil,
                    slot_capacity=16)
    n = s["X"].shape[0]
    rng = np.random.default_rng(22)
    dig = np.zeros((n, 15), np.uint8)
    # the first, a middle and the last digit in use; at most 4 codes meet at a node
    left = s["X"][:, 0] < 0.03
    dig[left, 14] = rng.integers(1, 3, size=left.sum())
    dig[~left, 0] = rng.integers(1, 3, size=(~left).sum())
    dig[:, 7] = 2
    F = (np.eye(3)[None] + 0.03 * rng.normal(size=(n, 3, 3))).astype(np.float32)
    v = (rng.normal(size=(n, 3)) * 0.1).astype(np.float32)
    print(f"[case] fifteen cuts stencil={stencil} n={n}", flush=True)
    g = tl.Scene(s)
    g.write(v=v, F=F, digits=dig)
    o = oracle.OracleScene(s)
    o.set(v=v, F=F.reshape(n, 9), digits=dig)
    g.step([])
    o.step([])
    assert g.status() == 0
    a, b = g.read(("u", "v", "F", "H", "digits")), o.get()
    assert np.array_equal(a["digits"], dig)
    assert np.array_equal(b["digits"], dig)
    eu, ev, eH = state_errs(a, b, s["X"], s["params"])
    print(f"[fifteen cuts] stencil={stencil} u {eu:.2e} v {ev:.2e} H {eH:.2e}", flush=True)
    assert eu < 1e-5 and ev < 1e-5 and eH < 1e-5, (eu, ev, eH)


@pytest.mark.parametrize("stencil", [0, 1])
def test_slot_overflow_is_a_status_error(tl, stencil):
    """slot_capacity = 1 with two compatible codes meeting at nodes: the scene
    reports TLMPM_E_SLOT_OVERFLOW and keeps running (no fault)."""
    s = W.box_scene(n_cells=(6, 4, 4), seed=23, floor_on=0, max_cuts=1, stencil=stencil, slot_capacity=1)
    n = s["X"].shape[0]
    dig = np.where(s["X"][:, 0] < 0.03, 0, 1).astype(np.uint8)[:, None]
    print(f"[case] slot overflow stencil={stencil}", flush=True)
    g = tl.Scene(s)
    g.write(digits=dig)
    g.step([], n_substeps=2)
    assert g.status() == tl.E_SLOT_OVERFLOW
