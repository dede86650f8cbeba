"""Pins of the oracle's quadratic B-spline stencil (reading R33: the 27-node
variant of the interpolation of Eq. 1) and of a substep taken with it.

The weights are checked against scipy's cardinal B-spline basis element (a library
routine, independent of the oracle's piecewise formula), linear reproduction and
gradient reproduction, finite differences; the substep against Prop. 1 (momentum
conservation holds for any partition of unity with zero gradient sum), uniform
translation, the patch test and zero exchange across opposite labels.
"""
import numpy as np
import pytest
from scipy.interpolate import BSpline

import oracle
from paper_2609_27342_amd import workloads as W


def _params(**kw):
    p = W.base_params(0.01, (-0.01, -0.01, -0.01), (8, 8, 8), 1e-4, 0.3, stencil=1)
    p.update(kw)
    return p


def _node_xyz(P, node):
    nx, ny = P["cells"][0] + 1, P["cells"][1] + 1
    ijk = np.stack([node % nx, (node // nx) % ny, node // (nx * ny)], axis=1)
    return np.asarray(P["origin"]) + ijk * P["dx"]


_B2 = BSpline.basis_element([-1.5, -0.5, 0.5, 1.5], extrapolate=False)


def _b2(r):
    v = _B2(np.asarray(r, np.float64))
    return np.nan_to_num(v, nan=0.0)


def test_quadratic_partition_of_unity_and_gradient_sum():
    P = _params()
    rng = np.random.default_rng(0)
    for _ in range(200):
        X = rng.uniform(0.0, 0.06, 3)
        node, w, g = oracle.shape(P, X)
        assert len(node) == 27 and len(set(node.tolist())) == 27
        assert abs(w.sum() - 1.0) < 1e-14
        assert np.abs(g.sum(axis=0)).max() < 1e-11
        assert (w >= 0).all()


def test_quadratic_weights_are_the_cardinal_bspline():
    """Each weight is the product over the axes of the cardinal quadratic B-spline
    (scipy's basis element on knots -3/2, -1/2, 1/2, 3/2) of the particle's distance
    to the node, in cells; nodes farther than 3/2 cells on an axis are not in the
    stencil."""
    P = _params()
    dx = P["dx"]
    rng = np.random.default_rng(1)
    for _ in range(100):
        X = rng.uniform(0.0, 0.06, 3)
        node, w, _ = oracle.shape(P, X)
        r = (X[None, :] - _node_xyz(P, node)) / dx
        assert np.all(np.abs(r) < 1.5 + 1e-12)
        ref = np.prod(_b2(r), axis=1)
        assert np.abs(ref - w).max() < 1e-13


def test_quadratic_reproduces_linear_fields():
    """B-splines of degree 2 reproduce linear functions: sum_i N_i x_i = X and
    sum_i x_i (x) grad N_i = I."""
    P = _params()
    rng = np.random.default_rng(2)
    for _ in range(100):
        X = rng.uniform(0.0, 0.06, 3)
        node, w, g = oracle.shape(P, X)
        xn = _node_xyz(P, node)
        assert np.abs(w @ xn - X).max() < 1e-15
        assert np.abs(xn.T @ g - np.eye(3)).max() < 1e-12


def test_quadratic_gradient_finite_difference():
    P = _params()
    rng = np.random.default_rng(3)
    h = 1e-7
    for _ in range(50):
        X = rng.uniform(0.001, 0.059, 3)
        node, w, g = oracle.shape(P, X)
        for a in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[a] += h
            Xm[a] -= h
            n1, w1, _ = oracle.shape(P, Xp)
            n2, w2, _ = oracle.shape(P, Xm)
            if not (np.array_equal(n1, node) and np.array_equal(n2, node)):
                continue
            fd = (w1 - w2) / (2 * h)
            assert np.abs(fd - g[:, a]).max() < 1e-6 / P["dx"]


def test_quadratic_stencil_needs_half_a_cell_of_margin():
    P = _params()
    with pytest.raises(ValueError):
        oracle.shape(P, np.array([-0.0051, 0.02, 0.02]))  # 0.49 cells from the grid edge
    oracle.shape(P, np.array([-0.0049, 0.02, 0.02]))


def _free_box(seed=0, n_cells=(6, 5, 4), **kw):
    kw.setdefault("floor_on", 0)
    kw.setdefault("gravity", [0.0, 0.0, 0.0])
    return W.box_scene(n_cells=n_cells, seed=seed, stencil=1, **kw)


@pytest.mark.parametrize("beta", [0.0, 0.95])
def test_quadratic_momentum_conservation_random_codes(beta):
    """Prop. 1 with the 27-node stencil: momentum kept to rounding, mass exact."""
    s = _free_box(seed=12, flip_beta=beta, max_cuts=3)
    o = oracle.OracleScene(s)
    n = o.n
    rng = np.random.default_rng(13)
    F = np.eye(3)[None] + 0.05 * rng.normal(size=(n, 3, 3))
    v = rng.normal(size=(n, 3)) * 0.1
    dig = rng.integers(0, 3, size=(n, 3)).astype(np.uint8)
    g = o.get()
    o.set(x=g["x"], v=v, F=F.reshape(n, 9), digits=dig)
    m = s["mass"].astype(np.float64)
    P0 = (m[:, None] * v).sum(axis=0)
    scale = (m[:, None] * np.abs(v)).sum()
    for _ in range(3):
        st, _ = o.step([])
        assert st == 0
        P1 = (m[:, None] * o.get()["v"]).sum(axis=0)
        assert np.abs(P1 - P0).max() < 1e-13 * scale
    gd = o.grid_dump()
    assert abs(gd["m"].sum() - m.sum()) < 1e-14 * m.sum()


def test_quadratic_uniform_translation():
    v0 = (0.3, -0.2, 0.1)
    s = _free_box(seed=14, v0=v0)
    o = oracle.OracleScene(s)
    X = o.get()["x"].copy()
    dt = s["params"]["dt"]
    vv = np.array(v0, np.float32).astype(np.float64)
    for j in range(1, 4):
        o.step([])
        g = o.get()
        assert np.abs(g["v"] - vv).max() < 1e-14
        assert np.abs(g["F"] - np.eye(3)).max() < 1e-13
        assert np.abs(g["x"] - (X + j * dt * vv)).max() < 1e-14


def test_quadratic_patch_test_interior_force_vanishes():
    """Unjittered lattice, uniform F, at rest: the B-spline derivative is odd and the
    particles sit symmetrically about every interior node, so particles three cells
    or more from the boundary stay at rest.  dx is a power of two so that the float32
    reference positions are exact (the quadratic weights, unlike the trilinear
    gradients, see their rounding)."""
    s = W.box_scene(n_cells=(10, 10, 10), dx=2.0 ** -7, seed=15, jitter=0.0, floor_on=0, gravity=[0.0, 0.0, 0.0],
                    flip_beta=0.0, stencil=1)
    o = oracle.OracleScene(s)
    n = o.n
    F = np.array([[1.01, 0.002, 0.0], [0.0, 0.99, 0.003], [0.001, 0.0, 1.005]])
    o.set(F=np.broadcast_to(F.reshape(1, 9), (n, 9)).copy())
    o.step([])
    g = o.get()
    X = s["X"].astype(np.float64)
    dx = s["params"]["dx"]
    inner = np.all((X > 3 * dx) & (X < 7 * dx), axis=1)
    assert inner.sum() > 100
    vmax = np.abs(g["v"]).max()
    assert vmax > 1e-6
    assert np.abs(g["v"][inner]).max() < 1e-9 * vmax


def test_quadratic_zero_exchange_across_opposite_labels():
    s = _free_box(seed=16, n_cells=(6, 4, 4), max_cuts=1)
    o = oracle.OracleScene(s)
    X = s["X"].astype(np.float64)
    A = X[:, 0] < 0.03
    dig = np.where(A, 1, 2).astype(np.uint8)[:, None]
    rng = np.random.default_rng(17)
    v = np.zeros((o.n, 3))
    v[A] = rng.normal(size=(A.sum(), 3)) * 0.2
    F = np.tile(np.eye(3).reshape(1, 9), (o.n, 1))
    F[A] += 0.02 * rng.normal(size=(A.sum(), 9))
    o.set(v=v, F=F, digits=dig)
    for _ in range(5):
        o.step([])
    g = o.get()
    assert np.all(g["v"][~A] == 0.0)
    assert np.all(g["x"][~A] == X[~A])
    assert np.abs(g["v"][A]).max() > 0.01


def test_quadratic_differs_from_trilinear():
    """The stencil is in use: the same resting strained box moves differently."""
    def run(st):
        s = W.box_scene(n_cells=(4, 4, 4), seed=19, floor_on=0, gravity=[0.0, 0.0, 0.0], stencil=st)
        o = oracle.OracleScene(s)
        F = np.tile((np.eye(3) * 1.02).reshape(1, 9), (o.n, 1))
        o.set(F=F)
        o.step([])
        return o.get()["v"]
    assert np.abs(run(0) - run(1)).max() > 1e-4
