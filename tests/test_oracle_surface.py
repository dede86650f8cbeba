"""Pins of the surface reconstruction reference (oracle/surface.py, Sec. III-F)
against what the geometry fixes: the surface of an uncut box is a closed,
consistently oriented quad mesh on the box's faces that encloses the box's volume;
a full planar cut gives two closed pieces whose cut faces are coincident pairs of
opposite orientation; the embedding moves each side with its own particles."""
import numpy as np

from oracle import surface
from paper_2609_27342_amd import workloads as W


def _box(n_cells=(6, 5, 4), dx=0.01, seed=3, jitter=0.25):
    return W.box_scene(n_cells=n_cells, dx=dx, seed=seed, jitter=jitter, max_cuts=2)


def _closed_oriented(quads):
    """Every mesh edge is used by exactly two quads, once in each direction."""
    for key, uses in surface.mesh_edges(quads).items():
        if len(uses) != 2 or uses[0][1] == uses[1][1]:
            return False
    return True


def _components(quads, nv):
    parent = list(range(nv))

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i
    for q in quads:
        for j in range(1, 4):
            a, b = find(int(q[0])), find(int(q[j]))
            parent[max(a, b)] = min(a, b)
    return len({find(int(v)) for q in quads for v in q})


def test_uncut_box_is_closed_and_exact():
    s = _box()
    n = s["X"].shape[0]
    L = np.array((6, 5, 4)) * 0.01
    sf = surface.build(s["X"], np.zeros((n, 2), np.uint8), s["params"]["origin"], s["params"]["dx"])
    V, Q = sf["vertices"], sf["quads"]
    assert len(Q) > 0 and not sf["cut"].any()
    assert _closed_oriented(Q)
    nE = len(surface.mesh_edges(Q))
    assert len(V) - nE + len(Q) == 2  # a sphere
    # every vertex on the box surface, the enclosed volume the box's
    on_face = np.isclose(V, 0.0, atol=1e-12) | np.isclose(V, L[None], atol=1e-12)
    assert on_face.any(axis=1).all()
    assert np.all((V > -1e-12) & (V < L[None] + 1e-12))
    assert abs(surface.enclosed_volume(V, Q) - L.prod()) < 1e-12
    # face quads: the box's outer sub-cell faces, (2 n)^2 per face pair direction
    assert len(Q) == 2 * (12 * 10 + 12 * 8 + 10 * 8)


def _cut_box(depth_frac=1.0):
    s = _box(n_cells=(6, 4, 4))
    X = s["X"].astype(np.float64)
    n = X.shape[0]
    dig = np.zeros((n, 2), np.uint8)
    # a vertical cut at x = 0.03 (a sub-cell face) from the top down to depth_frac
    sweep = X[:, 2] >= 0.04 * (1.0 - depth_frac)
    dig[sweep, 0] = np.where(X[sweep, 0] < 0.03, 1, 2)
    return s, X, dig


def test_full_cut_gives_two_closed_pieces_with_coincident_faces():
    s, X, dig = _cut_box(1.0)
    sf = surface.build(X, dig, s["params"]["origin"], s["params"]["dx"])
    V, Q, cut = sf["vertices"], sf["quads"], sf["cut"]
    assert _closed_oriented(Q)
    assert _components(Q, len(V)) == 2
    assert cut.sum() == 2 * 8 * 8  # the cut plane, 8 x 8 sub-cell faces, once per side
    # cut quads pair up: same vertex positions, opposite orientation
    cq = [tuple(map(tuple, np.round(V[q], 12))) for q in Q[cut]]
    keyset = {}
    for ring in cq:
        keyset.setdefault(frozenset(ring), []).append(ring)
    assert all(len(v) == 2 for v in keyset.values()) and len(keyset) == 8 * 8
    for a, b in keyset.values():
        i = a.index(b[0])
        assert list(a[i:] + a[:i]) == [b[0]] + list(reversed(b[1:]))
    assert np.allclose(V[np.unique(Q[cut])][:, 0], 0.03, atol=1e-12)
    vol = surface.enclosed_volume(V, Q)
    assert abs(vol - 0.06 * 0.04 * 0.04) < 1e-12


def test_partial_cut_keeps_one_closed_surface():
    s, X, dig = _cut_box(0.5)
    sf = surface.build(X, dig, s["params"]["origin"], s["params"]["dx"])
    V, Q, cut = sf["vertices"], sf["quads"], sf["cut"]
    assert _closed_oriented(Q)
    assert _components(Q, len(V)) == 1
    assert cut.sum() == 2 * 8 * 4  # the upper half of the cut plane, both sides
    nE = len(surface.mesh_edges(Q))
    assert len(V) - nE + len(Q) == 2
    assert abs(surface.enclosed_volume(V, Q) - 0.06 * 0.04 * 0.04) < 1e-12


def test_embedding_follows_each_side():
    s, X, dig = _cut_box(1.0)
    sf = surface.build(X, dig, s["params"]["origin"], s["params"]["dx"])
    n = X.shape[0]
    # a translation of everything moves every vertex by it
    t = np.array([0.001, -0.002, 0.0005])
    assert np.allclose(surface.embed(sf, np.tile(t, (n, 1))) - sf["vertices"], t, atol=1e-15)
    # move only side 2: side-1 vertices (all their particles on side 1) stay
    u = np.zeros((n, 3))
    side2 = dig[:, 0] == 2
    u[side2] = [0.004, 0.0, 0.0]
    x = surface.embed(sf, u)
    for i, cw in enumerate(sf["corners"]):
        sides = {int(dig[p, 0]) for p, _ in cw}
        if sides == {1}:
            assert np.allclose(x[i], sf["vertices"][i], atol=1e-15)
        if sides == {2}:
            assert np.allclose(x[i] - sf["vertices"][i], [0.004, 0, 0], atol=1e-15)
    assert all(abs(sum(w for _, w in cw) - 1.0) < 1e-12 for cw in sf["corners"])
