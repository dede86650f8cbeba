"""FP64 reference of the reference-grid surface reconstruction (Sec. III-F).

TEST INFRASTRUCTURE ONLY: the tests load it; the product library never does.  Plain
Python over dictionaries, written for obviousness; small scenes only.

Reading of the paper's linked-volume surface with local dual contouring (Sec.
III-F), on the 2x2x2 sub-cell lattice of the reference grid (spacing h = dx / 2),
the lattice the particles are sampled on:
  - a site s = floor((X - origin) / h) per axis is material when a particle lies in
    it (several particles: the one of smallest index);
  - a link joins two face-adjacent sites; it is intact when both are material and
    their side codes do not conflict (Sec. III-D: the blade sweep that assigned
    opposite digits disconnected it); a directed link a -> b from a material site a
    is a transition when b is empty or the link is cut;
  - Hermite data of a transition: the link midpoint and the unit link direction
    (from the material site outward);
  - each cube of 8 sites splits its material corners into local material regions,
    the connected components of its intact edges; a region with a transition edge
    gets one surface vertex (a surface representative), so a cube that a cut
    crosses holds a vertex on each side;
  - vertex position (dual contouring with axis-aligned normals): per axis a, the
    mean a-coordinate of the region's transition midpoints along axis a, or of all
    its transition midpoints when it has none along a (this minimises the quadratic
    error of the Hermite planes exactly);
  - one quad per directed transition a -> b, joining the vertices of a's regions in
    the four cubes around the link, ordered counter-clockwise about the outward
    direction; a cut link gives one quad per side (the two coincident faces of the
    cut);
  - one-way embedding (Sec. III-F): a vertex keeps fixed trilinear weights of its
    reference position in its cube, restricted to its region's corners and
    normalised; its displacement is the weighted sum of those corners' particle
    displacements, so it follows the motion of its own side only.
"""
import numpy as np

CORNERS = [(x, y, z) for z in (0, 1) for y in (0, 1) for x in (0, 1)]  # corner k: bits x | y << 1 | z << 2
EDGES = [(a, b) for a in range(8) for b in range(a + 1, 8) if bin(a ^ b).count("1") == 1]  # the cube's 12 edges


def conflict(da, db):
    """Two digit vectors conflict iff some cut has 1 in one and 2 in the other."""
    return any((x == 1 and y == 2) or (x == 2 and y == 1) for x, y in zip(da, db))


def build(X, digits, origin, dx):
    """Surface of particles at reference positions X [n,3] with side digits [n,K].
    Returns dict(vertices [nv,3] reference positions, corners [nv] list of
    (particle, weight) pairs, quads [nq,4] vertex indices, cut [nq] bool (quad on a
    cut face), keys [nv] (cube, lowest corner of the region))."""
    X = np.asarray(X, np.float64)
    digits = np.asarray(digits)
    origin = np.asarray(origin, np.float64)
    h = 0.5 * float(dx)
    site_of = np.floor((X - origin) / h).astype(np.int64)
    sites = {}
    for p in range(X.shape[0]):
        s = tuple(site_of[p])
        if s not in sites:
            sites[s] = p  # the particle of smallest index
    centre = lambda s: origin + (np.asarray(s, np.float64) + 0.5) * h

    def material(s):
        return s in sites

    def intact(a, b):
        return material(a) and material(b) and not conflict(digits[sites[a]], digits[sites[b]])

    def transition(a, b):  # a material
        return not intact(a, b)

    # cubes: min corner m; regions and vertices
    cubes = set()
    for s in sites:
        for c in CORNERS:
            cubes.add((s[0] - c[0], s[1] - c[1], s[2] - c[2]))
    vertex_of = {}  # (cube, corner) -> vertex index
    verts, corners, keys = [], [], []
    for m in sorted(cubes, key=lambda t: (t[2], t[1], t[0])):
        cs = [(m[0] + c[0], m[1] + c[1], m[2] + c[2]) for c in CORNERS]
        mat = [material(s) for s in cs]
        # connected components of the intact edges
        comp = list(range(8))

        def find(i):
            while comp[i] != i:
                i = comp[i]
            return i

        for a, b in EDGES:
            if intact(cs[a], cs[b]):
                ra, rb = find(a), find(b)
                if ra != rb:
                    comp[max(ra, rb)] = min(ra, rb)
        regions = {}
        for k in range(8):
            if mat[k]:
                regions.setdefault(find(k), []).append(k)
        for root in sorted(regions):
            members = regions[root]
            pts = []  # (midpoint, axis) of the region's transition edges in this cube
            for a, b in EDGES:
                for u, w in ((a, b), (b, a)):
                    if u in members and transition(cs[u], cs[w]):
                        axis = [i for i in range(3) if CORNERS[u][i] != CORNERS[w][i]][0]
                        pts.append((0.5 * (centre(cs[u]) + centre(cs[w])), axis))
            if not pts:
                continue
            allm = np.mean([p for p, _ in pts], axis=0)
            pos = np.empty(3)
            for a in range(3):
                along = [p[a] for p, ax in pts if ax == a]
                pos[a] = np.mean(along) if along else allm[a]
            t = (pos - centre(m)) / h
            wts = []
            for k in members:
                c = CORNERS[k]
                wts.append(np.prod([t[i] if c[i] else 1.0 - t[i] for i in range(3)]))
            tot = sum(wts)
            corners.append([(sites[cs[k]], w / tot) for k, w in zip(members, wts)])
            verts.append(pos)
            keys.append((m, min(members)))
            for k in members:
                vertex_of[(m, k)] = len(verts) - 1
    # quads: one per directed transition, counter-clockwise about the outward direction
    quads, cut = [], []
    for a in sorted(sites, key=lambda t: (t[2], t[1], t[0])):
        for d in range(3):
            e1, e2 = (d + 1) % 3, (d + 2) % 3
            for sg in (1, -1):
                b = list(a)
                b[d] += sg
                b = tuple(b)
                if not transition(a, b):
                    continue
                ring = []
                for o1, o2 in ((-1, -1), (0, -1), (0, 0), (-1, 0)):
                    m = [0, 0, 0]
                    m[d] = min(a[d], b[d])
                    m[e1] = a[e1] + o1
                    m[e2] = a[e2] + o2
                    m = tuple(m)
                    k = (a[0] - m[0]) | ((a[1] - m[1]) << 1) | ((a[2] - m[2]) << 2)
                    ring.append(vertex_of[(m, k)])
                quads.append(ring if sg > 0 else ring[::-1])
                cut.append(material(b))
    return dict(vertices=np.array(verts).reshape(-1, 3), corners=corners, quads=np.array(quads, np.int64).reshape(-1, 4),
                cut=np.array(cut, bool), keys=keys)


def embed(surf, u):
    """Current vertex positions: reference position plus the weighted displacement of
    the region's particles (u [n,3])."""
    u = np.asarray(u, np.float64)
    out = np.array(surf["vertices"], np.float64, copy=True)
    for i, cw in enumerate(surf["corners"]):
        for p, w in cw:
            out[i] += w * u[p]
    return out


def mesh_edges(quads):
    """Undirected edge -> list of (quad, direction +1 / -1)."""
    E = {}
    for qi, q in enumerate(quads):
        for j in range(4):
            a, b = int(q[j]), int(q[(j + 1) % 4])
            key = (min(a, b), max(a, b))
            E.setdefault(key, []).append((qi, 1 if a < b else -1))
    return E


def enclosed_volume(verts, quads):
    """Volume enclosed by the quad mesh (divergence theorem, each quad split into two
    triangles)."""
    v = np.asarray(verts, np.float64)
    vol = 0.0
    for q in quads:
        for tri in ((q[0], q[1], q[2]), (q[0], q[2], q[3])):
            a, b, c = v[list(tri)]
            vol += np.dot(a, np.cross(b, c)) / 6.0
    return vol


__all__ = ["build", "embed", "mesh_edges", "enclosed_volume", "conflict"]
