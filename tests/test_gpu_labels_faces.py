"""Side labels of particles that sit on a band face at the extreme of their brick
(Eqs. 3, 4, 6), through the C ABI: the label pass skips bricks whose box cannot
meet the band, and the box holds FP32 positions fl(X + u) while the predicate reads
the exact X + u.  Each blade here puts its band's +s face (s = h) 1e-12 m beyond
the exact position of the particle with the smallest x of one brick, whose FP32
position is rounded up by about half an ulp, so that the brick's FP32 box lies
entirely beyond the face; the GPU labels must still equal the oracle's on the same
FP32 state (shared-input mode, bit-exact)."""
import numpy as np
import pytest

import oracle
from paper_2609_27342_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_27342_amd import tlmpm
    tlmpm.lib()
    return tlmpm


def test_band_face_at_brick_extreme_bit_exact(tl):
    s = W.box_scene(n_cells=(24, 8, 8), dx=0.005, seed=51, floor_on=0, gravity=[0.0, 0.0, 0.0], max_cuts=8)
    X = s["X"]
    n = X.shape[0]
    p = s["params"]
    cell = np.floor((X.astype(np.float64) - np.asarray(p["origin"])) / p["dx"]).astype(np.int64)
    brick = cell // 4
    bid = (brick[:, 2] * 100 + brick[:, 1]) * 100 + brick[:, 0]
    u = np.zeros((n, 3), np.float32)
    blades = []
    dt = p["dt"]
    # the particle of smallest x in each brick whose X_min >= 0.0625 (FP32 ulp 7.45e-9)
    targets = []
    for b in np.unique(bid):
        idx = np.nonzero(bid == b)[0]
        i = idx[np.argmin(X[idx, 0])]
        if X[i, 0] >= 0.0625:
            targets.append(i)
    assert len(targets) >= 8
    for k, i in enumerate(targets[:8]):
        ulp = np.spacing(np.float32(X[i, 0]))
        u[i, 0] = -np.float32(0.45) * ulp           # exact X + u is 0.45 ulp below fl(X + u) = X
        assert np.float32(X[i, 0] + u[i, 0]) == X[i, 0]
        x_exact = float(X[i, 0]) + float(u[i, 0])
        h = 6 * p["dx"]
        xe = (x_exact - h + 1e-12, float(X[i, 1]), float(X[i, 2]) - 0.002)  # s = h - 1e-12
        blades.append(W.blade(k, xe, (1, 0, 0), (0, 0, -1), (0, 0, -0.1), 0.05, h, 0.05, p["dx"]))
    g = tl.Scene(s)
    g.write(u=u)
    pre = g.read(("u", "v", "digits"))
    g.assign_labels(blades[:4])  # at most 4 blades per call
    g.assign_labels(blades[4:])
    post = g.read(("digits",))["digits"]
    ref = oracle.labels_on(X, pre["u"], pre["v"], pre["digits"], blades, dt)
    for k, i in enumerate(targets[:8]):
        assert ref[i, k] == 2, (k, i)  # s = h - 1e-12 >= 0: side 2
    assert np.array_equal(post, ref)
