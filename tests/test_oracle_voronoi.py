"""Pins of the oracle's Voronoi grid and Lloyd iteration (Sec. 2.3: the grid
is built on the generation sites and regularised by 5 Lloyd iterations
before the forward mapping).  Closed forms for slab and octant cells, the
nearest-generator definition checked point by point and by Monte Carlo, and
the exact Lloyd sequence of two generators on a line."""
import numpy as np
import pytest
from scipy.spatial import cKDTree


def faces_of(v, c):
    a, b = v["cell_face_off"][c], v["cell_face_off"][c + 1]
    return range(a, b)


def test_two_slabs(oracle):
    v = oracle.voronoi([[0.3, 0.5, 0.5], [0.7, 0.5, 0.5]])
    assert np.allclose(v["volume"], [0.5, 0.5], atol=1e-14)
    assert np.allclose(v["centroid"], [[0.25, 0.5, 0.5], [0.75, 0.5, 0.5]], atol=1e-14)
    shared = [f for f in faces_of(v, 0) if v["face_id"][f] == 1]
    assert len(shared) == 1 and abs(v["face_area"][shared[0]] - 1.0) < 1e-14
    assert sorted(v["face_id"][list(faces_of(v, 0))]) == [-6, -5, -4, -3, -1, 1]


def test_octants(oracle):
    g = np.array([[(i + 0.5) / 2, (j + 0.5) / 2, (k + 0.5) / 2] for k in range(2) for j in range(2) for i in range(2)])
    v = oracle.voronoi(g)
    assert np.allclose(v["volume"], 0.125, atol=1e-14)
    assert np.allclose(v["centroid"], g, atol=1e-14)
    for c in range(8):
        ids = v["face_id"][list(faces_of(v, c))]
        assert len(ids) == 6 and (ids < 0).sum() == 3
        assert np.allclose(v["face_area"][list(faces_of(v, c))], 0.25, atol=1e-14)
    # the iteration leaves centroidal generators where they are
    assert np.allclose(oracle.lloyd(g, 5), g, atol=1e-14)


def test_lloyd_two_on_a_line(oracle):
    # slab cells [0, b] and [b, 1] with b the midpoint: x1 <- b/2, x2 <- (1+b)/2
    x1, x2 = 0.3, 0.4
    seq = []
    for _ in range(5):
        b = 0.5 * (x1 + x2)
        x1, x2 = 0.5 * b, 0.5 * (1.0 + b)
        seq.append((x1, x2))
    got = oracle.lloyd([[0.3, 0.5, 0.5], [0.4, 0.5, 0.5]], 5)
    assert np.allclose(got[:, 0], seq[-1], atol=1e-14)
    assert np.allclose(got[:, 1:], 0.5, atol=1e-14)
    assert np.allclose(oracle.lloyd([[0.3, 0.5, 0.5], [0.4, 0.5, 0.5]], 2)[:, 0], seq[1], atol=1e-14)


@pytest.mark.parametrize("kind", ["uniform", "turbulent"])
def test_partition_and_symmetry(oracle, workloads, kind):
    pos = workloads.make_cloud(kind, 1500, seed=11)[0]
    lo, hi = np.array([0.0, 0.0, 0.0]), np.array([1.0, 1.0, 1.0])
    v = oracle.voronoi(pos, lo, hi)
    assert abs(v["volume"].sum() - 1.0) < 1e-12
    assert (v["volume"] > 0).all()
    # every interior face appears once from each side with the same area
    area = {}
    for c in range(len(pos)):
        for f in faces_of(v, c):
            j = int(v["face_id"][f])
            if j >= 0:
                area[(c, j)] = area.get((c, j), 0.0) + v["face_area"][f]
    for (c, j), a in area.items():
        assert abs(area.get((j, c), 0.0) - a) <= 1e-12 * max(a, 1e-3), (c, j)
    # every face point is equidistant from the two generators of its face and
    # no other generator is closer
    tree = cKDTree(pos)
    for c in range(0, len(pos), 37):
        for f in faces_of(v, c):
            pts = v["face_pts"][v["face_vtx_off"][f]:v["face_vtx_off"][f + 1]]
            dc = np.linalg.norm(pts - pos[c], axis=1)
            dmin, _ = tree.query(pts)
            assert np.all(dc <= dmin + 1e-12)
            j = int(v["face_id"][f])
            if j >= 0:
                assert np.allclose(np.linalg.norm(pts - pos[j], axis=1), dc, atol=1e-12)
            else:
                axis, side = (-1 - j) // 2, (-1 - j) % 2
                assert np.allclose(pts[:, axis], (lo if side == 0 else hi)[axis], atol=1e-14)


def test_monte_carlo_volumes_and_centroids(oracle):
    g = np.random.default_rng(12).random((60, 3))
    lo, hi = np.array([-0.5, 0.0, 0.25]), np.array([1.5, 1.0, 1.0])
    g = lo + g * (hi - lo)
    v = oracle.voronoi(g, lo, hi)
    box = np.prod(hi - lo)
    assert abs(v["volume"].sum() - box) < 1e-12
    x = lo + np.random.default_rng(13).random((400000, 3)) * (hi - lo)
    _, own = cKDTree(g).query(x)
    frac = np.bincount(own, minlength=60) / len(x) * box
    sig = np.sqrt(v["volume"] * (box - v["volume"]) / len(x))
    assert np.all(np.abs(frac - v["volume"]) <= 5 * sig + 1e-12)
    for c in range(60):
        sel = x[own == c]
        err = np.abs(sel.mean(axis=0) - v["centroid"][c])
        assert np.all(err <= 5 * sel.std(axis=0) / np.sqrt(len(sel)) + 1e-12)
